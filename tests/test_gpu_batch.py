"""Batched engine on the GPU: many uneven grids in one launch per step.

* every grid of a batch is bit-identical to the same grid run alone (the
  solo path uses 64-wide tiles, the batch 32-wide ones or two-step passes
  over 60 x 8 tiles);
* replaying a captured HIP graph gives the same bits as eager launches,
  with eager work and synchronisations between replays;
* the full 256-grid sweep (2000 steps) reproduces the stored FP64-oracle
  waveforms of its 16-grid subset to relative L2 1e-5.
"""
import os

import numpy as np
import pytest

from paper_2207_06908_amd import scenarios as S
from tests.parity import assert_probes_close

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def fd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_06908_amd import fdtd
    fdtd.lib()
    return fdtd


def _say(msg):
    print(msg, flush=True)


def _small_sweep(n=6, steps=240):
    grids = S.config3(n_grids=n, seed=11, n_steps=steps)
    return grids


def _solo(fd, sc):
    g = fd.Grid.from_params(sc.params())
    ids = S.apply(sc, g)
    g.step(sc.n_steps)
    return {p[0]: g.probe(i) for p, i in zip(sc.probes, ids)}, [g.get_field(c) for c in range(6)]


def _batch(fd, scs, tile=(32, 8, 32), graph_steps=0, chunks=None, fields=True, persistent=None):
    grids, ids = [], []
    for sc in scs:
        g = fd.Grid.from_params(sc.params())
        ids.append(S.apply(sc, g))
        grids.append(g)
    b = fd.Batch(grids, tile=tile, graph_steps=graph_steps, persistent=persistent)
    for n in (chunks or [scs[0].n_steps]):
        b.run(n)
        import torch
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
    probes = [{p[0]: b.probe(gi, i) for p, i in zip(sc.probes, gid)} for gi, (sc, gid) in enumerate(zip(scs, ids))]
    fields = [[g.get_field(c) for c in range(6)] for g in grids] if fields else None
    del b
    return probes, fields


@pytest.mark.parametrize("tile,persistent", [((32, 8, 32), None), ((32, 16, 16), None), ((64, 8, 64), None),
                                             ((60, 8, 32), True), ((60, 8, 32), False), ((60, 8, 16), True)])
def test_batch_bitwise_equals_solo(fd, tile, persistent):
    """Two-step passes as one persistent work-queue launch and as one launch
    per CPML group give the same bits as the solo runs."""
    scs = _small_sweep()
    _say(f"batch vs solo tile={tile} persistent={persistent}: " + ", ".join(f"{s.nx}x{s.ny}x{s.nz}" for s in scs))
    bp, bf = _batch(fd, scs, tile=tile, persistent=persistent)
    for gi, sc in enumerate(scs):
        sp, sf = _solo(fd, sc)
        for k in sp:
            assert np.array_equal(bp[gi][k], sp[k]), (gi, k)
        for c in range(6):
            assert np.array_equal(bf[gi][c], sf[c]), (gi, c)


@pytest.mark.parametrize("tile,persistent", [((32, 8, 32), None), ((60, 8, 32), True), ((60, 8, 32), False)])
def test_batch_graph_replay_matches_eager(fd, tile, persistent):
    """(60, 8, ...) selects the two-step passes: odd chunks end with one fused
    step, graphs hold whole passes (with the persistent launch, its counter
    reset kernel too)."""
    scs = _small_sweep(n=5, steps=250)
    ep, ef = _batch(fd, scs)
    # 250 = 3 eager + 4 x 60 graph + 7 eager, in pieces with eager work between
    gp, gf = _batch(fd, scs, tile=tile, graph_steps=20, chunks=[3, 60, 60, 1, 60, 59, 7], persistent=persistent)
    for gi in range(len(scs)):
        for k in ep[gi]:
            assert np.array_equal(ep[gi][k], gp[gi][k]), (gi, k)
        for c in range(6):
            assert np.array_equal(ef[gi][c], gf[gi][c]), (gi, c)


def test_persistent_pass_with_every_tile_group(fd):
    """Larger grids in one batch give tiles in all four CPML groups (clear of
    the x and y slabs, x slabs, y slabs, corners), which the persistent
    launch serves with two code paths: bit for bit the solo runs and the
    per-group launches."""
    scs = [S.random_case(150, 70, 40, 6, seed=21, nsteps=25, n_mats=3),
           S.random_case(190, 45, 33, 3, seed=22, nsteps=25, n_mats=3),
           S.random_case(77, 21, 15, 4, seed=23, nsteps=25, n_mats=3)]
    _say("persistent pass, every tile group")
    qp, qf = _batch(fd, scs, tile=(60, 8, 16), persistent=True)
    gp, gf = _batch(fd, scs, tile=(60, 8, 16), persistent=False)
    for gi, sc in enumerate(scs):
        sp, sf = _solo(fd, sc)
        for k in sp:
            assert np.array_equal(qp[gi][k], sp[k]), (gi, k)
            assert np.array_equal(gp[gi][k], sp[k]), (gi, k)
        for c in range(6):
            assert np.array_equal(qf[gi][c], sf[c]), (gi, c)
            assert np.array_equal(gf[gi][c], sf[c]), (gi, c)


@pytest.mark.parametrize("precision,npml", [(32, 0), (64, 4)])
def test_persistent_pass_with_one_code_path(fd, precision, npml):
    """The persistent two-step pass launches one queue per code path and
    skips an empty one: FP32 grids without a CPML have no y-slab tiles (only
    the x-slab path runs), FP64 grids send every tile to the all-axes path.
    Each grid stays bit for bit its solo run."""
    scs = [S.random_case(130, 30, 24, npml, seed=31, nsteps=21, n_mats=3),
           S.random_case(70, 52, 17, npml, seed=32, nsteps=21, n_mats=3)]
    _say(f"persistent pass, one code path: FP{precision}, npml {npml}")

    def grid(sc):
        g = fd.Grid.from_params(sc.params(), precision=precision)
        return g, S.apply(sc, g)

    solo = []
    for sc in scs:
        g, ids = grid(sc)
        g.step(sc.n_steps)
        solo.append(({p[0]: g.probe(i) for p, i in zip(sc.probes, ids)}, [g.get_field(c) for c in range(6)]))
    made = [grid(sc) for sc in scs]
    b = fd.Batch([g for g, _ in made], tile=(60, 8, 16), persistent=True)
    b.run(scs[0].n_steps)
    for gi, (sc, (g, ids)) in enumerate(zip(scs, made)):
        sp, sf = solo[gi]
        for p, i in zip(sc.probes, ids):
            assert np.array_equal(b.probe(gi, i), sp[p[0]]), (gi, p[0])
        for c in range(6):
            assert np.array_equal(g.get_field(c), sf[c]), (gi, c)
    del b


@pytest.mark.parametrize("tile", [(32, 8, 16), (60, 8, 32)])
def test_full_sweep_against_stored_oracle_subset(fd, tile):
    path = os.path.join(GOLD, "config3_subset.npz")
    if not os.path.exists(path):
        pytest.skip("golden subset not generated")
    from tests.golden.make_golden import CONFIG3_SUBSET
    gold = np.load(path)
    scs = S.config3()
    _say(f"full sweep: {len(scs)} grids, {sum(s.cells for s in scs)} cells, {scs[0].n_steps} steps")
    probes, _fields = _batch(fd, scs, tile=tile, graph_steps=100, fields=False)
    for gi in CONFIG3_SUBSET:
        sc = scs[gi]
        ref = {p[0]: gold[f"{sc.name}/{p[0]}"] for p in sc.probes}
        assert_probes_close(probes[gi], ref, 1e-5)
