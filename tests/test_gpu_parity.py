"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.  FP32 waveforms must agree to relative L2 1e-5
per probe (config 1: or 4 times the FP32-storage floor of a probe where
that floor is above 1e-5); the FP64 instantiation of the same kernels to
1e-11.
Stored expected waveforms under tests/golden/ were written by
tests/golden/make_golden.py, which calls only the oracle."""
import os

import numpy as np
import pytest

from paper_2207_06908_amd import scenarios as S
from tests.parity import assert_probes_close, probe_errors

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
VARIANTS = [1, 2, 3]  # split, fused, two-step blocked


@pytest.fixture(scope="module")
def fd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_06908_amd import fdtd
    fdtd.lib()
    return fdtd


def _say(msg):
    print(msg, flush=True)


def _golden(name, sc_list):
    path = os.path.join(GOLD, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    d = np.load(path)
    return [{p[0]: d[f"{sc.name}/{p[0]}"] for p in sc.probes} for sc in sc_list]


@pytest.fixture(scope="module")
def config1_ref(oracle_mod):
    """Oracle probes of the 48^3 workload and the FP32-storage floor of each
    probe (the error an FP32-storage run of the same recurrence leaves)."""
    from tests.fp32_emulation import run_fp32
    from tests.parity import probe_errors
    sc = S.config1()
    ref = oracle_mod.run_scenario(sc, S.apply)
    floor = probe_errors(run_fp32(sc, oracle_mod), ref)
    return sc, ref, floor


@pytest.mark.parametrize("variant", VARIANTS)
def test_config1_fp64_and_fp32(fd, config1_ref, variant):
    """The 48^3 workload is specified in FP64: the FP64 build of the kernels
    must match the oracle to 1e-11 per probe.  The FP32 build is held to the
    waveform rule (relative L2 per probe, near-zero probes against the
    largest norm) at 1e-5, except where FP32 storage alone cannot reach it:
    this workload's Gaussian current leaves a permanent charge dipole in
    air, rounding near the source leaves spurious static charge, and an
    FP32-storage run of the same recurrence already misses 1e-5 on several
    far probes in air (tests/test_fp32_floor.py).  Such a probe is held to
    4 times that floor."""
    sc, ref, floor = config1_ref
    _say(f"config1 variant={variant}")
    got64 = fd.run_scenario(sc, S.apply, precision=64, variant=variant)
    e64 = assert_probes_close(got64, ref, 1e-11)
    got32 = fd.run_scenario(sc, S.apply, precision=32, variant=variant)
    e32 = probe_errors(got32, ref)
    _say(f"fp64 {e64}")
    for k in ref:
        _say(f"fp32 {k}: error {e32[k]:.3e}, FP32-storage floor {floor[k]:.3e}")
    for k in ref:
        assert e32[k] <= max(1e-5, 4.0 * floor[k]), (k, e32[k], floor[k])


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dims,npml", [((70, 13, 11), 3), ((130, 9, 17), 4), ((5, 66, 7), 2), ((64, 8, 8), 0)])
def test_fields_elementwise(fd, oracle_mod, variant, dims, npml):
    """All six components after 60 steps, element by element, on grids that
    span several tiles with ragged tails (x not a multiple of 64, y not a
    multiple of 4), with CPML, wires along all three axes and sources."""
    nx, ny, nz = dims
    sc = S.random_case(nx, ny, nz, npml, seed=nx + ny)
    _say(f"fields {dims} npml={npml} variant={variant}")
    o = oracle_mod.Oracle.from_params(sc.params())
    S.apply(sc, o)
    o.step(sc.n_steps)
    for prec, tol in ((64, 1e-11), (32, 2e-5)):
        g = fd.Grid.from_params(sc.params(), precision=prec)
        S.apply(sc, g)
        g.set_kernel(variant)
        g.step(sc.n_steps)
        for c in range(6):
            ref, got = o.get_field(c), g.get_field(c)
            scale = max(float(np.abs(ref).max()), 1e-300)
            err = float(np.abs(got - ref).max()) / scale
            assert err <= tol, (prec, c, err)


@pytest.mark.parametrize("variant", VARIANTS)
def test_config2_small_against_stored_oracle(fd, variant):
    sc = S.config2_small()
    ref = _golden("config2_small", [sc])[0]
    _say(f"config2_small variant={variant}")
    got = fd.run_scenario(sc, S.apply, precision=32, variant=variant)
    assert_probes_close(got, ref, 1e-5)


@pytest.mark.parametrize("variant,ty,tz", [(0, 0, 0), (2, 8, 32)])
def test_config2_full_against_stored_oracle(fd, variant, ty, tz):
    """Full 512 x 512 x 384, 4000 steps: the default launch, which is the
    two-step pass with its default tile shape (60 x 8 tiles, 20-plane chunks;
    the other two-step shapes give the same bits, see
    test_variants_bitwise_equal), and the fused pass."""
    sc = S.config2()
    ref = _golden("config2_full", [sc])[0]
    _say(f"config2 full variant={variant} ty={ty} tz={tz}")
    got = fd.run_scenario(sc, S.apply, precision=32, variant=variant, tile_y=ty, tile_z=tz)
    assert_probes_close(got, ref, 1e-5)


def test_config3_subset_against_stored_oracle(fd):
    grids = S.config3()
    from tests.golden.make_golden import CONFIG3_SUBSET
    sub = [grids[g] for g in CONFIG3_SUBSET]
    refs = _golden("config3_subset", sub)
    for sc, ref in zip(sub, refs):
        _say(f"config3 {sc.name} {sc.nx}x{sc.ny}x{sc.nz}")
        got = fd.run_scenario(sc, S.apply, precision=32)
        assert_probes_close(got, ref, 1e-5)


@pytest.mark.parametrize("dims,npml", [((77, 21, 15), 4), ((130, 19, 70), 6), ((61, 9, 9), 0),
                                       ((150, 70, 40), 6), ((190, 45, 33), 3)])
def test_variants_bitwise_equal(fd, dims, npml):
    """All kernel variants and tile shapes give the same bits, also when the
    steps come in odd chunks (the two-step pass then ends with one fused
    step).  The larger grids have tiles in every CPML group of the tile
    lists (clear of the x and y slabs, x only, y only, corners)."""
    sc = S.random_case(*dims, npml, seed=3, nsteps=41, n_mats=3)
    runs = [(1, 0, 0, [41]), (2, 8, 32, [41]), (2, 4, 7, [41]), (3, 8, 64, [41]), (3, 4, 5, [3, 10, 1, 27]),
            (3, 8, 16, [2, 39]), (3, 12, 64, [41]), (3, 12, 8, [5, 36])]
    outs = []
    for variant, ty, kz, chunks in runs:
        g = fd.Grid.from_params(sc.params(), precision=32)
        ids = S.apply(sc, g)
        g.set_kernel(variant, ty, kz)
        for c in chunks:
            g.step(c)
        outs.append(([g.get_field(c) for c in range(6)], [g.probe(i) for i in ids]))
    for r in range(1, len(runs)):
        for a, b in zip(outs[0][0], outs[r][0]):
            assert np.array_equal(a, b), runs[r]
        for a, b in zip(outs[0][1], outs[r][1]):
            assert np.array_equal(a, b), runs[r]


def test_sources_on_tile_seams(fd, oracle_mod):
    """Sources on the seams of every tile shape (the tile kernels test for
    sources once per column), two sources in one column at heights in
    different z chunks, and two on one node (same and different component):
    each variant and tile shape against the oracle element by element, and
    all of them bit for bit against the split variant."""
    nx, ny, nz, npml, nsteps = 150, 40, 35, 6, 30
    sc = S.random_case(nx, ny, nz, npml, seed=11, nsteps=nsteps, n_mats=3)
    amps = S.gaussian(nsteps, sc.dt, 10 * sc.dt, 4 * sc.dt, 2.0)
    spots = [(2, 7, 8, 9), (0, 8, 15, 16), (1, 67, 16, 17), (2, 68, 23, 8), (2, 69, 24, 24), (0, 127, 7, 12),
             (1, 128, 31, 20), (2, 63, 12, 16), (2, 64, 13, 31), (0, 65, 32, 7),
             (2, 40, 20, 5), (2, 40, 20, 30),            # one column, two z chunks
             (0, 90, 17, 17), (2, 90, 17, 17),           # one node, two components
             (1, 100, 25, 10), (1, 100, 25, 10)]         # one node, one component twice
    sc.sources = [(c, i, j, k, amps * (1.0 + 0.1 * q)) for q, (c, i, j, k) in enumerate(spots)]
    _say("sources on tile seams")
    o = oracle_mod.Oracle.from_params(sc.params())
    S.apply(sc, o)
    o.step(nsteps)
    ref = [o.get_field(c) for c in range(6)]
    runs = [(1, 0, 0), (2, 8, 32), (2, 4, 8), (3, 8, 64), (3, 8, 8), (3, 12, 16), (3, 4, 5)]
    base = None
    for variant, ty, kz in runs:
        g = fd.Grid.from_params(sc.params(), precision=32)
        S.apply(sc, g)
        g.set_kernel(variant, ty, kz)
        g.step(nsteps)
        got = [g.get_field(c) for c in range(6)]
        for c in range(6):
            err = float(np.abs(got[c] - ref[c]).max()) / max(float(np.abs(ref[c]).max()), 1e-300)
            assert err <= 2e-5, (variant, ty, kz, c, err)
        if base is None:
            base = got
        else:
            for c in range(6):
                assert np.array_equal(base[c], got[c]), (variant, ty, kz, c)


def test_thick_cpml_two_step_request_takes_the_fused_pass(fd):
    """With 2 npml above what the two-step tiles hold in LDS, a two-step (or
    default) request runs the fused pass: same bits as the split pass."""
    sc = S.random_case(150, 150, 146, 70, seed=5, nsteps=9, n_mats=2)
    outs = []
    for variant in (1, 3, 0):
        g = fd.Grid.from_params(sc.params(), precision=32)
        S.apply(sc, g)
        g.set_kernel(variant)
        g.step(9)
        outs.append([g.get_field(c) for c in range(6)])
    for r in (1, 2):
        for c in range(6):
            assert np.array_equal(outs[0][c], outs[r][c]), (r, c)


def test_edge_cases(fd):
    # smallest grid: every E edge lies on a wall, so everything stays zero
    g = fd.Grid(2, 2, 2, 0.5, max_steps=5)
    pid = g.add_probe(2, 2, 1, 1, 0)
    g.step(5)
    assert np.all(g.probe(pid) == 0) and all(np.all(g.get_field(c) == 0) for c in range(6))
    # no source: zero fields stay exactly zero, with CPML and wires
    g = fd.Grid(40, 33, 29, 0.5, npml=6, max_steps=20)
    g.add_wire(2, 20, 16, 8, 10, 0.01)
    pid = g.add_probe(1, 0, 7, 16, 14, 20)
    g.step(20)
    assert np.all(g.probe(pid) == 0)
    # set_field zeroes perfect-conductor edges and round-trips the rest
    g = fd.Grid(9, 8, 7, 0.5, max_steps=2, precision=64)
    g.add_wire(2, 4, 4, 1, 4, 0.01)
    v = np.random.default_rng(0).standard_normal((7, 8, 9))
    g.set_field(2, v)
    back = g.get_field(2)
    assert np.all(back[1:5, 4, 4] == 0)          # wire edges
    assert np.all(back[:, 0, :] == 0) and np.all(back[:, :, 0] == 0)  # walls
    assert back[3, 2, 2] == v[3, 2, 2]
    # stepping beyond max_steps is refused before any launch
    with pytest.raises(fd.FdtdError):
        g.step(3)
