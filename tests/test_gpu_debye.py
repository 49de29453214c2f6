"""GPU parity for Debye media (Section 2.4, auxiliary differential equation):
the fused and split passes with polarisation currents against the FP64
oracle on the same seeded inputs, element by element (FP64 1e-11, FP32 2e-5
of the largest value), and the special cases that must reproduce other runs
bit for bit."""
import numpy as np
import pytest

from paper_2207_06908_amd import scenarios as S

pytestmark = pytest.mark.gpu

TAU = [2e-10, 3e-9, 4e-8]


@pytest.fixture(scope="module")
def fd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_06908_amd import fdtd
    fdtd.lib()
    return fdtd


def _say(msg):
    print(msg, flush=True)


def _debye_case(nx, ny, nz, npml, seed, nsteps=60, n_mats=None):
    """The random case (CPML, wires along all axes, sources, every probe
    kind) with pole increments on half of its materials."""
    kw = {} if n_mats is None else {"n_mats": n_mats}
    sc = S.random_case(nx, ny, nz, npml, seed=seed, nsteps=nsteps, **kw)
    rng = np.random.default_rng(seed + 100)
    de = rng.uniform(0.5, 30.0, size=(len(sc.materials), len(TAU)))
    de[::2] = 0.0
    sc.debye = (TAU, de)
    return sc


@pytest.mark.parametrize("variant", [2, 1])   # fused, split (the default)
@pytest.mark.parametrize("dims,npml", [((70, 13, 11), 3), ((33, 41, 17), 4), ((64, 8, 8), 0),
                                       ((130, 19, 37), 5)])
def test_debye_fields_elementwise(fd, oracle_mod, dims, npml, variant):
    sc = _debye_case(*dims, npml, seed=dims[0] + dims[2], n_mats=3 if dims[0] > 100 else None)
    _say(f"debye fields {dims} npml={npml} variant={variant}")
    o = oracle_mod.Oracle.from_params(sc.params())
    ids_o = S.apply(sc, o)
    o.step(sc.n_steps)
    for prec, tol in ((64, 1e-11), (32, 2e-5)):
        g = fd.Grid.from_params(sc.params(), precision=prec)
        ids = S.apply(sc, g)
        g.set_kernel(variant)
        g.step(sc.n_steps)
        for c in range(6):
            ref, got = o.get_field(c), g.get_field(c)
            scale = max(float(np.abs(ref).max()), 1e-300)
            assert np.isfinite(got).all()
            err = float(np.abs(got - ref).max()) / scale
            assert err <= tol, (prec, c, err)
        for a, b in zip(ids_o, ids):
            ref, got = o.probe(a), g.probe(b)
            scale = max(float(np.abs(ref).max()), 1e-300)
            assert float(np.abs(got - ref).max()) / scale <= tol * 10, prec


def test_debye_changes_the_fields(fd):
    """The pole terms are not a no-op: with increments the fields differ from
    the same grid without them by far more than rounding."""
    sc = _debye_case(40, 20, 16, 3, seed=7)
    runs = []
    for debye in (True, False):
        s2 = _debye_case(40, 20, 16, 3, seed=7)
        if not debye:
            s2.debye = None
        g = fd.Grid.from_params(s2.params(), precision=32)
        S.apply(s2, g)
        g.step(sc.n_steps)
        runs.append(g.get_field(2))
    scale = float(np.abs(runs[1]).max())
    assert float(np.abs(runs[0] - runs[1]).max()) > 1e-3 * scale


def test_debye_zero_increments_bitwise_split(fd):
    """Poles whose increments are all zero give the bits of the plain split
    pass (classes, coefficients and the update reduce exactly)."""
    outs = []
    for debye in (True, False):
        sc = S.random_case(45, 21, 13, 3, seed=9, nsteps=40)
        if debye:
            sc.debye = (TAU, np.zeros((len(sc.materials), len(TAU))))
        g = fd.Grid.from_params(sc.params(), precision=32)
        ids = S.apply(sc, g)
        g.set_kernel(1)
        g.step(sc.n_steps)
        outs.append(([g.get_field(c) for c in range(6)], [g.probe(i) for i in ids]))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dims,npml", [((50, 19, 15), 3), ((150, 70, 40), 6), ((70, 21, 19), 0)])
def test_debye_variants_bitwise_equal(fd, dims, npml):
    """Every kernel request on a Debye grid gives the bits of the split pass,
    in odd step chunks and with split and fused steps mixed: the fused pass
    over CPML tile lists (the larger grid has tiles in all four slab groups)
    or, without a CPML, over plain 64 x 8 tiles, also when 4-row tiles are
    asked for (it takes 8); the default and a two-step request run the split
    pass."""
    runs = [((1, 0, 0), (3, 20, 18)), ((0, 0, 0), (3, 20, 18)), ((2, 8, 32), (41,)), ((2, 4, 7), (2, 39)),
            ((3, 8, 20), (5, 36)), ((3, 12, 16), (41,)), ("mixed", (10, 11, 20))]
    outs = []
    for kern, chunks in runs:
        sc = _debye_case(*dims, npml, seed=12, nsteps=41, n_mats=3)
        g = fd.Grid.from_params(sc.params(), precision=32)
        ids = S.apply(sc, g)
        for q, c in enumerate(chunks):
            g.set_kernel(*((1 + (q % 2), 0, 0) if kern == "mixed" else kern))
            g.step(c)
        outs.append(([g.get_field(c) for c in range(6)], [g.probe(i) for i in ids]))
    _say(f"debye variants {dims} npml={npml}")
    for r in range(1, len(runs)):
        for a, b in zip(outs[0][0], outs[r][0]):
            assert np.array_equal(a, b), runs[r]
        for a, b in zip(outs[0][1], outs[r][1]):
            assert np.array_equal(a, b), runs[r]


def test_config2_debye_small_probes(fd, oracle_mod):
    """The config-2 scene on a 96 x 96 x 80 grid with the paper's measured
    four-pole Debye soil in both layers, 600 steps: every probe within
    relative L2 1e-5 of the oracle."""
    from tests.parity import assert_probes_close
    sc = S.config2_debye(nx=96, ny=96, nz=80, dx=0.5, npml=10, wire_cells=12, n_steps=600,
                         e_probe_offsets=(5, 10, 20, 30))
    _say("config2 debye small")
    ref = oracle_mod.run_scenario(sc, S.apply)
    got = fd.run_scenario(sc, S.apply, precision=32)
    assert_probes_close(got, ref, 1e-5)
