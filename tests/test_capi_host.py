"""C-ABI checks that need no GPU: the library loads, exports every symbol its
header declares, and rejects bad set-up on the host before any HIP call."""
import math
import os
import re

import numpy as np
import pytest

from paper_2207_06908_amd import fdtd
from paper_2207_06908_amd import scenarios as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b((?:fdtd|sur)_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = fdtd.lib()
    names = _declared("fdtd.h")
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert sorted(n for n, _r, _a in fdtd.SIGNATURES) == names


def test_library_exports_every_surrogate_symbol():
    from paper_2207_06908_amd import sur
    L = sur.lib()
    names = _declared("sur.h")
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert sorted(n for n, _r, _a in sur.SIGNATURES) == names


def test_surrogate_create_validation():
    import ctypes as C
    from paper_2207_06908_amd import sur
    L = sur.lib()

    def create(widths, nets=1, rows=1024):
        h = C.c_void_p()
        arr = (C.c_int * len(widths))(*widths)
        rc = L.sur_create(arr, len(widths), nets, rows, None, C.byref(h))
        return rc, h

    assert create([5, 100, 256])[0] == -1          # hidden width not a multiple of 64
    assert create([33, 64, 64])[0] == -1           # more than 32 inputs
    assert create([5, 64], nets=17)[0] == -1
    assert create([5, 64], rows=1000)[0] == -1     # rows not a multiple of 64
    rc, h = create([5, 512, 512, 512, 512, 256], nets=4, rows=1024)
    assert rc == 0
    assert L.sur_num_params(h) == 922368           # 5 -> 512 x4 -> 256
    assert L.sur_workspace_bytes(h) > 4 * 922368 * 4 * 4
    assert L.sur_train_step(h, 0, None, None, None, 64, 1e-3, 1, None) == -3   # no workspace
    assert L.sur_init_params(h, 7, 1) == -1        # bad net index
    L.sur_destroy(h)


def _grid(**kw):
    base = dict(nx=12, ny=10, nz=9, dx=0.5, max_steps=10)
    base.update(kw)
    return fdtd.Grid(**base)


def _code(fn):
    with pytest.raises(fdtd.FdtdError) as e:
        fn()
    return e.value.code


def test_create_validation():
    assert _code(lambda: _grid(nx=1)) == -1
    assert _code(lambda: _grid(dt=1e-6)) == -4                  # above Courant
    assert _code(lambda: _grid(npml=5)) == -1                   # 2 npml >= ny
    assert _code(lambda: _grid(precision=16)) == -1
    assert _code(lambda: _grid(loss_mode=3)) == -1
    assert _code(lambda: _grid(wire_r0_factor=1.5)) == -1
    g = _grid()
    assert g.dt == pytest.approx(0.99 * 0.5 / (299792458.0 * math.sqrt(3)), rel=1e-15)


def test_largest_grid_accepted_and_the_next_rejected():
    """Every field component must stay below 4 GiB (the kernels use 32-bit
    element offsets): 1024 x 1024 x 1023 FP32 cells are accepted, 1024^3
    (exactly 4 GiB per component) are not; FP64 halves the limit.  Creation
    allocates nothing per cell, so this runs on any host."""
    _grid(nx=1024, ny=1024, nz=1023)
    assert _code(lambda: _grid(nx=1024, ny=1024, nz=1024)) == -1
    _grid(nx=1024, ny=1024, nz=511, precision=64)
    assert _code(lambda: _grid(nx=1024, ny=1024, nz=512, precision=64)) == -1


def test_two_step_batch_tiles_need_the_z_cpml_table_to_fit_lds():
    """The two-step tiles keep the z CPML table (2 npml values per row) in LDS:
    a batch with a thicker CPML rejects them, and keeps its previous tiles."""
    thick = [fdtd.Grid(150, 150, 150, 0.5, npml=70, max_steps=8) for _ in range(2)]
    b = fdtd.Batch(thick, tile=(32, 8, 32))
    assert _code(lambda: b.set_kernel(60, 8, 32, 0)) == -1
    b.set_kernel(32, 8, 16, 0)
    ok = [fdtd.Grid(40, 40, 40, 0.5, npml=8, max_steps=8) for _ in range(2)]
    fdtd.Batch(ok, tile=(60, 8, 32))


def test_setup_validation():
    g = _grid()
    cm = np.zeros(g.shape, np.uint8)
    assert _code(lambda: g.set_materials(cm + 2, [(1, 0, 1)])) == -2         # id outside table
    assert _code(lambda: g.set_materials(cm, [(-1, 0, 1)])) == -1
    assert _code(lambda: g.set_materials(cm, [(float("nan"), 0, 1)])) == -7
    assert _code(lambda: g.add_wire(0, 2, 2, 2, 3, 0.3)) == -1               # radius >= dx/2
    assert _code(lambda: g.add_wire(0, 10, 2, 2, 3, 0.01)) == -2             # leaves the grid
    assert _code(lambda: g.add_wire(3, 1, 1, 1, 1, 0.01)) == -1
    assert _code(lambda: g.add_source(2, 0, 5, 5, np.ones(3))) == -2          # x = 0 wall
    assert _code(lambda: g.add_source(0, 3, 0, 5, np.ones(3))) == -2          # y = 0 wall
    assert _code(lambda: g.add_source(2, 3, 3, 3, np.array([1.0, np.inf]))) == -7
    assert _code(lambda: g.add_probe(2, 2, 0, 3, 3)) == -2                    # loop on a wall
    assert _code(lambda: g.add_probe(1, 0, 3, 3, 3, 20)) == -2                # line leaves
    assert _code(lambda: g.add_probe(0, 0, 3, 3, 3, 2)) == -1
    g.add_probe(0, 2, 3, 3, 3)
    assert g.workspace_bytes() > 0
    assert _code(lambda: g.add_wire(0, 2, 2, 2, 3, 0.01)) == -3               # frozen
    assert fdtd.lib().fdtd_step(g._h, 1) == -3                                # no workspace bound


def test_source_on_wire_edge_rejected_at_freeze():
    g = _grid()
    g.add_wire(2, 5, 5, 2, 4, 0.01)
    g.add_source(2, 5, 5, 3, np.ones(3))
    assert _code(g.workspace_bytes) == -2


def test_explicit_loss_stability_check():
    g = _grid(loss_mode=1, dx=0.5)
    cm = np.zeros(g.shape, np.uint8)
    g.set_materials(cm, [(1.0, 50.0, 1.0)])   # sigma dt / eps >> 2
    assert _code(g.workspace_bytes) == -4
    g2 = _grid(loss_mode=0, dx=0.5)
    g2.set_materials(cm, [(1.0, 50.0, 1.0)])  # semi-implicit stays stable
    assert g2.workspace_bytes() > 0


def test_classes_and_bytes_config1():
    sc = S.config1(n_steps=2)
    g = fdtd.Grid.from_params(sc.params())
    S.apply(sc, g)
    nb = g.workspace_bytes()
    # air, soil, the interface, and the wall patterns: a handful of classes
    assert 3 <= g.num_classes <= 64
    # two field sets of six FP32 components dominate the workspace
    assert nb >= 12 * 4 * sc.cells
    assert g.algorithmic_bytes_per_step() == pytest.approx(sc.cells * 49.0)


def test_classes_config2_small_with_cpml():
    sc = S.config2_small(n_steps=2)
    g = fdtd.Grid.from_params(sc.params())
    S.apply(sc, g)
    g.workspace_bytes()
    assert g.num_classes <= 256
    # CPML state: 4 psi of 4 bytes read and written per slab node and axis
    n, npml = sc.nx, sc.npml
    slab = 2 * npml * (sc.ny * sc.nz + sc.nx * sc.nz + sc.nx * sc.ny)
    assert g.algorithmic_bytes_per_step() == pytest.approx(sc.cells * 49.0 + slab * 32.0)


def test_debye_validation_and_workspace():
    """fdtd_set_debye: tau > 0, increments >= 0 and finite, at most 4
    poles, before the set-up freezes, the semi-implicit loss form only; the currents add 3 n_poles
    arrays to the workspace; a Debye grid cannot join a batch."""
    cm = np.zeros((9, 10, 12), np.uint8)
    cm[:4] = 1
    mats = [(1.0, 0.0, 1.0), (10.0, 0.01, 1.0)]
    d_eps = [[0.0, 0.0], [5.0, 20.0]]
    g = _grid()
    g.set_materials(cm, mats)
    assert _code(lambda: g.set_debye([1e-9, -1e-8], d_eps)) == -1
    assert _code(lambda: g.set_debye([1e-9, 1e-8], [[0.0, 0.0], [5.0, -1.0]])) == -1
    assert _code(lambda: g.set_debye([1e-9, float("nan")], d_eps)) == -7
    assert _code(lambda: g.set_debye([1e-9] * 5, [[0.0] * 5, [1.0] * 5])) == -1
    with pytest.raises(ValueError):
        g.set_debye([1e-9], d_eps)
    plain = _grid()
    plain.set_materials(cm, mats)
    g.set_debye([1e-9, 1e-8], d_eps)
    extra = g.workspace_bytes() - plain.workspace_bytes()
    n = 12 * 10 * 9
    assert 3 * 2 * n * 4 <= extra <= 3 * 2 * n * 4 + 4096
    # the currents' traffic counts only nodes next to a cell with poles: the
    # 4 soil planes (k < 4) and the interface plane k = 4, not the air above
    n_deb = (g.algorithmic_bytes_per_step() - plain.algorithmic_bytes_per_step()) / (3 * 2 * 2 * 4)
    assert 4 * 10 * 12 <= n_deb <= 5 * 10 * 12
    assert _code(lambda: g.set_debye([1e-9], [[0.0], [1.0]])) == -3  # frozen
    lit = _grid(loss_mode=1)
    lit.set_materials(cm, mats)
    assert _code(lambda: lit.set_debye([1e-9, 1e-8], d_eps)) == -1
    b = _grid()
    b.set_materials(cm, mats)
    b.set_debye([1e-9, 1e-8], d_eps)
    assert _code(lambda: fdtd.Batch([b], tile=(32, 8, 32))) == -1


def test_lumped_and_nonideal_source_validation():
    """Lumped values > 0 and finite on an updated edge; a voltage source needs
    a series resistance; both add to the coefficient classes."""
    g = _grid()
    amps = np.ones(10)
    assert _code(lambda: g.add_lumped(2, 2, 5, 5, 4, 50.0)) == -1       # kind
    assert _code(lambda: g.add_lumped(0, 2, 5, 5, 4, -50.0)) == -1
    assert _code(lambda: g.add_lumped(0, 2, 5, 5, 4, float("inf"))) == -7
    assert _code(lambda: g.add_lumped(0, 2, 0, 5, 4, 50.0)) == -2       # Ez on the x = 0 wall
    assert _code(lambda: g.add_source_r(1, 2, 5, 5, 4, amps, 0.0)) == -1
    assert _code(lambda: g.add_source_r(2, 2, 5, 5, 4, amps, 50.0)) == -1
    plain = _grid()
    g.add_lumped(0, 2, 5, 5, 4, 50.0)
    g.add_lumped(1, 0, 3, 3, 3, 1e-9)
    g.add_source_r(1, 1, 6, 4, 4, amps, 75.0)
    g.add_source_r(0, 1, 7, 4, 4, amps, 0.0)   # ideal
    g.workspace_bytes()
    plain.workspace_bytes()
    assert g.num_classes >= plain.num_classes + 3
    w = _grid()
    w.add_wire(2, 5, 5, 2, 4, 0.01)
    w.add_lumped(0, 2, 5, 5, 3, 50.0)            # on the wire's axial edge
    assert _code(lambda: w.workspace_bytes() or w.finalize()) == -2


def test_oblique_wire_junction_validation():
    """fdtd_join_oblique_wires: at least two ends, valid ids and ends (0 or
    1), no end listed twice or joined twice, ends that meet (within 1e-6
    cells), and only before the workspace size is taken."""
    g = _grid(npml=0)
    w0 = g.add_oblique_wire((2, 2, 2), (5, 5, 5), 0.01)
    w1 = g.add_oblique_wire((5, 5, 5), (2, 6, 3), 0.01)
    w2 = g.add_oblique_wire((2, 2, 5), (5, 2, 2), 0.01)
    w3 = g.add_oblique_wire((2, 2, 2), (2, 6, 6), 0.004)
    assert _code(lambda: g.join_oblique_wires([w0], [1])) == -1                 # one end
    assert _code(lambda: g.join_oblique_wires([w0, 4], [1, 0])) == -1           # no wire 4
    assert _code(lambda: g.join_oblique_wires([w0, w1], [1, 2])) == -1          # end not 0 or 1
    assert _code(lambda: g.join_oblique_wires([w0, w2], [1, 0])) == -1          # (5,5,5) vs (2,2,5)
    assert _code(lambda: g.join_oblique_wires([w0, w1, w0], [1, 0, 1])) == -1   # listed twice
    g.join_oblique_wires([w0, w1], [1, 0])
    assert _code(lambda: g.join_oblique_wires([w1, w0], [0, 1])) == -1          # already joined
    g.join_oblique_wires([w3, w0], [0, 0])                                      # both start at (2,2,2)
    g.workspace_bytes()
    assert _code(lambda: g.join_oblique_wires([w2, w1], [1, 1])) == -3


def test_oblique_wire_validation():
    """fdtd_add_oblique_wire: ends one cell clear of the walls (and CPML), at
    least one cell long, 0 < radius < r0, segment indices in [-1, n_seg),
    finite inputs, not with Debye media either way round; the segment count
    is floor(length) before a workspace exists."""
    g = _grid(npml=0)
    amps = np.ones(4)
    assert _code(lambda: g.add_oblique_wire((0.5, 2, 2), (5, 5, 5), 0.01)) == -2     # off the x = 0 wall by < 1
    assert _code(lambda: g.add_oblique_wire((2, 2, 2), (2, 2, 7.5), 0.01)) == -2     # z > nz - 2
    assert _code(lambda: g.add_oblique_wire((2, 2, 2), (2.5, 2.5, 2.5), 0.01)) == -1 # shorter than a cell
    assert _code(lambda: g.add_oblique_wire((2, 2, 2), (6, 5, 5), 0.2)) == -1        # radius >= r0 = 0.104 m
    assert _code(lambda: g.add_oblique_wire((2, 2, 2), (float("nan"), 5, 5), 0.01)) == -7
    assert _code(lambda: g.add_oblique_wire((2, 2, 2), (6, 5, 5), 0.01, src_seg=5, amps=amps)) == -2
    assert _code(lambda: g.add_oblique_wire((2, 2, 2), (6, 5, 5), 0.01, rec_seg=-2)) == -2
    assert _code(lambda: g.add_oblique_wire((2, 2, 2), (6, 5, 5), 0.01, src_seg=0, amps=[1.0, float("inf")])) == -7
    w = g.add_oblique_wire((2, 2, 2), (6, 5, 5), 0.01, src_seg=0, amps=amps, rec_seg=4)  # length 5.83
    assert w == 0
    assert g.oblique_wire_segments(w) == 5
    assert _code(lambda: g.oblique_wire(w)) == -3                                    # no workspace yet
    cm = np.zeros((9, 10, 12), np.uint8)
    g.set_materials(cm, [(1.0, 0.0, 1.0)])
    assert _code(lambda: g.set_debye([1e-6], [[5.0]])) == -1
    d = _grid(npml=0)
    d.set_materials(cm, [(1.0, 0.0, 1.0)])
    d.set_debye([1e-6], [[5.0]])
    assert _code(lambda: d.add_oblique_wire((2, 2, 2), (6, 5, 5), 0.01)) == -1
    g.workspace_bytes()
    assert _code(lambda: g.add_oblique_wire((2, 2, 2), (6, 5, 5), 0.01)) == -3
