"""The allocation-free binding fdtd_bind_static, through the C ABI: a grid
bound to the library's static device array gives the same bits as the same
grid bound to a caller-owned workspace, on two calls in a row (the second
grid smaller than the first, so it lands on the first one's leftovers), and
a grid larger than the array is refused on the host."""
import ctypes as C
import gc

import numpy as np
import pytest

from paper_2207_06908_amd import fdtd
from paper_2207_06908_amd import scenarios as S


def test_static_binding_rejects_an_oversized_grid():
    """168^3 cells need more than the 64 MiB array: FDTD_ENOMEM, decided on
    the host before any HIP call."""
    g = fdtd.Grid(168, 168, 168, 0.5, max_steps=4)
    g.set_materials(np.zeros((168, 168, 168), np.uint8), [(1.0, 0.0, 1.0)])
    assert g.workspace_bytes() > (64 << 20)
    rc = fdtd.lib().fdtd_bind_static(g._h)
    assert rc == -5
    assert b"static array" in fdtd.lib().fdtd_last_error(g._h)


def _run(sc, static, variant=0):
    g = fdtd.Grid.from_params(sc.params(), precision=32)
    ids = S.apply(sc, g)
    g.set_kernel(variant)
    if static:
        g.bind_static()
    g.step(sc.n_steps)
    out = [g.probe(i) for i in ids] + [g.get_field(c) for c in range(6)]
    g.close()
    return out


@pytest.mark.gpu
def test_static_binding_matches_a_caller_workspace():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cases = [S.config1(n_steps=120), S.random_case(30, 26, 22, 3, seed=5, nsteps=70)]
    for n, sc in enumerate(cases):
        print(f"no-alloc call {n}: {sc.name} {sc.nx}x{sc.ny}x{sc.nz}", flush=True)
        ref = _run(sc, static=False)
        got = _run(sc, static=True)
        assert np.abs(ref[0]).max() > 0
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        gc.collect()


@pytest.mark.gpu
def test_static_binding_is_held_by_one_context_at_a_time():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sc = S.random_case(20, 18, 16, 2, seed=8, nsteps=10)
    a = fdtd.Grid.from_params(sc.params(), precision=32)
    S.apply(sc, a)
    a.bind_static()
    b = fdtd.Grid.from_params(sc.params(), precision=32)
    S.apply(sc, b)
    with pytest.raises(fdtd.FdtdError):
        b.bind_static()
    a.close()
    b.bind_static()          # released by the destruction of the first
    b.step(sc.n_steps)
    b.close()
