"""FP32-storage run of the Yee recurrence in NumPy, for tolerance evidence.

Test infrastructure only.  It steps a PEC-box grid (no CPML, no wires) with
every field stored in float32 and every operation rounded to float32, in
the same rearranged form the GPU kernels use (H + db (dE+ - dE-) with one
rounding; E + ((ca - 1) E + cb curl) with the inner product-sum rounded
once), from coefficients the FP64 oracle built.  Comparing it with the FP64
oracle gives the error that FP32 storage alone leaves on a workload: a floor
that no FP32 implementation of the recurrence can be expected to beat.
Products of two float32 values are exact in float64, so a fused
multiply-add is emulated by one float64 evaluation rounded to float32.
"""
import numpy as np

F32 = np.float32


def _fma(a, b, c):
    if a.dtype == np.float64:
        return a * b + c
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def _up(a, ax):
    """a[index + 1 along axis ax] (arrays are (z, y, x)), zero past the end."""
    out = np.zeros_like(a)
    d = 2 - ax
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    src[d], dst[d] = slice(1, None), slice(None, -1)
    out[tuple(dst)] = a[tuple(src)]
    return out


def _down(a, ax):
    """a[index - 1 along axis ax], zero before the start."""
    out = np.zeros_like(a)
    d = 2 - ax
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    src[d], dst[d] = slice(None, -1), slice(1, None)
    out[tuple(dst)] = a[tuple(src)]
    return out


def run_fp32(sc, oracle_mod, dtype=F32):
    """Probe waveforms of scenario `sc` (PEC box, E probes, current sources)
    from a run that stores and rounds in `dtype` (float32 by default;
    float64 reproduces the oracle, which checks this recurrence itself);
    coefficients from the oracle."""
    assert sc.npml == 0 and not sc.wires and not sc.owires and sc.debye is None
    o = oracle_mod.Oracle.from_params(sc.params())
    S_apply_materials(sc, o)
    dx = sc.dx
    Ca = [o.get_coef(c, 0) for c in range(3)]
    Cb = [o.get_coef(c, 1) for c in range(3)]
    Db = [o.get_coef(3 + c, 0) for c in range(3)]
    cam1 = [(Ca[c] - 1.0).astype(dtype) for c in range(3)]
    cbd = [(Cb[c] / dx).astype(dtype) for c in range(3)]
    dbd = [(Db[c] / dx).astype(dtype) for c in range(3)]
    E = [np.zeros(o.shape, dtype) for _ in range(3)]
    H = [np.zeros(o.shape, dtype) for _ in range(3)]
    src = [(ax, i, j, k, (Cb[ax][k, j, i] * np.asarray(amps) / (dx * dx)).astype(dtype))
           for (ax, i, j, k, amps) in sc.sources]
    out = {p[0]: np.zeros(sc.n_steps) for p in sc.probes}
    for n in range(sc.n_steps):
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            H[a] = _fma(dbd[a], (_up(E[b], c) - E[b]) - (_up(E[c], b) - E[c]), H[a])
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            curl = (H[c] - _down(H[c], b)) - (H[b] - _down(H[b], c))
            E[a] = E[a] + _fma(cam1[a], E[a], cbd[a] * curl)
        for (ax, i, j, k, s) in src:
            if n < s.size:
                E[ax][k, j, i] = E[ax][k, j, i] - s[n]
        for (name, kind, ax, i, j, k, _n) in sc.probes:
            assert kind == 0
            out[name][n] = E[ax][k, j, i]
    return out


def S_apply_materials(sc, o):
    o.set_materials(sc.cell_mat, sc.materials)
    o.step(0)
