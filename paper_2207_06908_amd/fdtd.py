"""Python binding of the HIP FDTD library (argument marshalling only).

Every step of the method runs in the HIP kernels of ``libmi355fdtd.so``;
PyTorch only provides the device workspace and the stream.  If the library
is missing this module raises at import time -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmi355fdtd.so")

FDTD_EX, FDTD_EY, FDTD_EZ, FDTD_HX, FDTD_HY, FDTD_HZ = range(6)
PR_E, PR_VLINE, PR_ILOOP = 0, 1, 2
KERNEL_AUTO, KERNEL_SPLIT, KERNEL_FUSED, KERNEL_TB2 = 0, 1, 2, 3
ERRORS = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "ESTATE", -4: "EUNSTABLE", -5: "ENOMEM",
          -6: "EDEVICE", -7: "ENONFINITE", -8: "ECLASS"}


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("dt", C.c_double), ("npml", C.c_int), ("pml_m", C.c_double),
                ("pml_sigma_factor", C.c_double), ("pml_kappa_max", C.c_double),
                ("pml_alpha_max", C.c_double), ("pml_ma", C.c_double), ("loss_mode", C.c_int),
                ("wire_r0_factor", C.c_double), ("max_steps", C.c_int), ("precision", C.c_int)]


class Material(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("sigma", C.c_double), ("mu_r", C.c_double)]


# (name, restype, argtypes) of every exported symbol declared in include/fdtd.h
_vp = C.c_void_p
SIGNATURES = [
    ("fdtd_default_params", None, [C.POINTER(Params)]),
    ("fdtd_create", C.c_int, [C.POINTER(Params), _vp, C.POINTER(_vp)]),
    ("fdtd_set_materials", C.c_int, [_vp, _vp, C.POINTER(Material), C.c_int]),
    ("fdtd_set_debye", C.c_int, [_vp, C.c_int, _vp, _vp]),
    ("fdtd_add_lumped", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]),
    ("fdtd_add_oblique_wire", C.c_int, [_vp, _vp, _vp, C.c_double, C.c_int, _vp, C.c_int, C.c_int,
                                        C.POINTER(C.c_int)]),
    ("fdtd_oblique_wire_read", C.c_int, [_vp, C.c_int, _vp, _vp, _vp, C.c_int, C.POINTER(C.c_int),
                                         C.POINTER(C.c_int)]),
    ("fdtd_join_oblique_wires", C.c_int, [_vp, C.c_int, _vp, _vp]),
    ("fdtd_add_source_r", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, C.c_int, C.c_double]),
    ("fdtd_add_wire", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]),
    ("fdtd_add_source", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, C.c_int]),
    ("fdtd_add_probe", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                 C.POINTER(C.c_int)]),
    ("fdtd_finalize", C.c_int, [_vp]),
    ("fdtd_workspace_bytes", C.c_size_t, [_vp]),
    ("fdtd_bind_workspace", C.c_int, [_vp, _vp, C.c_size_t]),
    ("fdtd_bind_static", C.c_int, [_vp]),
    ("fdtd_set_kernel", C.c_int, [_vp, C.c_int, C.c_int, C.c_int]),
    ("fdtd_set_graph", C.c_int, [_vp, C.c_int]),
    ("fdtd_step", C.c_int, [_vp, C.c_int]),
    ("fdtd_probe", C.c_int, [_vp, C.c_int, _vp, C.c_int, C.POINTER(C.c_int)]),
    ("fdtd_set_field", C.c_int, [_vp, C.c_int, _vp]),
    ("fdtd_get_field", C.c_int, [_vp, C.c_int, _vp]),
    ("fdtd_dt", C.c_double, [_vp]),
    ("fdtd_steps_done", C.c_longlong, [_vp]),
    ("fdtd_num_classes", C.c_int, [_vp]),
    ("fdtd_algorithmic_bytes_per_step", C.c_double, [_vp]),
    ("fdtd_timing", C.c_int, [_vp, C.c_int]),
    ("fdtd_kernel_time", C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    ("fdtd_last_error", C.c_char_p, [_vp]),
    ("fdtd_destroy", None, [_vp]),
    ("fdtd_batch_pack", C.c_int, [C.POINTER(_vp), C.c_int, _vp, C.POINTER(_vp)]),
    ("fdtd_batch_workspace_bytes", C.c_size_t, [_vp]),
    ("fdtd_batch_bind_workspace", C.c_int, [_vp, _vp, C.c_size_t]),
    ("fdtd_batch_set_kernel", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int]),
    ("fdtd_batch_set_persistent", C.c_int, [_vp, C.c_int]),
    ("fdtd_batch_run", C.c_int, [_vp, C.c_int]),
    ("fdtd_batch_probe", C.c_int, [_vp, C.c_int, C.c_int, _vp, C.c_int, C.POINTER(C.c_int)]),
    ("fdtd_batch_timing", C.c_int, [_vp, C.c_int]),
    ("fdtd_batch_time", C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    ("fdtd_batch_cells", C.c_longlong, [_vp]),
    ("fdtd_batch_algorithmic_bytes_per_step", C.c_double, [_vp]),
    ("fdtd_batch_last_error", C.c_char_p, [_vp]),
    ("fdtd_batch_destroy", None, [_vp]),
]

_lib = None


def lib():
    """Load libmi355fdtd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2207_06908_amd/csrc/build.py` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class FdtdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _stream_handle(device):
    import torch
    if not torch.cuda.is_available():
        return None
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Grid:
    """One FDTD grid on the GPU.  Same call surface as the FP64 reference."""

    def __init__(self, nx, ny, nz, dx, dt=0.0, npml=0, pml_m=3.0, pml_sigma_factor=1.0,
                 pml_kappa_max=1.0, pml_alpha_max=0.0, pml_ma=1.0, loss_mode=0,
                 wire_r0_factor=math.exp(-math.pi / 2), max_steps=1, precision=32,
                 device="cuda:0", stream=None):
        self.shape = (nz, ny, nx)
        self.max_steps = max_steps
        self.device = device
        p = Params(nx, ny, nz, dx, dt, npml, pml_m, pml_sigma_factor, pml_kappa_max, pml_alpha_max,
                   pml_ma, loss_mode, wire_r0_factor, max_steps, precision)
        h = C.c_void_p()
        st = stream if stream is not None else _stream_handle(device)
        rc = lib().fdtd_create(C.byref(p), st, C.byref(h))
        if rc:
            raise FdtdError(rc, "fdtd_create rejected the parameters")
        self._h = h
        self._ws = None

    @classmethod
    def from_params(cls, params: dict, **kw):
        return cls(**params, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.fdtd_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    def _chk(self, rc):
        if rc:
            raise FdtdError(rc, lib().fdtd_last_error(self._h).decode())

    # -- set-up ------------------------------------------------------------
    def set_materials(self, cell_mat, materials):
        cm = np.ascontiguousarray(cell_mat, dtype=np.uint8)
        if cm.shape != self.shape:
            raise ValueError(f"cell_mat shape {cm.shape} != {self.shape}")
        tab = (Material * len(materials))(*[Material(*m) for m in materials])
        self._chk(lib().fdtd_set_materials(self._h, cm.ctypes.data, tab, len(materials)))

    def set_debye(self, tau, d_eps):
        """Debye poles, after set_materials: time constants tau[p] [s] and,
        per material, increments d_eps[m][p]; the materials' eps_r is eps_inf."""
        t = np.ascontiguousarray(tau, dtype=np.float64)
        d = np.ascontiguousarray(d_eps, dtype=np.float64)
        if d.ndim != 2 or d.shape[1] != t.size:
            raise ValueError("d_eps must be [n_materials][n_poles]")
        self._chk(lib().fdtd_set_debye(self._h, t.size, t.ctypes.data, d.ctypes.data))

    def add_lumped(self, kind, axis, i, j, k, value):
        """Lumped resistor (kind 0, ohm) or capacitor (kind 1, F) on an E edge."""
        self._chk(lib().fdtd_add_lumped(self._h, kind, axis, i, j, k, float(value)))

    def add_oblique_wire(self, a, b, radius, src_seg=-1, amps=None, rec_seg=-1) -> int:
        """Oblique thin wire from a to b (cells); src_seg drives that segment's
        current with amps (A), rec_seg records that segment's current."""
        pa = np.ascontiguousarray(a, dtype=np.float64)
        pb = np.ascontiguousarray(b, dtype=np.float64)
        am = np.ascontiguousarray([] if amps is None else amps, dtype=np.float64)
        wid = C.c_int(-1)
        self._chk(lib().fdtd_add_oblique_wire(self._h, pa.ctypes.data, pb.ctypes.data, float(radius), int(src_seg),
                                              am.ctypes.data, am.size, int(rec_seg), C.byref(wid)))
        return wid.value

    def join_oblique_wires(self, ids, ends) -> None:
        """Junction of the listed wire ends (0: the wire's start a, 1: its end
        b), which must meet at one point."""
        iv = np.ascontiguousarray(ids, dtype=np.int32)
        ev = np.ascontiguousarray(ends, dtype=np.int32)
        if iv.size != ev.size:
            raise ValueError("ids and ends differ in length")
        self._chk(lib().fdtd_join_oblique_wires(self._h, int(iv.size), iv.ctypes.data, ev.ctypes.data))

    def oblique_wire_segments(self, wid) -> int:
        ns = C.c_int(0)
        self._chk(lib().fdtd_oblique_wire_read(self._h, wid, None, None, None, 0, C.byref(ns), None))
        return ns.value

    def oblique_wire(self, wid, max_rec=None):
        """(segment currents, end-point charges per unit length, record)."""
        ns, nw = C.c_int(self.oblique_wire_segments(wid)), C.c_int(0)
        cur = np.zeros(ns.value, np.float64)
        q = np.zeros(ns.value + 1, np.float64)
        rec = np.zeros(int(max_rec if max_rec is not None else self.max_steps), np.float64)
        self._chk(lib().fdtd_oblique_wire_read(self._h, wid, cur.ctypes.data, q.ctypes.data, rec.ctypes.data,
                                               rec.size, C.byref(ns), C.byref(nw)))
        return cur, q, rec[:nw.value].copy()

    def add_source_r(self, kind, axis, i, j, k, amps, r):
        """Non-ideal source: current (kind 0) with shunt r, or voltage (kind 1)
        with series r > 0."""
        a = np.ascontiguousarray(amps, dtype=np.float64)
        self._chk(lib().fdtd_add_source_r(self._h, kind, axis, i, j, k, a.ctypes.data, a.size, float(r)))

    def add_wire(self, axis, i, j, k, n, radius):
        self._chk(lib().fdtd_add_wire(self._h, axis, i, j, k, n, radius))

    def add_source(self, axis, i, j, k, amps):
        a = np.ascontiguousarray(amps, dtype=np.float64)
        self._chk(lib().fdtd_add_source(self._h, 0, axis, i, j, k, a.ctypes.data, a.size))

    def add_probe(self, kind, axis, i, j, k, n=1) -> int:
        pid = C.c_int(-1)
        self._chk(lib().fdtd_add_probe(self._h, kind, axis, i, j, k, n, C.byref(pid)))
        return pid.value

    def set_kernel(self, variant=KERNEL_AUTO, tile_y=0, tile_z=0):
        self._chk(lib().fdtd_set_kernel(self._h, variant, tile_y, tile_z))

    def set_graph(self, graph_steps):
        """Replay runs of graph_steps steps from a captured HIP graph (0: off)."""
        self._chk(lib().fdtd_set_graph(self._h, int(graph_steps)))

    # -- device ------------------------------------------------------------
    def finalize(self):
        self._chk(lib().fdtd_finalize(self._h))

    def workspace_bytes(self) -> int:
        self.finalize()
        n = lib().fdtd_workspace_bytes(self._h)
        if n == 0:
            raise FdtdError(-1, lib().fdtd_last_error(self._h).decode())
        return n

    def bind(self):
        if self._ws is not None:
            return
        import torch
        nbytes = self.workspace_bytes()
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._chk(lib().fdtd_bind_workspace(self._h, C.c_void_p(self._ws.data_ptr()), nbytes))

    def bind_static(self):
        """Bind the library's static device array instead of a workspace
        (fdtd_bind_static; no device allocation)."""
        if self._ws is not None:
            raise FdtdError(-3, "workspace already bound")
        self._chk(lib().fdtd_bind_static(self._h))
        self._ws = "static"

    def close(self):
        """Destroy the context now (releases the static array if it holds it)."""
        h = getattr(self, "_h", None)
        if h:
            lib().fdtd_destroy(h)
            self._h = None

    def step(self, n):
        self.bind()
        self._chk(lib().fdtd_step(self._h, int(n)))

    def probe(self, pid) -> np.ndarray:
        self.bind()
        out = np.zeros(self.max_steps, np.float64)
        nw = C.c_int(0)
        self._chk(lib().fdtd_probe(self._h, pid, out.ctypes.data, out.size, C.byref(nw)))
        return out[:nw.value].copy()

    def set_field(self, comp, arr):
        self.bind()
        a = np.ascontiguousarray(arr, dtype=np.float64)
        if a.shape != self.shape:
            raise ValueError("field shape mismatch")
        self._chk(lib().fdtd_set_field(self._h, comp, a.ctypes.data))

    def get_field(self, comp) -> np.ndarray:
        self.bind()
        out = np.zeros(self.shape, np.float64)
        self._chk(lib().fdtd_get_field(self._h, comp, out.ctypes.data))
        return out

    # -- diagnostics -------------------------------------------------------
    def timing(self, enable=True):
        self._chk(lib().fdtd_timing(self._h, int(enable)))

    def kernel_time(self):
        """(total ms, steps) of the update kernels timed since the last call."""
        ms, n = C.c_double(0), C.c_longlong(0)
        self._chk(lib().fdtd_kernel_time(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    @property
    def dt(self) -> float:
        return lib().fdtd_dt(self._h)

    @property
    def steps_done(self) -> int:
        return lib().fdtd_steps_done(self._h)

    @property
    def num_classes(self) -> int:
        return lib().fdtd_num_classes(self._h)

    def algorithmic_bytes_per_step(self) -> float:
        return lib().fdtd_algorithmic_bytes_per_step(self._h)


def run_scenario(sc, apply_fn, precision=32, variant=KERNEL_AUTO, tile_y=0, tile_z=0):
    """Run a scenario to completion on the GPU; returns {probe name: waveform}."""
    g = Grid.from_params(sc.params(), precision=precision)
    ids = apply_fn(sc, g)
    g.set_kernel(variant, tile_y, tile_z)
    g.step(sc.n_steps)
    return {p[0]: g.probe(i) for p, i in zip(sc.probes, ids)}


class Batch:
    """Many independent grids stepped together (one launch per step over all
    their tiles; optional HIP-graph replay).  Build each member with
    :class:`Grid` (set-up only, no stepping), then pack them here."""

    def __init__(self, grids, device="cuda:0", stream=None, tile=(32, 8, 32), graph_steps=0, persistent=None):
        self.grids = list(grids)
        self.device = device
        arr = (C.c_void_p * len(self.grids))(*[g._h for g in self.grids])
        h = C.c_void_p()
        st = stream if stream is not None else _stream_handle(device)
        rc = lib().fdtd_batch_pack(arr, len(self.grids), st, C.byref(h))
        if rc:
            raise FdtdError(rc, "fdtd_batch_pack rejected the grids")
        self._h = h
        self._ws = None
        self.set_kernel(*tile, graph_steps)
        if persistent is not None:
            self.set_persistent(persistent)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.fdtd_batch_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    def _chk(self, rc):
        if rc:
            raise FdtdError(rc, lib().fdtd_batch_last_error(self._h).decode())

    def set_kernel(self, tile_x=32, tile_y=8, tile_z=32, graph_steps=0):
        self._chk(lib().fdtd_batch_set_kernel(self._h, tile_x, tile_y, tile_z, graph_steps))

    def set_persistent(self, on=True):
        self._chk(lib().fdtd_batch_set_persistent(self._h, 1 if on else 0))

    def bind(self):
        if self._ws is not None:
            return
        import torch
        n = lib().fdtd_batch_workspace_bytes(self._h)
        self._ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._chk(lib().fdtd_batch_bind_workspace(self._h, C.c_void_p(self._ws.data_ptr()), n))
        for g in self.grids:   # members read their fields/probes from the batch workspace
            g._ws = self._ws

    def run(self, n):
        self.bind()
        self._chk(lib().fdtd_batch_run(self._h, int(n)))

    def probe(self, g, pid) -> np.ndarray:
        out = np.zeros(self.grids[g].max_steps, np.float64)
        nw = C.c_int(0)
        self._chk(lib().fdtd_batch_probe(self._h, g, pid, out.ctypes.data, out.size, C.byref(nw)))
        return out[:nw.value].copy()

    def timing(self, enable=True):
        self._chk(lib().fdtd_batch_timing(self._h, int(enable)))

    def time(self):
        ms, n = C.c_double(0), C.c_longlong(0)
        self._chk(lib().fdtd_batch_time(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    @property
    def cells(self) -> int:
        return lib().fdtd_batch_cells(self._h)

    def algorithmic_bytes_per_step(self) -> float:
        return lib().fdtd_batch_algorithmic_bytes_per_step(self._h)


def run_batch(scenarios, apply_fn, precision=32, tile=(32, 8, 32), graph_steps=0, persistent=None):
    """Run scenarios (equal step counts) as one batch; returns a list of
    {probe name: waveform} dicts."""
    grids, ids = [], []
    for sc in scenarios:
        g = Grid.from_params(sc.params(), precision=precision)
        ids.append(apply_fn(sc, g))
        grids.append(g)
    b = Batch(grids, tile=tile, graph_steps=graph_steps, persistent=persistent)
    b.run(scenarios[0].n_steps)
    out = [{p[0]: b.probe(gi, i) for p, i in zip(sc.probes, gid)}
           for gi, (sc, gid) in enumerate(zip(scenarios, ids))]
    del b
    return out
