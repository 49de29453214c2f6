"""ctypes binding of the FP64 FDTD oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this module.  It never touches a GPU.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")

ORC_EX, ORC_EY, ORC_EZ, ORC_HX, ORC_HY, ORC_HZ = range(6)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-Wall", "-o", LIB + ".tmp", os.path.join(HERE, "orc.cpp")]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("dt", C.c_double), ("npml", C.c_int), ("pml_m", C.c_double),
                ("pml_sigma_factor", C.c_double), ("pml_kappa_max", C.c_double),
                ("pml_alpha_max", C.c_double), ("pml_ma", C.c_double), ("loss_mode", C.c_int),
                ("wire_r0_factor", C.c_double), ("max_steps", C.c_int)]


class _Mat(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("sigma", C.c_double), ("mu_r", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Params), C.POINTER(vp)]
        L.orc_destroy.argtypes = [vp]
        L.orc_destroy.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_materials.argtypes = [vp, C.c_void_p, C.POINTER(_Mat), C.c_int]
        L.orc_set_debye.argtypes = [vp, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_add_wire.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_add_source.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int]
        L.orc_add_lumped.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_add_source_r.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int,
                                       C.c_double]
        L.orc_add_probe.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                    C.POINTER(C.c_int)]
        L.orc_add_oblique_wire.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_void_p, C.c_int,
                                           C.c_int, C.POINTER(C.c_int)]
        L.orc_oblique_wire_read.argtypes = [vp, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                            C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_join_oblique_wires.argtypes = [vp, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_step.argtypes = [vp, C.c_int]
        L.orc_probe.argtypes = [vp, C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_int)]
        L.orc_set_field.argtypes = [vp, C.c_int, C.c_void_p]
        L.orc_get_field.argtypes = [vp, C.c_int, C.c_void_p]
        L.orc_get_coef.argtypes = [vp, C.c_int, C.c_int, C.c_void_p]
        L.orc_dt.argtypes = [vp]
        L.orc_dt.restype = C.c_double
        L.orc_last_error.argtypes = [vp]
        L.orc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


class Oracle:
    """FP64 reference simulation with the same call surface as the GPU binding."""

    def __init__(self, nx, ny, nz, dx, dt=0.0, npml=0, pml_m=3.0, pml_sigma_factor=1.0,
                 pml_kappa_max=1.0, pml_alpha_max=0.0, pml_ma=1.0, loss_mode=0,
                 wire_r0_factor=0.20787957635076193, max_steps=1):
        self.shape = (nz, ny, nx)
        p = _Params(nx, ny, nz, dx, dt, npml, pml_m, pml_sigma_factor, pml_kappa_max,
                    pml_alpha_max, pml_ma, loss_mode, wire_r0_factor, max_steps)
        h = C.c_void_p()
        rc = lib().orc_create(C.byref(p), C.byref(h))
        if rc:
            raise OracleError(rc, "create")
        self._h = h
        self.max_steps = max_steps

    @classmethod
    def from_params(cls, params: dict):
        return cls(**params)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def _chk(self, rc):
        if rc:
            raise OracleError(rc, lib().orc_last_error(self._h).decode())

    @property
    def dt(self) -> float:
        return lib().orc_dt(self._h)

    def set_materials(self, cell_mat, materials):
        cm = np.ascontiguousarray(cell_mat, dtype=np.uint8)
        assert cm.shape == self.shape
        tab = (_Mat * len(materials))(*[_Mat(*m) for m in materials])
        self._chk(lib().orc_set_materials(self._h, cm.ctypes.data, tab, len(materials)))

    def set_debye(self, tau, d_eps):
        """Debye poles, after set_materials: time constants tau[p] [s] and,
        per material, increments d_eps[m][p]; the materials' eps_r is eps_inf
        (Section 2.4, ADE)."""
        t = np.ascontiguousarray(tau, dtype=np.float64)
        d = np.ascontiguousarray(d_eps, dtype=np.float64)
        assert d.ndim == 2 and d.shape[1] == t.size
        self._chk(lib().orc_set_debye(self._h, t.size, t.ctypes.data, d.ctypes.data))

    def add_wire(self, axis, i, j, k, n, radius):
        self._chk(lib().orc_add_wire(self._h, axis, i, j, k, n, radius))

    def add_source(self, axis, i, j, k, amps):
        a = np.ascontiguousarray(amps, dtype=np.float64)
        self._chk(lib().orc_add_source(self._h, axis, i, j, k, a.ctypes.data, a.size))

    def add_lumped(self, kind, axis, i, j, k, value):
        """Lumped resistor (kind 0, ohm) or capacitor (kind 1, F) on an E edge."""
        self._chk(lib().orc_add_lumped(self._h, kind, axis, i, j, k, float(value)))

    def add_source_r(self, kind, axis, i, j, k, amps, r):
        """Non-ideal source: current (kind 0) with shunt r, or voltage (kind 1)
        with series r > 0."""
        a = np.ascontiguousarray(amps, dtype=np.float64)
        self._chk(lib().orc_add_source_r(self._h, kind, axis, i, j, k, a.ctypes.data, a.size, float(r)))

    def add_probe(self, kind, axis, i, j, k, n=1) -> int:
        pid = C.c_int(-1)
        self._chk(lib().orc_add_probe(self._h, kind, axis, i, j, k, n, C.byref(pid)))
        return pid.value

    def add_oblique_wire(self, a, b, radius, src_seg=-1, amps=None, rec_seg=-1) -> int:
        """Oblique thin wire from a to b (cell units); src_seg drives that
        segment's current with amps, rec_seg records that segment's current."""
        pa = np.ascontiguousarray(a, dtype=np.float64)
        pb = np.ascontiguousarray(b, dtype=np.float64)
        am = np.ascontiguousarray([] if amps is None else amps, dtype=np.float64)
        wid = C.c_int(-1)
        self._chk(lib().orc_add_oblique_wire(self._h, pa.ctypes.data, pb.ctypes.data, float(radius), int(src_seg),
                                             am.ctypes.data, am.size, int(rec_seg), C.byref(wid)))
        return wid.value

    def join_oblique_wires(self, ids, ends) -> None:
        """Junction of the listed wire ends (0: the wire's start a, 1: its end
        b), which must meet at one point."""
        iv = np.ascontiguousarray(ids, dtype=np.int32)
        ev = np.ascontiguousarray(ends, dtype=np.int32)
        if iv.size != ev.size:
            raise ValueError("ids and ends differ in length")
        self._chk(lib().orc_join_oblique_wires(self._h, int(iv.size), iv.ctypes.data, ev.ctypes.data))

    def oblique_wire(self, wid):
        """(segment currents, end-point charges per unit length, record)."""
        ns = C.c_int(0)
        self._chk(lib().orc_oblique_wire_read(self._h, wid, None, None, None, 0, C.byref(ns), None))
        cur = np.zeros(ns.value, np.float64)
        q = np.zeros(ns.value + 1, np.float64)
        rec = np.zeros(self.max_steps, np.float64)
        nw = C.c_int(0)
        self._chk(lib().orc_oblique_wire_read(self._h, wid, cur.ctypes.data, q.ctypes.data, rec.ctypes.data,
                                              rec.size, C.byref(ns), C.byref(nw)))
        return cur, q, rec[:nw.value].copy()

    def step(self, n):
        self._chk(lib().orc_step(self._h, int(n)))

    def probe(self, pid) -> np.ndarray:
        out = np.zeros(self.max_steps, np.float64)
        nw = C.c_int(0)
        self._chk(lib().orc_probe(self._h, pid, out.ctypes.data, out.size, C.byref(nw)))
        return out[:nw.value].copy()

    def set_field(self, comp, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        assert a.shape == self.shape
        self._chk(lib().orc_set_field(self._h, comp, a.ctypes.data))

    def get_field(self, comp) -> np.ndarray:
        out = np.zeros(self.shape, np.float64)
        self._chk(lib().orc_get_field(self._h, comp, out.ctypes.data))
        return out

    def get_coef(self, comp, which=0) -> np.ndarray:
        out = np.zeros(self.shape, np.float64)
        self._chk(lib().orc_get_coef(self._h, comp, which, out.ctypes.data))
        return out


def run_scenario(sc, apply_fn, threads=None):
    """Run a scenario to completion; returns {probe name: waveform}."""
    if threads:
        set_threads(threads)
    o = Oracle.from_params(sc.params())
    ids = apply_fn(sc, o)
    o.step(sc.n_steps)
    return {p[0]: o.probe(i) for p, i in zip(sc.probes, ids)}
