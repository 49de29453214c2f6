"""Python binding of the surrogate network library (argument marshalling only).

Forward, backward, Adam and the ensemble routing all run in the HIP kernels
of ``libmi355fdtd.so``; PyTorch only provides device memory and the stream.
There is no CPU fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .fdtd import lib as _fdtd_lib

SUR_ERRORS = {0: "OK", -1: "EINVAL", -3: "ESTATE", -5: "ENOMEM", -6: "EDEVICE"}

_vp = C.c_void_p
# (name, restype, argtypes) of every exported symbol declared in include/sur.h
SIGNATURES = [
    ("sur_create", C.c_int, [C.POINTER(C.c_int), C.c_int, C.c_int, C.c_int, _vp, C.POINTER(_vp)]),
    ("sur_workspace_bytes", C.c_size_t, [_vp]),
    ("sur_bind_workspace", C.c_int, [_vp, _vp, C.c_size_t]),
    ("sur_num_params", C.c_longlong, [_vp]),
    ("sur_init_params", C.c_int, [_vp, C.c_int, C.c_ulonglong]),
    ("sur_set_params", C.c_int, [_vp, C.c_int, _vp]),
    ("sur_get_params", C.c_int, [_vp, C.c_int, _vp]),
    ("sur_get_grads", C.c_int, [_vp, C.c_int, _vp]),
    ("sur_train_step", C.c_int, [_vp, C.c_int, _vp, _vp, _vp, C.c_int, C.c_float, C.c_int, _vp]),
    ("sur_forward", C.c_int, [_vp, C.c_int, _vp, C.c_int, _vp]),
    ("sur_infer_route", C.c_int, [_vp, _vp, C.c_int, C.c_float, _vp, _vp, _vp, _vp]),
    ("sur_set_input_bound", C.c_int, [_vp, C.c_float]),
    ("sur_set_kernel", C.c_int, [_vp, C.c_int]),
    ("sur_last_error", C.c_char_p, [_vp]),
    ("sur_destroy", None, [_vp]),
]

_bound = False


def lib():
    global _bound
    L = _fdtd_lib()
    if not _bound:
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _bound = True
    return L


class SurError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{SUR_ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Ensemble:
    """n_nets independent MLPs of the same widths on one GPU."""

    def __init__(self, widths, n_nets=1, max_rows=8192, device="cuda:0"):
        import torch
        self.widths = [int(w) for w in widths]
        self.n_nets = n_nets
        self.max_rows = max_rows
        self.device = torch.device(device)
        arr = (C.c_int * len(self.widths))(*self.widths)
        h = C.c_void_p()
        st = C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        rc = lib().sur_create(arr, len(self.widths), n_nets, max_rows, st, C.byref(h))
        if rc:
            raise SurError(rc, "sur_create rejected the configuration")
        self._h = h
        nbytes = lib().sur_workspace_bytes(h)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._chk(lib().sur_bind_workspace(h, _ptr(self._ws), nbytes))
        self.n_params = lib().sur_num_params(h)
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().sur_destroy(h)
            self._h = None

    def _chk(self, rc):
        if rc:
            raise SurError(rc, lib().sur_last_error(self._h).decode())

    @property
    def workspace_bytes(self):
        return self._ws.numel()

    def init_params(self, net, seed):
        self._chk(lib().sur_init_params(self._h, net, seed))

    def set_params(self, net, flat):
        v = np.ascontiguousarray(flat, dtype=np.float32)
        assert v.size == self.n_params
        self._chk(lib().sur_set_params(self._h, net, v.ctypes.data_as(C.c_void_p)))

    def get_params(self, net):
        v = np.empty(self.n_params, np.float32)
        self._chk(lib().sur_get_params(self._h, net, v.ctypes.data_as(C.c_void_p)))
        return v

    def get_grads(self, net):
        v = np.empty(self.n_params, np.float32)
        self._chk(lib().sur_get_grads(self._h, net, v.ctypes.data_as(C.c_void_p)))
        return v

    def train_step(self, net, x, t, rows=None, batch=None, lr=1e-3, update=True, loss=None):
        """x, t: float32 device tensors [N x w0], [N x wL]; rows: int32 device
        tensor of batch row indices (or None for the first `batch` rows)."""
        if batch is None:
            batch = rows.numel() if rows is not None else x.shape[0]
        self._chk(lib().sur_train_step(self._h, net, _ptr(x), _ptr(t), _ptr(rows), int(batch), float(lr),
                                       int(bool(update)), _ptr(loss if loss is not None else self._loss)))
        return self._loss if loss is None else loss

    def forward(self, net, x, out=None):
        import torch
        n = x.shape[0]
        if out is None:
            out = torch.empty((n, self.widths[-1]), dtype=torch.float32, device=self.device)
        self._chk(lib().sur_forward(self._h, net, _ptr(x), n, _ptr(out)))
        return out

    def set_kernel(self, fused):
        """1: fused inference (default); 0: one product launch per layer."""
        self._chk(lib().sur_set_kernel(self._h, int(fused)))

    def set_input_bound(self, bound):
        """Route rows with any input outside [-bound, bound] (inf: off)."""
        self._chk(lib().sur_set_input_bound(self._h, float(bound)))

    def infer_route(self, x, threshold):
        """Mean prediction, spread and the ordered fallback row list."""
        import torch
        n = x.shape[0]
        ymean = torch.empty((n, self.widths[-1]), dtype=torch.float32, device=self.device)
        spread = torch.empty(n, dtype=torch.float32, device=self.device)
        ids = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._chk(lib().sur_infer_route(self._h, _ptr(x), n, float(threshold), _ptr(ymean), _ptr(spread),
                                        _ptr(ids), _ptr(cnt)))
        return ymean, spread, ids, cnt
