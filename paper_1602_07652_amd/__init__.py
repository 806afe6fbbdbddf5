"""MI355X two-level Lippmann-Schwinger solver: Python binding.

Thin ctypes layer over libls_mi355x.so (declared in include/ls.h).  It only
marshals arguments: every step of the solver runs in the library's HIP
kernels.  PyTorch provides device memory (complex128 tensors on a HIP
device, whose storage is interleaved (re, im) doubles, as the ABI expects)
and the stream.

The library must have been built (``python -m paper_1602_07652_amd.build``);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

from .build import lib_path

__all__ = [
    "Options", "SolveInfo", "LSError", "Plan", "lib", "solve_multi",
    "LS_PREC_BD", "LS_PREC_PT1", "LS_PREC_NONE", "LS_FP64", "LS_FP32_REFINE",
]

LS_PREC_BD, LS_PREC_PT1, LS_PREC_NONE = 0, 1, 2
LS_FP64, LS_FP32_REFINE = 0, 1
_STATUS = {0: "LS_OK", 1: "LS_EINVAL", 2: "LS_ENOMEM", 3: "LS_EDEVICE", 4: "LS_ENOCONV",
           5: "LS_ESINGULAR", 6: "LS_EUNSUPPORTED"}


class LSError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn}: {_STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("slabs", ctypes.c_int), ("ext", ctypes.c_int), ("inner_tol", ctypes.c_double),
        ("max_outer", ctypes.c_int), ("max_inner", ctypes.c_int), ("shift_c", ctypes.c_double),
        ("precision", ctypes.c_int), ("precond", ctypes.c_int),
        ("inner_fixed_iters", ctypes.c_int), ("max_batch", ctypes.c_int),
        ("lowp_tol", ctypes.c_double), ("max_refine", ctypes.c_int),
        ("use_graphs", ctypes.c_int), ("autotune", ctypes.c_int),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("outer_its", ctypes.c_int), ("inner_its_total", ctypes.c_int),
        ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double),
        ("converged", ctypes.c_int), ("t_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double


def lib():
    """Load libls_mi355x.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_1602_07652_amd.build`")
    L = ctypes.CDLL(path)
    sig = {
        "ls_options_default": (None, [ctypes.POINTER(Options)]),
        "ls_plan_create": (_i, [ctypes.POINTER(_vp), _i, _d, _d, _vp, ctypes.POINTER(Options), _vp]),
        "ls_plan_destroy": (_i, [_vp]),
        "ls_apply": (_i, [_vp, _vp, _vp, _i]),
        "ls_apply_c64": (_i, [_vp, _vp, _vp, _i]),
        "ls_rhs_from_incident": (_i, [_vp, _vp, _vp, _i]),
        "ls_precond_apply": (_i, [_vp, _vp, _vp, _i]),
        "ls_solve": (_i, [_vp, _vp, _vp, _i, _d, ctypes.POINTER(SolveInfo)]),
        "ls_status_str": (ctypes.c_char_p, [_i]),
        "ls_last_error": (ctypes.c_char_p, []),
        "ls_plan_dims": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "ls_get_kernel_samples": (_i, [_vp, _vp]),
        "ls_get_spectrum": (_i, [_vp, _vp]),
        "ls_get_stencils": (_i, [_vp, _vp, _vp]),
        "ls_stencil_A": (_i, [_vp, _vp, _vp, _i]),
        "ls_stencil_C": (_i, [_vp, _vp, _vp, _i]),
        "ls_slab_info": (_i, [_vp, _i, _i, ctypes.POINTER(_i)]),
        "ls_slab_solve": (_i, [_vp, _i, _i, _vp, _vp]),
        "ls_sweep": (_i, [_vp, _i, _vp, _vp]),
        "ls_bidirectional": (_i, [_vp, _vp, _vp]),
        "ls_solve_multi": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                ctypes.POINTER(_i), _d, ctypes.POINTER(ctypes.POINTER(SolveInfo))]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(fn, code):
    if code != 0:
        raise LSError(fn, code, lib().ls_last_error().decode())


def _ptr(t: torch.Tensor, n_elems: int, what: str, dtype=torch.complex128):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{what}: expected a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < n_elems:
        raise ValueError(f"{what}: expected contiguous {dtype} with >= {n_elems} elements")
    return ctypes.c_void_p(t.data_ptr())


def default_options(**kw) -> Options:
    o = Options()
    lib().ls_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Plan:
    """One medium: ls_plan_create ... ls_plan_destroy.

    m: float64 device tensor [n, n] (m[j, i] at (h(i+1), h(j+1))).  Keyword
    arguments set ls_options fields.  The plan uses the current torch stream.
    """

    def __init__(self, n: int, h: float, omega: float, m: torch.Tensor, **opts):
        self.n, self.h, self.omega = int(n), float(h), float(omega)
        self.options = default_options(**opts)
        self._m = m.contiguous()
        self.stream = torch.cuda.current_stream(m.device)
        handle = ctypes.c_void_p()
        _check("ls_plan_create", lib().ls_plan_create(
            ctypes.byref(handle), self.n, self.h, self.omega,
            _ptr(self._m, n * n, "m", torch.float64), ctypes.byref(self.options),
            ctypes.c_void_p(self.stream.cuda_stream)))
        self.handle = handle
        P, L, ss = _i(), _i(), _i()
        _check("ls_plan_dims", lib().ls_plan_dims(handle, ctypes.byref(P), ctypes.byref(L), ctypes.byref(ss)))
        self.P, self.L, self.spec_side = P.value, L.value, ss.value
        self.device = m.device

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().ls_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def _grid(self, batch=None):
        shape = (self.n, self.n) if batch is None else (batch, self.n, self.n)
        return torch.empty(shape, dtype=torch.complex128, device=self.device)

    @staticmethod
    def _batch(t):
        return 1 if t.dim() == 2 else t.shape[0]

    # -- ABI entry points ----------------------------------------------------
    def apply(self, v, out=None):
        b = self._batch(v)
        out = torch.empty_like(v) if out is None else out
        N = self.n * self.n * b
        _check("ls_apply", lib().ls_apply(self.handle, _ptr(v, N, "v"), _ptr(out, N, "Hv"), b))
        return out

    def apply_c64(self, v, out=None):
        """FP32 operator (LS_FP32_REFINE plans); v complex64."""
        b = self._batch(v)
        out = torch.empty_like(v) if out is None else out
        N = self.n * self.n * b
        _check("ls_apply_c64", lib().ls_apply_c64(
            self.handle, _ptr(v, N, "v", torch.complex64), _ptr(out, N, "Hv", torch.complex64), b))
        return out

    def rhs_from_incident(self, uI, out=None):
        b = self._batch(uI)
        out = torch.empty_like(uI) if out is None else out
        N = self.n * self.n * b
        _check("ls_rhs_from_incident", lib().ls_rhs_from_incident(
            self.handle, _ptr(uI, N, "uI"), _ptr(out, N, "f"), b))
        return out

    def precond_apply(self, r, out=None):
        b = self._batch(r)
        out = torch.empty_like(r) if out is None else out
        N = self.n * self.n * b
        code = lib().ls_precond_apply(self.handle, _ptr(r, N, "r"), _ptr(out, N, "z"), b)
        _check("ls_precond_apply", code)
        return out

    def solve(self, f, tol=1e-8, out=None, allow_noconv=False):
        b = self._batch(f)
        out = torch.empty_like(f) if out is None else out
        N = self.n * self.n * b
        infos = (SolveInfo * b)()
        code = lib().ls_solve(self.handle, _ptr(f, N, "f"), _ptr(out, N, "u"), b, float(tol), infos)
        if not (allow_noconv and code == 4):
            _check("ls_solve", code)
        return out, [i.as_dict() for i in infos]

    def kernel_samples(self):
        W = 2 * self.n - 1
        out = torch.empty((W, W), dtype=torch.complex128, device=self.device)
        _check("ls_get_kernel_samples", lib().ls_get_kernel_samples(self.handle, _ptr(out, W * W, "w")))
        return out

    def spectrum(self):
        s = self.spec_side
        out = torch.empty((s, s), dtype=torch.complex128, device=self.device)
        _check("ls_get_spectrum", lib().ls_get_spectrum(self.handle, _ptr(out, s * s, "S")))
        return out

    def stencils(self):
        import numpy as np
        a = np.zeros(162)
        b = np.zeros(162)
        _check("ls_get_stencils", lib().ls_get_stencils(
            self.handle, a.ctypes.data_as(_vp), b.ctypes.data_as(_vp)))
        ca = (a[0::2] + 1j * a[1::2]).reshape(3, 3, 3, 3)
        cb = (b[0::2] + 1j * b[1::2]).reshape(3, 3, 3, 3)
        return ca, cb

    def stencil_A(self, r, out=None):
        b = self._batch(r)
        out = torch.empty_like(r) if out is None else out
        N = self.n * self.n * b
        _check("ls_stencil_A", lib().ls_stencil_A(self.handle, _ptr(r, N, "r"), _ptr(out, N, "y"), b))
        return out

    def stencil_C(self, v, out=None):
        b = self._batch(v)
        out = torch.empty_like(v) if out is None else out
        N = self.n * self.n * b
        _check("ls_stencil_C", lib().ls_stencil_C(self.handle, _ptr(v, N, "v"), _ptr(out, N, "y"), b))
        return out

    def slab_info(self, orient, slab):
        lims = (_i * 4)()
        _check("ls_slab_info", lib().ls_slab_info(self.handle, orient, slab, lims))
        return tuple(lims)

    def slab_solve(self, orient, slab, b, out=None):
        a_, b_, z0, z1 = self.slab_info(orient, slab)
        q = z1 - z0 + 1
        out = torch.empty_like(b) if out is None else out
        _check("ls_slab_solve", lib().ls_slab_solve(
            self.handle, orient, slab, _ptr(b, self.n * q, "b"), _ptr(out, self.n * q, "x")))
        return out

    def sweep(self, orient, g, out=None):
        out = self._grid() if out is None else out
        N = self.n * self.n
        _check("ls_sweep", lib().ls_sweep(self.handle, orient, _ptr(g, N, "g"), _ptr(out, N, "v")))
        return out

    def bidirectional(self, g, out=None):
        out = self._grid() if out is None else out
        N = self.n * self.n
        _check("ls_bidirectional", lib().ls_bidirectional(self.handle, _ptr(g, N, "g"), _ptr(out, N, "v")))
        return out


def solve_multi(plans, fs, tol=1e-8, outs=None):
    """ls_solve_multi: solve several plans' right-hand sides concurrently.

    plans: list of Plan (distinct streams); fs: list of complex128 device
    tensors [batch_i, n_i, n_i] (or [n_i, n_i]).  Returns (us, infos)."""
    k = len(plans)
    outs = [torch.empty_like(f) for f in fs] if outs is None else outs
    P = (_vp * k)(*[p.handle.value for p in plans])
    F = (_vp * k)(*[f.data_ptr() for f in fs])
    U = (_vp * k)(*[u.data_ptr() for u in outs])
    bs = [Plan._batch(f) for f in fs]
    for p, f, u, b in zip(plans, fs, outs, bs):
        _ptr(f, p.n * p.n * b, "f")
        _ptr(u, p.n * p.n * b, "u")
    B = (_i * k)(*bs)
    infos = [(SolveInfo * b)() for b in bs]
    I = (ctypes.POINTER(SolveInfo) * k)(*[ctypes.cast(x, ctypes.POINTER(SolveInfo)) for x in infos])
    code = lib().ls_solve_multi(P, k, F, U, B, float(tol), I)
    _check("ls_solve_multi", code)
    return outs, [[i.as_dict() for i in x] for x in infos]
