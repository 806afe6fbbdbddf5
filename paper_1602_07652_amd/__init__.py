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
    "LS_SWEEP_SEQUENTIAL", "LS_SWEEP_DECOUPLED", "LS_LEVEL0_AUTO", "LS_LEVEL0_DENSE",
]

LS_PREC_BD, LS_PREC_PT1, LS_PREC_NONE = 0, 1, 2
LS_FP64, LS_FP32_REFINE = 0, 1
LS_SWEEP_SEQUENTIAL, LS_SWEEP_DECOUPLED = 0, 1
LS_LEVEL0_AUTO, LS_LEVEL0_DENSE = 0, 1
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
        ("use_graphs", ctypes.c_int), ("autotune", ctypes.c_int), ("fft_variant", ctypes.c_int),
        ("sweep", ctypes.c_int), ("level0", ctypes.c_int),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("outer_its", ctypes.c_int), ("inner_its_total", ctypes.c_int),
        ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double),
        ("converged", ctypes.c_int), ("t_ms", ctypes.c_double),
        ("fno_flags", ctypes.c_int),
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
        "ls_plan_create_like": (_i, [ctypes.POINTER(_vp), _vp, _vp, ctypes.POINTER(Options), _vp]),
        "ls_plan_timings": (_i, [_vp, ctypes.POINTER(_d), _i]),
        "ls_plan_info": (_i, [_vp, ctypes.POINTER(_i), _i]),
        "ls_apply": (_i, [_vp, _vp, _vp, _i]),
        "ls_apply_c64": (_i, [_vp, _vp, _vp, _i]),
        "ls_rhs_from_incident": (_i, [_vp, _vp, _vp, _i]),
        "ls_precond_apply": (_i, [_vp, _vp, _vp, _i]),
        "ls_solve": (_i, [_vp, _vp, _vp, _i, _d, ctypes.POINTER(SolveInfo)]),
        "ls_sparse_solve": (_i, [_vp, _vp, _vp, _i, _d, _i, ctypes.POINTER(SolveInfo)]),
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
        "ls_slab_solve_noalloc": (_i, [_vp, _i, _i, _vp, _vp]),
        "ls_noalloc_scratch_bytes": (ctypes.c_size_t, []),
        "ls_sweep": (_i, [_vp, _i, _vp, _vp]),
        "ls_bidirectional": (_i, [_vp, _vp, _vp]),
        "ls_solve_multi": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                ctypes.POINTER(_i), _d, ctypes.POINTER(ctypes.POINTER(SolveInfo))]),
        "ls_fno_param_count": (ctypes.c_size_t, []),
        "ls_fno_create": (_i, [ctypes.POINTER(_vp), _i, _i, _vp]),
        "ls_fno_destroy": (_i, [_vp]),
        "ls_fno_set_params": (_i, [_vp, _vp]),
        "ls_fno_get_params": (_i, [_vp, _vp]),
        "ls_fno_make_inputs": (_i, [_vp, _i, _i, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp]),
        "ls_fno_forward": (_i, [_vp, _i, _i, _vp, _vp, _i]),
        "ls_fno_loss": (_i, [_vp, _i, _i, _vp, _vp, _vp, ctypes.POINTER(_d)]),
        "ls_fno_backward": (_i, [_vp, _i, _i, _vp, _vp]),
        "ls_fno_adam": (_i, [_vp, _vp, _d, _d, _d, _d, _i]),
        "ls_fno_apply": (_i, [_vp, _i, _i, _vp, ctypes.c_size_t, _vp, _vp, _vp]),
        "ls_bf16_gemm": (_i, [_i, _i, _i, _i, _vp, ctypes.c_longlong, ctypes.c_longlong,
                              ctypes.c_longlong, _vp, ctypes.c_longlong, ctypes.c_longlong,
                              ctypes.c_longlong, _vp, ctypes.c_longlong, ctypes.c_longlong,
                              ctypes.c_longlong, ctypes.c_float, ctypes.c_float, _vp]),
        "ls_solve_fno": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _d, _i, ctypes.POINTER(SolveInfo)]),
        "ls_solve_fno_multi": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i, ctypes.POINTER(_vp),
                                    ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i), _d, _i,
                                    ctypes.POINTER(ctypes.POINTER(SolveInfo))]),
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

    def __init__(self, n: int, h: float, omega: float, m: torch.Tensor, like=None, **opts):
        """like: an existing Plan of the same (n, h, omega) whose spectrum and
        stencils are reused (ls_plan_create_like)."""
        self.n, self.h, self.omega = int(n), float(h), float(omega)
        self.options = default_options(**opts)
        self._m = m.contiguous()
        self.stream = torch.cuda.current_stream(m.device)
        handle = ctypes.c_void_p()
        if like is not None:
            if (like.n, like.h, like.omega) != (self.n, self.h, self.omega):
                raise ValueError("like: the source plan has another (n, h, omega)")
            _check("ls_plan_create_like", lib().ls_plan_create_like(
                ctypes.byref(handle), like.handle, _ptr(self._m, n * n, "m", torch.float64),
                ctypes.byref(self.options), ctypes.c_void_p(self.stream.cuda_stream)))
        else:
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

    def sparse_solve(self, g, tol=1e-6, max_its=200, out=None, allow_noconv=False):
        """ls_sparse_solve: GMRES on C v = g with the plan's inner preconditioner."""
        b = self._batch(g)
        out = torch.empty_like(g) if out is None else out
        N = self.n * self.n * b
        infos = (SolveInfo * b)()
        code = lib().ls_sparse_solve(self.handle, _ptr(g, N, "g"), _ptr(out, N, "v"), b, float(tol),
                                     int(max_its), infos)
        if not (allow_noconv and code == 4):
            _check("ls_sparse_solve", code)
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

    STAGES = ("samples", "stencils", "spectrum", "assembly", "factorisation", "top", "maps", "autotune",
              "total")

    def timings(self):
        """ls_plan_timings: wall ms of the off-line stage by step."""
        ms = (_d * 9)()
        _check("ls_plan_timings", lib().ls_plan_timings(self.handle, ms, 9))
        return dict(zip(self.STAGES, list(ms)))

    def info(self):
        """ls_plan_info: {"tridiagonal_level0": 0/1, "top_blocks": blocks,
        "fft_variant64": v, "fft_variant32": v or -1}."""
        v = (_i * 4)()
        _check("ls_plan_info", lib().ls_plan_info(self.handle, v, 4))
        return {"tridiagonal_level0": v[0], "top_blocks": v[1], "fft_variant64": v[2], "fft_variant32": v[3]}

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

    def slab_solve_noalloc(self, orient, slab, b, out=None):
        """ls_slab_solve_noalloc: ls_slab_solve with its scratch in the
        library's static device array (the call allocates nothing)."""
        a_, b_, z0, z1 = self.slab_info(orient, slab)
        q = z1 - z0 + 1
        out = torch.empty_like(b) if out is None else out
        _check("ls_slab_solve_noalloc", lib().ls_slab_solve_noalloc(
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

    def solve_fno(self, fno, uI, f, tol=1e-8, mode=3, out=None, allow_noconv=False):
        """ls_solve_fno: solve with the network as warm start (mode bit 1)
        and / or flexible-GMRES preconditioner (bit 2), plain BD fallback;
        bit 4 probes the warm start on the first right-hand side first."""
        b = self._batch(f)
        out = torch.empty_like(f) if out is None else out
        N = self.n * self.n * b
        infos = (SolveInfo * b)()
        code = lib().ls_solve_fno(self.handle, fno.handle, _ptr(uI, N, "uI"), _ptr(f, N, "f"),
                                  _ptr(out, N, "u"), b, float(tol), int(mode), infos)
        if not (allow_noconv and code == 4):
            _check("ls_solve_fno", code)
        return out, [i.as_dict() for i in infos]


LS_FNO_WARM, LS_FNO_PREC, LS_FNO_PROBE = 1, 2, 4
LS_FNO_WARM_USED, LS_FNO_WARM_REJECTED, LS_FNO_PREC_USED, LS_FNO_PREC_FALLBACK = 1, 2, 4, 8
LS_FNO_WARM_SKIPPED = 16


def fno_param_count() -> int:
    return int(lib().ls_fno_param_count())


class Fno:
    """The learned preconditioner: ls_fno_create ... ls_fno_destroy.

    Parameters and activations live on the device; every method enqueues the
    library's kernels on the handle's stream (the current torch stream of
    `device` at creation)."""

    def __init__(self, max_batch: int, max_n: int, device="cuda:0"):
        self.device = torch.device(device)
        self.max_batch, self.max_n = int(max_batch), int(max_n)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check("ls_fno_create", lib().ls_fno_create(ctypes.byref(h), self.max_batch, self.max_n,
                                                    ctypes.c_void_p(self.stream.cuda_stream)))
        self.handle = h
        self.nparams = fno_param_count()

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().ls_fno_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: torch.Tensor):
        _check("ls_fno_set_params", lib().ls_fno_set_params(
            self.handle, _ptr(params, self.nparams, "params", torch.float32)))

    def get_params(self) -> torch.Tensor:
        out = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check("ls_fno_get_params", lib().ls_fno_get_params(self.handle, _ptr(out, self.nparams, "params",
                                                                               torch.float32)))
        return out

    def make_inputs(self, m, uI, r, shared_medium=True):
        S, n = r.shape[0], r.shape[-1]
        P = n * n
        x = torch.empty((S, 5, n, n), dtype=torch.float32, device=self.device)
        s = torch.empty(S, dtype=torch.float64, device=self.device)
        _check("ls_fno_make_inputs", lib().ls_fno_make_inputs(
            self.handle, n, S, _ptr(m, P if shared_medium else S * P, "m", torch.float64),
            0 if shared_medium else P, _ptr(uI, S * P, "uI"), _ptr(r, S * P, "r"),
            _ptr(x, S * 5 * P, "x", torch.float32), _ptr(s, S, "s", torch.float64)))
        return x, s

    def forward(self, x, keep=False, out=None):
        S, n = x.shape[0], x.shape[-1]
        y = torch.empty((S, 2, n, n), dtype=torch.float32, device=self.device) if out is None else out
        _check("ls_fno_forward", lib().ls_fno_forward(
            self.handle, n, S, _ptr(x, S * 5 * n * n, "x", torch.float32),
            _ptr(y, S * 2 * n * n, "y", torch.float32), int(bool(keep))))
        return y

    def loss(self, y, target, dy=None):
        S, n = y.shape[0], y.shape[-1]
        dy = torch.empty_like(y) if dy is None else dy
        L = _d()
        Q = S * 2 * n * n
        _check("ls_fno_loss", lib().ls_fno_loss(
            self.handle, n, S, _ptr(y, Q, "y", torch.float32), _ptr(target, Q, "target", torch.float32),
            _ptr(dy, Q, "dy", torch.float32), ctypes.byref(L)))
        return L.value, dy

    def backward(self, dy, grad=None):
        S, n = dy.shape[0], dy.shape[-1]
        grad = torch.empty(self.nparams, dtype=torch.float32, device=self.device) if grad is None else grad
        _check("ls_fno_backward", lib().ls_fno_backward(
            self.handle, n, S, _ptr(dy, S * 2 * n * n, "dy", torch.float32),
            _ptr(grad, self.nparams, "grad", torch.float32)))
        return grad

    def adam(self, grad, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
        _check("ls_fno_adam", lib().ls_fno_adam(self.handle, _ptr(grad, self.nparams, "grad", torch.float32),
                                                float(lr), float(beta1), float(beta2), float(eps), int(t)))

    def apply(self, m, uI, r, out=None):
        S = Plan._batch(r)
        n = r.shape[-1]
        out = torch.empty_like(r) if out is None else out
        P = n * n
        _check("ls_fno_apply", lib().ls_fno_apply(
            self.handle, n, S, _ptr(m, P, "m", torch.float64), 0, _ptr(uI, S * P, "uI"),
            _ptr(r, S * P, "r"), _ptr(out, S * P, "z")))
        return out


def bf16_gemm(A, B, C, M, N, K, batch, sa, sb, sc, alpha=1.0, beta=0.0, stream=None):
    """ls_bf16_gemm on float32 device tensors; sa = (sam, sak, sab) etc."""
    st = torch.cuda.current_stream(A.device) if stream is None else stream
    _check("ls_bf16_gemm", lib().ls_bf16_gemm(
        M, N, K, batch, ctypes.c_void_p(A.data_ptr()), *sa, ctypes.c_void_p(B.data_ptr()), *sb,
        ctypes.c_void_p(C.data_ptr()), *sc, float(alpha), float(beta), ctypes.c_void_p(st.cuda_stream)))
    return C


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


def solve_fno_multi(plans, fnos, uIs, fs, tol=1e-8, mode=LS_FNO_WARM, outs=None):
    """ls_solve_fno_multi: ls_solve_fno on several plans concurrently, one
    network handle per plan.  Returns (us, infos)."""
    k = len(plans)
    outs = [torch.empty_like(f) for f in fs] if outs is None else outs
    bs = [Plan._batch(f) for f in fs]
    for p, uI, f, u, b in zip(plans, uIs, fs, outs, bs):
        for t, what in ((uI, "uI"), (f, "f"), (u, "u")):
            _ptr(t, p.n * p.n * b, what)
    P = (_vp * k)(*[p.handle.value for p in plans])
    Fh = (_vp * k)(*[x.handle.value for x in fnos])
    UI = (_vp * k)(*[t.data_ptr() for t in uIs])
    F = (_vp * k)(*[t.data_ptr() for t in fs])
    U = (_vp * k)(*[t.data_ptr() for t in outs])
    B = (_i * k)(*bs)
    infos = [(SolveInfo * b)() for b in bs]
    I = (ctypes.POINTER(SolveInfo) * k)(*[ctypes.cast(x, ctypes.POINTER(SolveInfo)) for x in infos])
    _check("ls_solve_fno_multi", lib().ls_solve_fno_multi(P, Fh, k, UI, F, U, B, float(tol), int(mode), I))
    return outs, [[i.as_dict() for i in x] for x in infos]
