"""Two-level solver: Alg. 3 and the outer flexible GMRES.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 4: off-line stage (stencils, C, local matrices and their
factorisations) done once per medium; on-line stage per right-hand side:
outer GMRES on H u = f preconditioned by Alg. 3,
u = GMRES(C, A f, BiDirectionalPreconditioner, tol = 1e-3).
The result of a solve is (up to the stopping tolerance) the exact discrete
solution u* = H^{-1} f of Section 2; `dense_solve` computes it directly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import kernel, sparsify, slabs, krylov


class Problem:
    """Everything the off-line stage builds for one medium."""

    def __init__(self, n, h, omega, m, slabs_L=4, ext=10, shift_c=0.0,
                 inner_tol=1e-3, max_inner=50, inner_fixed_iters=0, precond="bd"):
        self.n, self.h, self.omega = n, h, omega
        self.m = np.asarray(m, dtype=float)
        self.W = kernel.kernel_samples(n, h, omega)
        self.Ghat = kernel.circulant_spectrum(self.W)
        self.alpha, self.beta, self.sigma = sparsify.stencils(self.W, n)
        self.C = sparsify.assemble_C(self.alpha, self.beta, self.m, omega)
        self.inner_tol, self.max_inner = inner_tol, max_inner
        self.inner_fixed_iters = inner_fixed_iters
        self.precond = precond
        self.bd = None
        if precond in ("bd", "pt1"):
            self.bd = slabs.BiDirectional(self.alpha, self.beta, self.m, omega,
                                          slabs_L, ext, shift_c, C=self.C)
        self._lu = None

    # --- operators -------------------------------------------------------
    def H(self, v):
        return kernel.apply_H(self.W, self.m, v, self.omega, self.Ghat)

    def rhs(self, uI):
        return kernel.rhs_from_incident(self.W, self.m, uI, self.omega, self.Ghat)

    def A(self, r):
        return sparsify.apply_A(self.alpha, r)

    def Cmul(self, v):
        n = self.n
        return (self.C @ v.reshape(-1)).reshape(v.shape)

    def inner_prec(self, g):
        if self.precond == "bd":
            return self.bd.apply(g)
        if self.precond == "pt1":
            return self.bd.prec_h(g)
        return g

    # --- Alg. 3 -----------------------------------------------------------
    def precond_apply(self, r, return_info=False):
        """z = GMRES(C, A r, Alg. 2, inner_tol) (Alg. 3)."""
        g = self.A(r)
        if self.precond == "exact":
            if self._lu is None:
                self._lu = spla.splu(self.C.tocsc())
            z = self._lu.solve(g.reshape(-1)).reshape(g.shape)
            info = dict(iters=0)
        else:
            z, info = krylov.gmres_right(self.Cmul, self.inner_prec, g, self.inner_tol,
                                         self.max_inner, self.inner_fixed_iters)
        return (z, info) if return_info else z

    def solve(self, f, tol=1e-8, max_outer=200, precondition=True):
        """Outer flexible GMRES on H u = f with Alg. 3 as preconditioner."""
        inner_counts = []

        def prec(r):
            z, info = self.precond_apply(r, return_info=True)
            inner_counts.append(info["iters"])
            return z

        u, info = krylov.fgmres(self.H, prec if precondition else (lambda r: r), f, tol, max_outer)
        nf = np.linalg.norm(f)
        info["relres_true"] = float(np.linalg.norm(f - self.H(u)) / nf) if nf > 0 else 0.0
        info["inner_iters"] = inner_counts
        return u, info


def dense_solve(W, m, omega, f):
    """u* = H^{-1} f by dense LU (Section 2; n <= 64)."""
    H = kernel.dense_H(W, m, omega)
    return np.linalg.solve(H, f.reshape(-1)).reshape(f.shape)
