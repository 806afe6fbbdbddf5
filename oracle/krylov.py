"""GMRES with right preconditioning and flexible GMRES.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 4, Alg. 3: the inner level is GMRES(C, A f,
BiDirectionalPreconditioner, tol = 1e-3); the outer level is GMRES on
H u = f preconditioned by Alg. 3.  Section 6 names flexible GMRES (Saad) for
the outer loop.

Readings (the paper does not specify the GMRES variant):
* Both levels start from x0 = 0 and use the relative residual of the
  least-squares problem, ||b - A x|| / ||b||, in the 2-norm.
* Orthogonalisation is classical Gram-Schmidt applied twice (CGS2).
* The outer loop is flexible GMRES (the preconditioner is itself an inner
  GMRES and changes from one call to the next); the inner loop keeps the
  preconditioned vectors Z as well (for a fixed preconditioner this is the
  same as right-preconditioned GMRES, x = M V y).
* No restart.  `fixed_iters > 0` runs exactly that many iterations (used to
  make the inner solve a deterministic function of its right-hand side).
* An iteration whose least-squares residual is <= 1e-15 ||b|| ends the loop
  in every mode (the Krylov space has captured the solution).
"""
from __future__ import annotations

import numpy as np

BREAKDOWN = 1e-15


def _cgs2(V, w):
    h = np.zeros(len(V), dtype=complex)
    for _ in range(2):
        c = np.array([np.vdot(vi, w) for vi in V])
        for ci, vi in zip(c, V):
            w = w - ci * vi
        h += c
    return h, w


def fgmres(apply_op, apply_prec, b, tol, maxit, fixed_iters=0):
    """Flexible GMRES on op(x) = b with right preconditioner prec.

    Returns (x, info) with info = dict(iters, relres_est, history).
    """
    shape = b.shape
    b = b.reshape(-1)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(shape, dtype=complex), dict(iters=0, relres_est=0.0, history=[0.0])
    V = [b / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit), dtype=complex)
    hist = [1.0]
    limit = fixed_iters if fixed_iters > 0 else maxit
    y = None
    for j in range(limit):
        z = np.asarray(apply_prec(V[j].reshape(shape))).reshape(-1)
        Z.append(z)
        w = np.asarray(apply_op(z.reshape(shape))).reshape(-1)
        h, w = _cgs2(V, w)
        H[:j + 1, j] = h
        H[j + 1, j] = np.linalg.norm(w)
        e1 = np.zeros(j + 2, dtype=complex)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)
        res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y) / beta
        hist.append(res)
        done = (fixed_iters == 0 and res <= tol) or res <= BREAKDOWN
        if done or j + 1 == limit:
            break
        V.append(w / H[j + 1, j])
    x = np.zeros_like(b)
    for yi, zi in zip(y, Z):
        x = x + yi * zi
    return x.reshape(shape), dict(iters=len(Z), relres_est=hist[-1], history=hist)


def gmres_right(apply_op, apply_prec, b, tol, maxit, fixed_iters=0):
    """Right-preconditioned GMRES (inner level of Alg. 3)."""
    return fgmres(apply_op, apply_prec, b, tol, maxit, fixed_iters)
