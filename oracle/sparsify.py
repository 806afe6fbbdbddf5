"""Sparsifying preconditioner: stencils alpha, matrices A and C.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 2: mu(k) = {p : ||k - p||_inf <= 1, x_p in Omega}; A has the
pattern of mu, A(k, :) G(:, mu(k)^c) ~ 0; by translation invariance one
problem min_{|alpha|=1} ||alpha G(mu(0), mu(0)^c)|| solved by the SVD
G(mu, mu^c) = U S V^*.  C is A H = A + omega^2 A G D with everything off the
pattern of A dropped, and the preconditioner is u = C^{-1} A f (eq.
preconditioner).  Section 4.1: the SVD is of a 9 x N matrix.

Readings:
* The printed "alpha = U(:, mu(0))^*" is read as the conjugate of the left
  singular vector of the smallest singular value (that vector is the
  minimiser of ||alpha M|| for a row vector alpha).
* mu^c is the complement in the whole n x n grid.
* Boundary points (the paper omits their treatment): the same minimisation
  with mu(k) clipped to the grid, giving 9 stencil types (interior, 4 edges,
  4 corners) from representative points: the grid centre (n//2, n//2), edge
  midpoints and corners (0-based indices).
* The singular vector's phase is arbitrary; it is fixed so that the centre
  coefficient is real and positive.
* "Threshold the small entries" keeps exactly the pattern of A:
  C(k, k+d) = alpha_d + omega^2 beta_d m_{k+d} with
  beta_d = sum_{d'} alpha_{d'} w_{d'-d} for d, d' in mu.

Stencil tables are arrays [tz, tx, dz+1, dx+1] with tz, tx in {0: low edge,
1: interior, 2: high edge}; entries outside the type's mu are zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps


def type_offsets(tz: int, tx: int):
    """Offsets (dz, dx) of mu for a stencil type."""
    rz = {0: (0, 1), 1: (-1, 0, 1), 2: (-1, 0)}[tz]
    rx = {0: (0, 1), 1: (-1, 0, 1), 2: (-1, 0)}[tx]
    return [(dz, dx) for dz in rz for dx in rx]


def representative_point(n: int, tz: int, tx: int):
    pick = {0: 0, 1: n // 2, 2: n - 1}
    return pick[tz], pick[tx]


def stencil_matrix(W: np.ndarray, n: int, tz: int, tx: int):
    """M = G(mu(k0), mu(k0)^c) for the type's representative point k0."""
    offs = type_offsets(tz, tx)
    j0, i0 = representative_point(n, tz, tx)
    jj, ii = np.divmod(np.arange(n * n), n)
    inmu = np.zeros(n * n, dtype=bool)
    for dz, dx in offs:
        inmu[(j0 + dz) * n + (i0 + dx)] = True
    pj, pi = jj[~inmu], ii[~inmu]
    M = np.empty((len(offs), pj.size), dtype=complex)
    for r, (dz, dx) in enumerate(offs):
        M[r] = W[(j0 + dz) - pj + n - 1, (i0 + dx) - pi + n - 1]
    return M, offs


def stencils(W: np.ndarray, n: int):
    """alpha, beta tables [3, 3, 3, 3] (Section 2; readings above)."""
    alpha = np.zeros((3, 3, 3, 3), dtype=complex)
    beta = np.zeros((3, 3, 3, 3), dtype=complex)
    sigma = np.zeros((3, 3, 2))
    for tz in range(3):
        for tx in range(3):
            M, offs = stencil_matrix(W, n, tz, tx)
            U, s, _ = np.linalg.svd(M, full_matrices=False)
            a = np.conj(U[:, -1])
            c = a[offs.index((0, 0))]
            a = a * (np.conj(c) / abs(c))
            sigma[tz, tx] = s[-1], s[0]
            for r, (dz, dx) in enumerate(offs):
                alpha[tz, tx, dz + 1, dx + 1] = a[r]
            for dz, dx in offs:
                b = 0j
                for r, (ez, ex) in enumerate(offs):
                    b += a[r] * W[ez - dz + n - 1, ex - dx + n - 1]
                beta[tz, tx, dz + 1, dx + 1] = b
    return alpha, beta, sigma


def point_types(n: int):
    """Per-index stencil type along one axis: 0 at index 0, 2 at n-1, else 1."""
    t = np.ones(n, dtype=int)
    t[0] = 0
    t[-1] = 2
    return t


def apply_A(alpha: np.ndarray, r: np.ndarray) -> np.ndarray:
    """(A r)_k = sum_{d in mu(k)} alpha^{type(k)}_d r_{k+d}."""
    n = r.shape[-1]
    tzs, txs = point_types(n), point_types(n)
    out = np.zeros(r.shape, dtype=complex)
    rp = np.pad(r, [(0, 0)] * (r.ndim - 2) + [(1, 1), (1, 1)])
    for dz in (-1, 0, 1):
        for dx in (-1, 0, 1):
            coef = alpha[tzs[:, None], txs[None, :], dz + 1, dx + 1]
            out += coef * rp[..., 1 + dz:1 + dz + n, 1 + dx:1 + dx + n]
    return out


def assemble_C(alpha, beta, m, omega):
    """C = A + omega^2 B D as a CSR matrix in the row-by-row ordering."""
    n = m.shape[0]
    tzs, txs = point_types(n), point_types(n)
    rows, cols, vals = [], [], []
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for dz in (-1, 0, 1):
        for dx in (-1, 0, 1):
            a = alpha[tzs[:, None], txs[None, :], dz + 1, dx + 1]
            b = beta[tzs[:, None], txs[None, :], dz + 1, dx + 1]
            Jn, In = J + dz, I + dx
            ok = (Jn >= 0) & (Jn < n) & (In >= 0) & (In < n)
            mn = np.zeros((n, n))
            mn[ok] = m[Jn[ok], In[ok]]
            v = a + omega**2 * b * mn
            rows.append((J * n + I)[ok])
            cols.append((Jn * n + In)[ok])
            vals.append(v[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sps.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def dense_A(alpha, n):
    """Dense A (small n only)."""
    N = n * n
    A = np.zeros((N, N), dtype=complex)
    for k in range(N):
        e = np.zeros(N, dtype=complex)
        e[k] = 1.0
        A[:, k] = apply_A(alpha, e.reshape(n, n)).reshape(-1)
    return A
