"""Layered decomposition, local slab matrices and the polarized-traces sweeps.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 3.1: Omega split into L horizontal layers Omega^l, each
extended to Omega^l_ext; local problems C^l w^l = g^l = chi_l g.
Compatibility: C^l equals C in the interior of Omega^l.
Section 3.2: block-tridiagonal structure of C in the row-by-row ordering,
local traces v^l_k (k = 0 ghost row below, 1 bottom row, n^l top row,
n^l + 1 ghost row above), delta_k, and eq. (pde_GRF_real), the discrete
Green's representation formula, exact for the global traces.
Section 3.3: the perturbation is localised by a smooth cut-off xi^l (1 on
Omega^l, 0 outside Omega^l_ext), constant in x, a third-order spline in z;
D^l = diag(xi^l m); the rows at the boundary of Omega^l_ext use the
stencils generated at the boundary of Omega; an O(omega) complex shift may be
put in the cut-off region.
Section 3.4, Alg. 1 (Gauss-Seidel preconditioner): a downward sweep then an
upward sweep of local solves with traces passed through the GRF sources.
Section 3.5, Alg. 2 (bi-directional preconditioner):
u1 = Prec(g); e = g - C u1; u2 = Prec^T(e); v = u1 + u2.

Readings:
* Layer sizes: t = n // L rows each, the first n mod L layers get one more
  row (layer 0 is at the bottom, smallest z).  The extension is e rows on
  each side, clipped to the grid.
* Local stencil types: the bottom/top rows of Omega^l_ext use the
  bottom/top edge stencils, the x-edges use the x-edge stencils.
* xi^l = 1 on the layer and on its two ghost rows (the GRF needs C^l = C on
  the rows coupling the layer to its ghost rows), and
  xi = 1 - 3 tau^2 + 2 tau^3 on the rest of the extension, with
  tau = (dist - 1)/(e - 1) and dist the row distance from the layer
  (tau = 0 at the ghost row, 1 at distance e).
* Complex shift: D^l = xi m + i sigma (1 - xi) with sigma = shift_c / omega,
  so omega^2 sigma = shift_c * omega is O(omega); shift_c = 0 by default.
* Alg. 1 as printed has its superscripts garbled: the downward loop reads
  the traces of the layer above (l+1), skipping the top layer; the upward
  loop reads the layer below (l-1), skipping the bottom layer.  The upward
  trace pair is (v0, v1) with v0 = v^{l-1} on its top layer row and
  v1 = v^{l-1} on its upper ghost row plus w^l on its first layer row: the
  downward GRF sources of v^{l-1} annihilate the down-going field above its
  top row, and adding w^l there restores the total field, which makes the
  pair consistent.  g^l keeps the downward sources in the upward sweep
  ("g^l +=" in the printed algorithm).
* Prec^T ("applied to the transpose of C") is Alg. 1 on the grid-transposed
  problem (vertical slabs): x and z swapped, stencil tables transposed and
  m transposed, not Alg. 1 for the matrix transpose of C.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .sparsify import type_offsets, point_types, assemble_C


def layer_partition(n: int, L: int, ext: int):
    """List of (a, b, z0, z1): layer rows [a, b], extended rows [z0, z1]."""
    t, rem = divmod(n, L)
    out = []
    a = 0
    for l in range(L):
        sz = t + 1 if l < rem else t
        b = a + sz - 1
        out.append((a, b, max(0, a - ext), min(n - 1, b + ext)))
        a = b + 1
    return out


def cutoff(j: int, a: int, b: int, ext: int) -> float:
    """xi^l at global row j (reading above)."""
    if a - 1 <= j <= b + 1:
        return 1.0
    dist = a - j if j < a else j - b
    tau = (dist - 1) / (ext - 1)
    return 1.0 - 3.0 * tau**2 + 2.0 * tau**3


def assemble_slab(alpha, beta, m, omega, part, ext, shift_c=0.0):
    """Local matrix C^l on Omega^l_ext as CSR, local index r*n + i with
    r = j - z0 (Section 3.3; readings above)."""
    n = m.shape[1]
    a, b, z0, z1 = part
    q = z1 - z0 + 1
    sigma = shift_c / omega
    xi = np.array([cutoff(j, a, b, ext) for j in range(z0, z1 + 1)])
    D = xi[:, None] * m[z0:z1 + 1, :] + 1j * sigma * (1.0 - xi)[:, None]
    txs = point_types(n)
    rows, cols, vals = [], [], []
    for r in range(q):
        j = z0 + r
        tz = 0 if j == z0 else (2 if j == z1 else 1)
        for i in range(n):
            tx = txs[i]
            for dz, dx in type_offsets(tz, tx):
                rr, ii = r + dz, i + dx
                rows.append(r * n + i)
                cols.append(rr * n + ii)
                vals.append(alpha[tz, tx, dz + 1, dx + 1]
                            + omega**2 * beta[tz, tx, dz + 1, dx + 1] * D[rr, ii])
    return sps.csr_matrix((vals, (rows, cols)), shape=(q * n, q * n))


class Sweep:
    """Alg. 1 (Gauss-Seidel polarized traces) on horizontal slabs."""

    def __init__(self, alpha, beta, m, omega, L, ext, shift_c=0.0):
        self.n = m.shape[1]
        self.parts = layer_partition(self.n, L, ext)
        self.mats = [assemble_slab(alpha, beta, m, omega, p, ext, shift_c) for p in self.parts]
        self.lus = [spla.splu(C.tocsc()) for C in self.mats]

    def block(self, l, j_row, j_col):
        """Coupling block C^l(row j_row, row j_col) as an n x n sparse matrix."""
        n = self.n
        z0 = self.parts[l][2]
        r1, r2 = j_row - z0, j_col - z0
        return self.mats[l][r1 * n:(r1 + 1) * n, r2 * n:(r2 + 1) * n]

    def local_solve(self, l, g_loc):
        q = g_loc.shape[0]
        return self.lus[l].solve(g_loc.reshape(-1)).reshape(q, self.n)

    def apply(self, g: np.ndarray) -> np.ndarray:
        """v = Preconditioner(g), Alg. 1 with the readings above."""
        L = len(self.parts)
        gl, w = [None] * L, [None] * L
        for l in range(L - 1, -1, -1):            # downward sweep
            a, b, z0, z1 = self.parts[l]
            gloc = np.zeros((z1 - z0 + 1, self.n), dtype=complex)
            gloc[a - z0:b - z0 + 1] = g[a:b + 1]
            if l != L - 1:
                up = w[l + 1]
                zu = self.parts[l + 1][2]
                w_above = up[b + 1 - zu]      # w^{l+1} on its first layer row
                w_at = up[b - zu]             # w^{l+1} on its lower ghost row
                gloc[b - z0] += -(self.block(l, b, b + 1) @ w_above)
                gloc[b + 1 - z0] += self.block(l, b + 1, b) @ w_at
            gl[l] = gloc
            w[l] = self.local_solve(l, gloc)
        v = np.zeros_like(g, dtype=complex)
        vl = [None] * L
        for l in range(L):                       # upward sweep
            a, b, z0, z1 = self.parts[l]
            if l != 0:
                dn = vl[l - 1]
                zd = self.parts[l - 1][2]
                v0 = dn[a - 1 - zd]                       # top layer row of l-1
                v1 = dn[a - zd] + w[l][a - z0]            # its upper ghost row + w^l
                gl[l][a - z0] += -(self.block(l, a, a - 1) @ v0)
                gl[l][a - 1 - z0] += self.block(l, a - 1, a) @ v1
            vl[l] = self.local_solve(l, gl[l])
            v[a:b + 1] = vl[l][a - z0:b - z0 + 1]
        return v


class BiDirectional:
    """Alg. 2: horizontal sweep, residual correction, vertical sweep."""

    def __init__(self, alpha, beta, m, omega, L, ext, shift_c=0.0, C=None):
        self.C = assemble_C(alpha, beta, m, omega) if C is None else C
        self.h = Sweep(alpha, beta, m, omega, L, ext, shift_c)
        aT = alpha.transpose(1, 0, 3, 2)
        bT = beta.transpose(1, 0, 3, 2)
        self.v = Sweep(aT, bT, m.T.copy(), omega, L, ext, shift_c)
        self.n = m.shape[0]

    def prec_h(self, g):
        return self.h.apply(g)

    def prec_v(self, g):
        return self.v.apply(g.T.copy()).T.copy()

    def apply(self, g: np.ndarray) -> np.ndarray:
        n = self.n
        u1 = self.prec_h(g)
        e = g - (self.C @ u1.reshape(-1)).reshape(n, n)
        u2 = self.prec_v(e)
        return u1 + u2
