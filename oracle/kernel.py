"""Green's function samples and the discrete Lippmann-Schwinger operator.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 1, eq. (Greens_function): G(x) = -(i/4) H_0^(1)(omega |x|),
the free-space Green's function of Delta + omega^2, and eq.
(Lippmann-Schwinger): u + omega^2 G*(m u) = -omega^2 G*(m u_I).

Paper, Section 2: uniform grid x_{i,j} = (h i, h j); the convolution is
discretised by the trapezoidal rule with only the diagonal weight modified,
giving order h^4 log h; H = I + omega^2 G D, f = -omega^2 G D u_I, and G is
applied through a Toeplitz (circulant) embedding and the FFT.

Reading (the paper names the rule but not the weight): the off-diagonal
weights are h^2 G(h|q|).  The diagonal weight is the integral of G against a
smooth density minus the punctured lattice sum, i.e. the regular part of G at
0, -(i/4) + (ln(omega/2) + gamma)/(2 pi), plus the lattice correction of the
logarithmic singularity (1/(2 pi)) ln r, which is (ln h + c_L)/(2 pi) with
c_L = ln(2 sqrt(pi) / Gamma(1/4)^2) (half the derivative at 0 of the Epstein
zeta function of Z^2).  c_L is pinned against a lattice sum and the whole
rule against the Gaussian-source identity G*((Delta+omega^2) psi) = psi, which
converges at O(h^4) only with this weight.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.special as sp

EULER_GAMMA = float(np.euler_gamma)
C_L = float(np.log(2.0 * np.sqrt(np.pi) / sp.gamma(0.25) ** 2))


def green(r, omega):
    """G(r) = -(i/4) H_0^(1)(omega r), r > 0 (Section 1)."""
    return -0.25j * sp.hankel1(0, omega * np.asarray(r, dtype=float))


def diagonal_weight(h: float, omega: float) -> complex:
    """Modified trapezoidal weight at q = 0 (Section 2; reading above)."""
    return h * h * (-0.25j + (np.log(omega * h / 2.0) + EULER_GAMMA + C_L) / (2.0 * np.pi))


def kernel_samples(n: int, h: float, omega: float) -> np.ndarray:
    """Quadrature weights w_q for q in [-(n-1), n-1]^2.

    Returns W with W[qz + n - 1, qx + n - 1] = w_(qx, qz):
    h^2 G(h |q|) for q != 0 and the diagonal weight at q = 0.
    The Hankel argument is evaluated as (omega*h) * sqrt(qx^2 + qz^2).
    """
    q = np.arange(-(n - 1), n, dtype=float)
    QZ, QX = np.meshgrid(q, q, indexing="ij")
    rho = np.sqrt(QX * QX + QZ * QZ)
    W = np.empty(rho.shape, dtype=complex)
    nz = rho > 0
    W[nz] = h * h * (-0.25j) * sp.hankel1(0, (omega * h) * rho[nz])
    W[n - 1, n - 1] = diagonal_weight(h, omega)
    return W


def apply_G_direct(W: np.ndarray, u: np.ndarray) -> np.ndarray:
    """(G u)_k = sum_p w_{k-p} u_p by the O(N^2) direct sum (small n only)."""
    n = u.shape[-1]
    out = np.zeros(u.shape, dtype=complex)
    for j in range(n):
        for i in range(n):
            # w_{(i - i', j - j')} for i', j' = 0..n-1
            blk = W[j:j + n, i:i + n][::-1, ::-1]
            out[..., j, i] = np.sum(blk * u, axis=(-2, -1))
    return out


def circulant_spectrum(W: np.ndarray, P: int | None = None) -> np.ndarray:
    """FFT of the P x P circulant embedding of w (Section 2, Toeplitz embed).

    Entries with |qx| or |qz| > n-1 are zero; any P >= 2n-1 gives the same
    cropped linear convolution.
    """
    n = (W.shape[0] + 1) // 2
    if P is None:
        P = 2 * n
    assert P >= 2 * n - 1
    c = np.zeros((P, P), dtype=complex)
    idx = np.arange(-(n - 1), n) % P
    c[np.ix_(idx, idx)] = W
    return scipy.fft.fft2(c, workers=-1)


def apply_G_fft(W: np.ndarray, u: np.ndarray, Ghat: np.ndarray | None = None) -> np.ndarray:
    """G u by zero padding to P = 2n and the FFT (Section 2, Section 4.2)."""
    n = u.shape[-1]
    if Ghat is None:
        Ghat = circulant_spectrum(W)
    P = Ghat.shape[0]
    U = scipy.fft.fft2(u, s=(P, P), axes=(-2, -1), workers=-1)
    return scipy.fft.ifft2(Ghat * U, axes=(-2, -1), workers=-1)[..., :n, :n]


def apply_H(W, m, v, omega, Ghat=None, direct=False):
    """H v = v + omega^2 G (m v)  (Section 2, eq. discrete_Lipmann-Schwinger)."""
    mv = m * v
    Gmv = apply_G_direct(W, mv) if direct else apply_G_fft(W, mv, Ghat)
    return v + omega**2 * Gmv


def rhs_from_incident(W, m, uI, omega, Ghat=None, direct=False):
    """f = -omega^2 G D u_I  (Section 2)."""
    mu = m * uI
    Gmu = apply_G_direct(W, mu) if direct else apply_G_fft(W, mu, Ghat)
    return -omega**2 * Gmu


def dense_G(W: np.ndarray) -> np.ndarray:
    """Dense N x N matrix of G in the row-by-row ordering k = j*n + i."""
    n = (W.shape[0] + 1) // 2
    jj, ii = np.divmod(np.arange(n * n), n)
    dz = jj[:, None] - jj[None, :]
    dx = ii[:, None] - ii[None, :]
    return W[dz + n - 1, dx + n - 1]


def dense_H(W, m, omega):
    """Dense H = I + omega^2 G D (small n only)."""
    n = m.shape[0]
    return np.eye(n * n, dtype=complex) + omega**2 * dense_G(W) * m.reshape(-1)[None, :]
