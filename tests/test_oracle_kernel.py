"""Pins of the oracle's quadrature and operator H (Sections 1-2 of the paper).

Each test checks the oracle against something other than itself: a closed
form, a lattice sum, a convergence order, brute force or an invariant.
"""
import numpy as np
import pytest

from oracle import kernel
import ls_inputs as li


def lattice_constant_estimate(sigma):
    # int ln|x| phi - sum'_{p != 0} ln|p| phi(p), phi = exp(-|x|^2 / (2 sigma^2))
    R = int(12 * sigma)
    p = np.arange(-R, R + 1)
    PZ, PX = np.meshgrid(p, p, indexing="ij")
    rho = np.sqrt(PX**2 + PZ**2)
    phi = np.exp(-rho**2 / (2 * sigma * sigma))
    nz = rho > 0
    s = np.sum(np.log(rho[nz]) * phi[nz])
    integral = np.pi * sigma**2 * (np.log(2 * sigma**2) - np.euler_gamma)  # closed form
    return integral - s


def test_lattice_constant_matches_lattice_sum():
    e20 = lattice_constant_estimate(20.0) - kernel.C_L
    e40 = lattice_constant_estimate(40.0) - kernel.C_L
    assert abs(e40) < 6e-5
    # O(sigma^-2) approach: the error drops by ~4 when sigma doubles
    assert 3.0 < e20 / e40 < 5.0


def test_diagonal_weight_is_regular_part_of_G():
    # G(r) - ln(r)/(2 pi) -> -(i/4) + (ln(omega/2) + gamma)/(2 pi) as r -> 0
    omega, h = 7.0, 0.01
    r = 1e-7
    reg = kernel.green(r, omega) - np.log(r) / (2 * np.pi)
    w0 = kernel.diagonal_weight(h, omega) / h**2 - (np.log(h) + kernel.C_L) / (2 * np.pi)
    assert abs(reg - w0) < 1e-9


def gaussian_source_error(n, omega=2 * np.pi * 4, s=0.05, drop_correction=False):
    h = 1.0 / n
    W = kernel.kernel_samples(n, h, omega)
    if drop_correction:
        W[n - 1, n - 1] = h * h * (-0.25j + (np.log(omega * h / 2) + kernel.EULER_GAMMA) / (2 * np.pi))
    X, Z = li.grid_coords(n)
    r2 = (X - 0.5) ** 2 + (Z - 0.5) ** 2
    psi = np.exp(-r2 / (2 * s * s))
    lap_plus = psi * (r2 / s**4 - 2 / s**2 + omega**2)      # (Delta + omega^2) psi
    return np.max(np.abs(kernel.apply_G_fft(W, lap_plus) - psi))


def test_gaussian_source_identity_fourth_order():
    """G * ((Delta + omega^2) psi) = psi: O(h^4 log h) with the corrected weight."""
    e64, e128 = gaussian_source_error(64), gaussian_source_error(128)
    assert e128 < 3e-5
    assert e64 / e128 > 12.0
    # without the lattice correction the rule is only second order
    d64, d128 = gaussian_source_error(64, drop_correction=True), gaussian_source_error(128, drop_correction=True)
    assert d64 / d128 < 5.0 and d128 > 1e-3


@pytest.mark.parametrize("n", [9, 14])
def test_fft_convolution_equals_direct_sum(n):
    h, omega = 1.0 / n, 2 * np.pi * 1.3
    W = kernel.kernel_samples(n, h, omega)
    rng = np.random.default_rng(n)
    m = rng.uniform(-0.3, 0.3, (n, n))
    v = li.random_complex((2, n, n), seed=n)
    a = kernel.apply_H(W, m, v, omega, direct=True)
    b = kernel.apply_H(W, m, v, omega)
    assert np.max(np.abs(a - b)) / np.max(np.abs(a)) < 1e-13
    # and the dense matrix agrees with the direct sum
    H = kernel.dense_H(W, m, omega)
    c = (H @ v[0].reshape(-1)).reshape(n, n)
    assert np.max(np.abs(a[0] - c)) / np.max(np.abs(c)) < 1e-13


def test_zero_medium_is_identity():
    n, omega = 16, 2 * np.pi * 1.6
    W = kernel.kernel_samples(n, 1 / n, omega)
    v = li.random_complex((n, n), 3)
    m = np.zeros((n, n))
    assert np.array_equal(kernel.apply_H(W, m, v, omega), v)
    assert np.all(kernel.rhs_from_incident(W, m, li.plane_wave(n, omega, 0.2), omega) == 0)


def test_DH_is_complex_symmetric_and_H_linear():
    n, omega = 12, 2 * np.pi * 1.2
    W = kernel.kernel_samples(n, 1 / n, omega)
    m = li.gaussian_disk_medium(n)
    H = kernel.dense_H(W, m, omega)
    DH = m.reshape(-1)[:, None] * H
    assert np.max(np.abs(DH - DH.T)) < 1e-15 * np.max(np.abs(DH)) * 10
    x, y = li.random_complex((n, n), 1), li.random_complex((n, n), 2)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    lhs = kernel.apply_H(W, m, a * x + b * y, omega)
    rhs = a * kernel.apply_H(W, m, x, omega) + b * kernel.apply_H(W, m, y, omega)
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(lhs))


def test_kernel_samples_even_and_match_green():
    n, h, omega = 10, 0.1, 9.0
    W = kernel.kernel_samples(n, h, omega)
    assert np.array_equal(W, W[::-1, :]) and np.array_equal(W, W[:, ::-1]) and np.array_equal(W, W.T)
    # one off-diagonal sample against the Green's function directly
    assert abs(W[n - 1 + 2, n - 1 + 3] - h * h * kernel.green(h * np.sqrt(13.0), omega)) < 1e-17
