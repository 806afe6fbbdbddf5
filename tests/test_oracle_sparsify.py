"""Pins of the oracle's sparsifying stencils and C (Section 2 of the paper)."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import kernel, sparsify, solver
import ls_inputs as li


def setup_small(n=16, f=1.6, seed=None):
    omega = 2 * np.pi * f
    W = kernel.kernel_samples(n, 1 / n, omega)
    alpha, beta, _ = sparsify.stencils(W, n)
    m = li.gaussian_disk_medium(n) if seed is None else li.gaussian_bumps_medium(n, seed)[0]
    return n, omega, W, alpha, beta, m


def test_alpha_is_the_minimiser():
    n, omega, W, alpha, beta, m = setup_small()
    for tz in range(3):
        for tx in range(3):
            M, offs = sparsify.stencil_matrix(W, n, tz, tx)
            a = np.array([alpha[tz, tx, dz + 1, dx + 1] for dz, dx in offs])
            assert abs(np.linalg.norm(a) - 1) < 1e-14
            val = np.linalg.norm(a @ M)
            # independent route: smallest eigenvalue of M M^*
            lam = np.linalg.eigvalsh(M @ M.conj().T)
            assert abs(val - np.sqrt(max(lam[0], 0))) < 1e-9 * np.sqrt(lam[-1])
            assert val < 2e-2 * np.sqrt(lam[-1])
            rng = np.random.default_rng(tz * 3 + tx)
            for _ in range(5):
                b = a + 0.05 * (rng.standard_normal(a.size) + 1j * rng.standard_normal(a.size))
                b /= np.linalg.norm(b)
                assert np.linalg.norm(b @ M) > val
            # phase convention
            c = alpha[tz, tx, 1, 1]
            assert abs(c.imag) < 1e-15 and c.real > 0


def test_C_equals_AH_on_the_pattern():
    """C = A H restricted to A's pattern, by a dense product (Section 2)."""
    n, omega, W, alpha, beta, m = setup_small()
    C = sparsify.assemble_C(alpha, beta, m, omega).toarray()
    AH = sparsify.dense_A(alpha, n) @ kernel.dense_H(W, m, omega)
    pat = C != 0
    assert pat.sum() == (3 * n - 2) ** 2   # 9-point pattern on the grid
    assert np.max(np.abs(AH[pat] - C[pat])) < 1e-13 * np.max(np.abs(C))
    # the product is approximately sparse: what is dropped is small
    assert np.max(np.abs(AH[~pat])) < 1e-3 * np.max(np.abs(C))


def test_interior_stencil_has_lattice_symmetry():
    n = 15   # odd: the representative point is the exact centre
    omega = 2 * np.pi * 1.5
    W = kernel.kernel_samples(n, 1 / n, omega)
    alpha, _, _ = sparsify.stencils(W, n)
    a = alpha[1, 1]
    for b in (a[::-1, :], a[:, ::-1], a.T):
        assert np.max(np.abs(a - b)) < 1e-12
    # edge stencils map onto each other under the grid symmetries
    assert np.max(np.abs(alpha[0, 1] - alpha[2, 1][::-1, :])) < 1e-12
    assert np.max(np.abs(alpha[1, 0] - alpha[0, 1].T)) < 1e-12


def test_stencil_phase_does_not_change_the_preconditioner():
    """Multiplying the rows of one stencil type of A by e^{i t} scales the
    same rows of C, so C^{-1} A r is unchanged."""
    n, omega, W, alpha, beta, m = setup_small(n=20, f=2.0, seed=4)
    r = li.random_complex((n, n), 7)

    def prec(al, be):
        C = sparsify.assemble_C(al, be, m, omega)
        return spla.spsolve(C.tocsc(), sparsify.apply_A(al, r).reshape(-1))

    x0 = prec(alpha, beta)
    a2, b2 = alpha.copy(), beta.copy()
    for t, (tz, tx) in zip((0.7, -2.1, 1.3), ((1, 1), (0, 1), (2, 2))):
        a2[tz, tx] *= np.exp(1j * t)
        b2[tz, tx] *= np.exp(1j * t)
    x1 = prec(a2, b2)
    assert np.max(np.abs(x1 - x0)) < 1e-11 * np.max(np.abs(x0))


def test_exact_sparsified_preconditioner_cuts_outer_iterations():
    cfg = li.config_inputs("c1_64_gauss_disk")
    P = solver.Problem(cfg["n"], cfg["h"], cfg["omega"], cfg["m"], precond="exact")
    f = P.rhs(cfg["uI"])
    _, info_p = P.solve(f, tol=1e-8)
    _, info_u = P.solve(f, tol=1e-8, precondition=False)
    assert info_p["iters"] <= 5 < info_u["iters"]
    assert info_p["relres_true"] < 1e-8
