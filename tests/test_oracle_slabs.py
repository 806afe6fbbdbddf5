"""Pins of the oracle's layered decomposition and sweeps (Section 3)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import kernel, sparsify, slabs, krylov, solver
import ls_inputs as li


def test_partition_and_cutoff():
    parts = slabs.layer_partition(50, 4, 10)
    assert [b - a + 1 for a, b, _, _ in parts] == [13, 13, 12, 12]
    assert parts[0][2] == 0 and parts[-1][3] == 49
    assert parts[1] == (13, 25, 3, 35)
    a, b, e = 20, 30, 10
    assert slabs.cutoff(a - 1, a, b, e) == 1.0 and slabs.cutoff(b + 1, a, b, e) == 1.0
    assert slabs.cutoff(a - e, a, b, e) == 0.0 and slabs.cutoff(b + e, a, b, e) == 0.0
    vals = [slabs.cutoff(b + d, a, b, e) for d in range(1, e + 1)]
    assert all(x >= y for x, y in zip(vals, vals[1:]))


def grf_case(n=48, L=3, ext=6, seed=3):
    omega = 2 * np.pi * n / 10
    m, _ = li.gaussian_bumps_medium(n, seed=seed)
    W = kernel.kernel_samples(n, 1 / n, omega)
    al, be, _ = sparsify.stencils(W, n)
    return n, omega, m, al, be


@pytest.mark.parametrize("shift_c", [0.0, 1.5])
def test_grf_is_exact_with_global_traces(shift_c):
    """eq. (pde_GRF_real): with the traces of v = C^{-1} g on both sides the
    local solve gives v on the layer and 0 on the extension."""
    n, omega, m, al, be = grf_case()
    C = sparsify.assemble_C(al, be, m, omega)
    g = li.random_complex((n, n), 1)
    v = spla.spsolve(C.tocsc(), g.reshape(-1)).reshape(n, n)
    sw = slabs.Sweep(al, be, m, omega, 3, 6, shift_c)
    for l, (a, b, z0, z1) in enumerate(sw.parts):
        gl = np.zeros((z1 - z0 + 1, n), complex)
        gl[a - z0:b - z0 + 1] = g[a:b + 1]
        if b + 1 <= n - 1:
            gl[b - z0] += -(sw.block(l, b, b + 1) @ v[b + 1])
            gl[b + 1 - z0] += sw.block(l, b + 1, b) @ v[b]
        if a - 1 >= 0:
            gl[a - z0] += -(sw.block(l, a, a - 1) @ v[a - 1])
            gl[a - 1 - z0] += sw.block(l, a - 1, a) @ v[a]
        w = sw.local_solve(l, gl)
        expect = np.zeros_like(w)
        expect[a - z0:b - z0 + 1] = v[a:b + 1]
        assert np.max(np.abs(w - expect)) < 1e-12 * np.max(np.abs(v))


def test_compatibility_local_rows_equal_global_rows():
    n, omega, m, al, be = grf_case()
    C = sparsify.assemble_C(al, be, m, omega).tocsr()
    sw = slabs.Sweep(al, be, m, omega, 3, 6, shift_c=2.0)
    for l, (a, b, z0, z1) in enumerate(sw.parts):
        Cl = sw.mats[l]
        for j in range(a, b + 1):
            loc = Cl[(j - z0) * n:(j - z0 + 1) * n].toarray()
            glob = C[j * n:(j + 1) * n].toarray()[:, z0 * n:(z1 + 1) * n]
            assert np.max(np.abs(loc - glob)) < 1e-14 * np.max(np.abs(glob))


def test_single_layer_is_exact():
    n, omega, m, al, be = grf_case(n=32)
    bd = slabs.BiDirectional(al, be, m, omega, 1, 10)
    g = li.random_complex((n, n), 5)
    v = bd.apply(g)
    Cv = (bd.C @ v.reshape(-1)).reshape(n, n)
    assert np.max(np.abs(Cv - g)) < 1e-11 * np.max(np.abs(g))
    _, info = krylov.gmres_right(lambda x: (bd.C @ x.reshape(-1)).reshape(n, n), bd.apply, g, 1e-3, 10)
    assert info["iters"] == 1


def test_sweeps_are_linear_and_vertical_is_transposed_horizontal():
    n, omega, m, al, be = grf_case(n=40, L=3)
    bd = slabs.BiDirectional(al, be, m, omega, 3, 6)
    x, y = li.random_complex((n, n), 1), li.random_complex((n, n), 2)
    a, b = 1.5 - 0.2j, -0.7 + 2j
    lhs = bd.apply(a * x + b * y)
    rhs = a * bd.apply(x) + b * bd.apply(y)
    assert np.max(np.abs(lhs - rhs)) < 1e-11 * np.max(np.abs(lhs))
    # the vertical sweep on m equals the horizontal sweep on the transposed problem
    bdT = slabs.BiDirectional(al.transpose(1, 0, 3, 2), be.transpose(1, 0, 3, 2), m.T.copy(), omega, 3, 6)
    assert np.max(np.abs(bd.prec_v(x) - bdT.prec_h(x.T.copy()).T)) < 1e-12 * np.max(np.abs(bd.prec_v(x)))


@pytest.mark.slow
def test_alg1_reading_converges_fast_and_bidirectional_faster():
    """Iteration counts for C v = A u_I at 256^2, L = 4, tol 1e-6 (Section
    5.1 setting).  The paper's Table 2 has PT 3.6-12.6, BD 2.7-5.3."""
    n = 256
    omega = 2 * np.pi * 25.6
    m, _ = li.gaussian_bumps_medium(n, seed=1)
    P = solver.Problem(n, 1 / n, omega, m, slabs_L=4, ext=10)
    g = P.A(li.plane_wave(n, omega, 0.3))
    _, i1 = krylov.gmres_right(P.Cmul, P.bd.prec_h, g, 1e-6, 100)
    _, i2 = krylov.gmres_right(P.Cmul, P.bd.apply, g, 1e-6, 100)
    assert i1["iters"] <= 12
    assert i2["iters"] <= min(i1["iters"], 5)
