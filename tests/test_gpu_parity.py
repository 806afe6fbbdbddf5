"""GPU parity: every step of the HIP path against the FP64 CPU oracle.

Inputs are seeded (ls_inputs); all calls go through the C ABI (via the thin
binding).  Tolerances are stated per test; they follow from FP64 rounding
(FFT ~ eps log P, GEMV/BCR ~ eps * cond) and, for everything downstream of
the stencils, from the stencil construction: the GPU forms the Gram matrix
M M^* (eigenvector error ~ eps ||M||^2 / gap ~ 1e-11) while the oracle takes
the SVD of M.
"""
import numpy as np
import pytest
import torch

from oracle import kernel, sparsify, slabs, solver
import ls_inputs as li
from gpu_helpers import dev, host, rel, banner

pytestmark = pytest.mark.gpu


def make_plan(n, f, m, **kw):
    from paper_1602_07652_amd import Plan
    omega = 2 * np.pi * f
    banner(f"plan n={n} f={f} opts={kw}")
    return Plan(n, 1.0 / n, omega, dev(m, torch.float64), **kw), omega


@pytest.mark.parametrize("n", [8, 37, 64, 1024])
def test_kernel_samples_and_spectrum(n):
    f = n / 10.0
    p, omega = make_plan(n, f, np.zeros((n, n)), precond=2)
    w_gpu = host(p.kernel_samples())
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    err = np.max(np.abs(w_gpu - W)) / np.max(np.abs(W))
    banner(f"kernel samples n={n} max rel err {err:.3e}")
    assert err < 1e-13
    # pointwise relative error on the off-diagonal samples
    assert np.max(np.abs(w_gpu - W) / np.abs(W)) < 1e-12
    S_gpu = host(p.spectrum())
    P = p.P
    Gh = kernel.circulant_spectrum(W, P) * omega**2 / P**2
    S = Gh[:P // 2 + 1, :P // 2 + 1]
    err = np.max(np.abs(S_gpu - S)) / np.max(np.abs(S))
    banner(f"spectrum n={n} P={P} max rel err {err:.3e}")
    assert err < 1e-12
    p.close()


@pytest.mark.parametrize("n,batch", [(8, 1), (37, 3), (64, 2), (100, 1), (129, 2), (256, 1), (300, 2),
                                     (1024, 2), (2048, 1)])
def test_apply_matches_oracle(n, batch):
    m, _ = li.gaussian_bumps_medium(n, seed=n)
    p, omega = make_plan(n, n / 10.0, m, precond=2, max_batch=batch)
    v = li.random_complex((batch, n, n), seed=100 + n)
    y = host(p.apply(dev(v)))
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    y_ref = kernel.apply_H(W, m, v, omega)
    e = rel(y, y_ref)
    banner(f"apply n={n} batch={batch} rel err {e:.3e}")
    assert e < 1e-13
    # in place, and the right-hand side
    vt = dev(v)
    p.apply(vt, out=vt)
    assert rel(host(vt), y_ref) < 1e-13
    uI = np.stack([li.plane_wave(n, omega, 0.3 * k) for k in range(batch)])
    f = host(p.rhs_from_incident(dev(uI)))
    e = rel(f, kernel.rhs_from_incident(W, m, uI, omega))
    banner(f"rhs n={n} rel err {e:.3e}")
    assert e < 1e-13
    p.close()


def test_apply_zero_medium_is_identity():
    n = 48
    p, _ = make_plan(n, 4.8, np.zeros((n, n)), precond=2)
    v = li.random_complex((n, n), 5)
    assert rel(host(p.apply(dev(v))), v) == 0.0
    p.close()


@pytest.mark.parametrize("n", [37, 64])
def test_stencils_and_sparse_operators(n):
    m = li.gaussian_disk_medium(n)
    p, omega = make_plan(n, n / 10.0, m, precond=2)
    al_g, be_g = p.stencils()
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    al, be, _ = sparsify.stencils(W, n)
    ea = np.max(np.abs(al_g - al))
    eb = np.max(np.abs(be_g - be)) / np.max(np.abs(be))
    banner(f"stencils n={n} alpha err {ea:.3e} beta rel err {eb:.3e}")
    assert ea < 1e-9 and eb < 1e-9
    r = li.random_complex((2, n, n), 7)
    Ar = host(p.stencil_A(dev(r)))
    assert rel(Ar, sparsify.apply_A(al, r)) < 1e-9
    C = sparsify.assemble_C(al, be, m, omega)
    Cv = host(p.stencil_C(dev(r)))
    Cv_ref = np.stack([(C @ r[k].reshape(-1)).reshape(n, n) for k in range(2)])
    e = rel(Cv, Cv_ref)
    banner(f"C v n={n} rel err {e:.3e}")
    assert e < 1e-9
    p.close()


SLAB_CASES = [(64, 6.0, 4, 10, 0.0, None), (100, 10.0, 3, 8, 1.0, 3), (130, 13.0, 4, 10, 0.0, 1)]


def oracle_problem(n, f, L, ext, shift, seed):
    omega = 2 * np.pi * f
    m = li.gaussian_disk_medium(n) if seed is None else li.gaussian_bumps_medium(n, seed)[0]
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    al, be, _ = sparsify.stencils(W, n)
    return m, omega, al, be


@pytest.mark.parametrize("n,f,L,ext,shift,seed", SLAB_CASES)
@pytest.mark.parametrize("level0", [0, 1])
def test_slab_solves(n, f, L, ext, shift, seed, level0):
    m, omega, al, be = oracle_problem(n, f, L, ext, shift, seed)
    p, _ = make_plan(n, f, m, slabs=L, ext=ext, shift_c=shift, level0=level0)
    assert p.info()["tridiagonal_level0"] == 1 - level0
    parts = slabs.layer_partition(n, L, ext)
    for orient in (0, 1):
        a_, b_ = (al, be) if orient == 0 else (al.transpose(1, 0, 3, 2), be.transpose(1, 0, 3, 2))
        mm = m if orient == 0 else m.T.copy()
        for l in range(L):
            assert p.slab_info(orient, l) == parts[l]
            Cl = slabs.assemble_slab(a_, b_, mm, omega, parts[l], ext, shift)
            q = parts[l][3] - parts[l][2] + 1
            b = li.random_complex((n, q), seed=10 * l + orient)      # frame [long][short]
            x = host(p.slab_solve(orient, l, dev(b)))
            import scipy.sparse.linalg as spla
            x_ref = spla.spsolve(Cl.tocsc(), b.T.reshape(-1)).reshape(q, n).T
            e = rel(x, x_ref)
            banner(f"slab n={n} orient={orient} l={l} q={q} rel err {e:.3e}")
            assert e < 1e-10
    p.close()


@pytest.mark.parametrize("n,f,L,ext,shift,seed", SLAB_CASES)
def test_sweeps_and_bidirectional(n, f, L, ext, shift, seed):
    m, omega, al, be = oracle_problem(n, f, L, ext, shift, seed)
    p, _ = make_plan(n, f, m, slabs=L, ext=ext, shift_c=shift)
    bd = slabs.BiDirectional(al, be, m, omega, L, ext, shift)
    g = li.random_complex((n, n), 3)
    vh = host(p.sweep(0, dev(g)))
    e0 = rel(vh, bd.prec_h(g))
    vv = host(p.sweep(1, dev(g)))
    e1 = rel(vv, bd.prec_v(g))
    vb = host(p.bidirectional(dev(g)))
    e2 = rel(vb, bd.apply(g))
    banner(f"sweeps n={n} L={L} H {e0:.3e} V {e1:.3e} BD {e2:.3e}")
    assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10
    p.close()


@pytest.mark.parametrize("level0", [0, 1])
@pytest.mark.parametrize("n,f,L,ext,shift,seed", SLAB_CASES + [(80, 8.0, 2, 8, 0.0, 7), (200, 20.0, 20, 4, 0.0, 5)])
def test_decoupled_sweep_matches_oracle(n, f, L, ext, shift, seed, level0):
    """Alg. 1 with the layers decoupled by trace-transfer maps (independent
    local solves, two chains of dense products for the traces, independent
    solves again) is the same linear operator as the sequential sweep: both
    orientations and Alg. 2 against the oracle's sequential sweeps.  The
    independent solves run as multi-slab launches over groups of like slabs:
    one group per layer (n = 130), two groups of two (n = 64), two layers
    only (n = 80: no chain step beyond the first, no upward chain), and at
    n = 200, L = 20 more like slabs than one launch takes (groups of 16, 2
    and 2; the per-layer launches in chunks of 16 and 4).  level0 0: the
    level-0 odd blocks as tridiagonal systems (the plan must have kept them),
    1: by their dense inverses."""
    from paper_1602_07652_amd import LS_SWEEP_DECOUPLED
    m, omega, al, be = oracle_problem(n, f, L, ext, shift, seed)
    p, _ = make_plan(n, f, m, slabs=L, ext=ext, shift_c=shift, sweep=LS_SWEEP_DECOUPLED, level0=level0)
    assert p.info()["tridiagonal_level0"] == 1 - level0
    bd = slabs.BiDirectional(al, be, m, omega, L, ext, shift)
    g = li.random_complex((n, n), 13)
    e0 = rel(host(p.sweep(0, dev(g))), bd.prec_h(g))
    e1 = rel(host(p.sweep(1, dev(g))), bd.prec_v(g))
    e2 = rel(host(p.bidirectional(dev(g))), bd.apply(g))
    banner(f"decoupled sweeps n={n} L={L} shift={shift}: H {e0:.3e} V {e1:.3e} BD {e2:.3e}")
    assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10
    p.close()


@pytest.mark.parametrize("level0", [0, 1])
@pytest.mark.parametrize("n,f,L,ext,shift,seed", [SLAB_CASES[1], (200, 20.0, 20, 4, 0.0, 5)])
def test_decoupled_sweep_fp32_plan(n, f, L, ext, shift, seed, level0):
    """The decoupled Alg. 2 of an FP32 plan against the FP64 oracle: at n =
    100, L = 3 the two boundary layers share a launch, at n = 200, L = 20
    the interior groups take 16 and 2 slabs, so level 1 runs through the
    tridiagonal level-0 blocks in FP32 (level0 0) or as dense products
    (level0 1)."""
    from paper_1602_07652_amd import LS_SWEEP_DECOUPLED, LS_FP32_REFINE
    m, omega, al, be = oracle_problem(n, f, L, ext, shift, seed)
    p, _ = make_plan(n, f, m, slabs=L, ext=ext, shift_c=shift, sweep=LS_SWEEP_DECOUPLED,
                     precision=LS_FP32_REFINE, level0=level0)
    assert p.info()["tridiagonal_level0"] == 1 - level0
    bd = slabs.BiDirectional(al, be, m, omega, L, ext, shift)
    g = li.random_complex((n, n), 14)
    e = rel(host(p.bidirectional(dev(g))), bd.apply(g))
    banner(f"decoupled sweeps FP32 n={n} L={L} level0={level0}: BD {e:.3e}")
    assert e < 5e-5
    p.close()


@pytest.mark.parametrize("fixed,B", [(2, 1), (1, 1), (1, 3)])
def test_precond_fixed_iterations(fixed, B):
    """Alg. 3 with a fixed number of inner iterations against the oracle's:
    two (the flexible GMRES loop) and one (its closed form on the device,
    z = (w^H g / w^H w) M g with w = C M g), one and three right-hand sides,
    the third a zero vector (z = 0)."""
    n, f, L = 64, 6.0, 4
    m = li.gaussian_disk_medium(n)
    p, omega = make_plan(n, f, m, slabs=L, ext=10, inner_fixed_iters=fixed, max_batch=B)
    P = solver.Problem(n, 1.0 / n, omega, m, slabs_L=L, ext=10, inner_fixed_iters=fixed)
    r = li.random_complex((B, n, n), 11)
    if B > 2:
        r[2] = 0.0
    z = host(p.precond_apply(dev(r)))
    for b in range(B):
        if not np.any(r[b]):
            assert not np.any(z[b])
            continue
        e = rel(z[b], P.precond_apply(r[b]))
        banner(f"precond fixed={fixed} rhs {b} rel err {e:.3e}")
        assert e < 1e-12
    p.close()


@pytest.mark.parametrize("inner", [{}, {"inner_fixed_iters": 1}])
def test_solve_c1_matches_dense_solution(inner):
    """The 64^2 workload against the dense solution of H u = f, with Alg. 3
    as printed (inner tolerance 1e-3) and with the inner solve relaxed to
    one iteration per outer iteration (Section 6); the oracle's own runs of
    both forms take 4 outer iterations."""
    cfg = li.config_inputs("c1_64_gauss_disk")
    n, omega, m = cfg["n"], cfg["omega"], cfg["m"]
    p, _ = make_plan(n, 6.0, m, slabs=4, ext=10, **inner)
    f = p.rhs_from_incident(dev(cfg["uI"]))
    u, info = p.solve(f, tol=1e-8)
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    f_ref = kernel.rhs_from_incident(W, m, cfg["uI"], omega)
    u_star = solver.dense_solve(W, m, omega, f_ref)
    e = rel(host(u), u_star)
    banner(f"solve c1 inner={inner} info={info[0]} rel err vs dense {e:.3e}")
    assert info[0]["converged"] == 1 and info[0]["relres_true"] < 1e-8
    assert e < 1e-6
    assert info[0]["outer_its"] <= 6
    if inner:
        assert info[0]["inner_its_total"] == info[0]["outer_its"]
    p.close()

def test_long_arnoldi_runs_match_dense_solutions():
    """Unpreconditioned inner GMRES (LS_PREC_NONE) runs well past 8 Arnoldi
    steps, so every solve goes through both Gram-Schmidt forms: the fused
    device form (up to 8 basis vectors) and the multi-dot / multi-axpy one
    beyond.  Three right-hand sides at once; each must reach the dense
    solution of H u = f (Section 2) to the accuracy its residual allows."""
    n, fq = 48, 6.0
    m = li.gaussian_disk_medium(n)
    p, omega = make_plan(n, fq, m, slabs=3, ext=10, precond=2, max_batch=3)
    uI = np.stack([li.plane_wave(n, omega, th) for th in (0.0, 1.0, 2.5)])
    f = p.rhs_from_incident(dev(uI))
    u, infos = p.solve(f, tol=1e-9)
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    uh = host(u)
    for b, info in enumerate(infos):
        f_ref = kernel.rhs_from_incident(W, m, uI[b], omega)
        e = rel(uh[b], solver.dense_solve(W, m, omega, f_ref))
        banner(f"long Arnoldi, wave {b}: {info}, rel err vs dense {e:.3e}")
        assert info["converged"] == 1 and info["relres_true"] < 1e-9
        assert info["inner_its_total"] > 8 * info["outer_its"]
        assert e < 1e-6
    p.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_solve_equals_single_solves(precision):
    """B right-hand sides solved together (lockstep Krylov, batched slab
    solves) give the same solutions as one at a time."""
    n, f, L = 96, 9.6, 3
    m, _ = li.gaussian_bumps_medium(n, seed=5)
    p, omega = make_plan(n, f, m, slabs=L, ext=8, max_batch=4, precision=precision)
    uI = np.stack([li.plane_wave(n, omega, 2 * np.pi * k / 4) for k in range(4)])
    fb = p.rhs_from_incident(dev(uI))
    ub, infos = p.solve(fb, tol=1e-9)
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    Gh = kernel.circulant_spectrum(W)
    for k in range(4):
        uk, ik = p.solve(fb[k].contiguous(), tol=1e-9)
        e = rel(host(ub[k]), host(uk))
        # and the oracle's FP64 residual of the batched solution
        fr = kernel.rhs_from_incident(W, m, uI[k], omega, Gh)
        res = np.linalg.norm(fr - kernel.apply_H(W, m, host(ub[k]), omega, Gh)) / np.linalg.norm(fr)
        banner(f"batched prec={precision} k={k} vs single {e:.3e} oracle residual {res:.3e} "
               f"info {infos[k]}")
        assert infos[k]["converged"] == 1 and res < 2e-9
        assert e < 1e-7
    p.close()


def test_batched_sweep_and_precond_match_oracle():
    n, f, L, ext = 100, 10.0, 3, 8
    m, omega, al, be = oracle_problem(n, f, L, ext, 0.0, 3)
    p, _ = make_plan(n, f, m, slabs=L, ext=ext, max_batch=3, inner_fixed_iters=2)
    P = solver.Problem(n, 1.0 / n, omega, m, slabs_L=L, ext=ext, inner_fixed_iters=2)
    r = li.random_complex((3, n, n), 21)
    z = host(p.precond_apply(dev(r)))
    for k in range(3):
        e = rel(z[k], P.precond_apply(r[k]))
        banner(f"batched precond k={k} rel err {e:.3e}")
        assert e < 1e-12
    p.close()


@pytest.fixture(scope="module")
def bench_shape():
    """The 1024^2 bench workload (8 bumps, omega = 2 pi 100, 16 layers,
    extension 10) with the oracle's stencils."""
    cfg = li.config_inputs("c2_1024_bumps")
    n, omega, m = cfg["n"], cfg["omega"], cfg["m"]
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    al, be, _ = sparsify.stencils(W, n)
    p, om = make_plan(n, omega / (2 * np.pi), m, slabs=16, ext=10, max_batch=8)
    assert abs(om - omega) <= 1e-12 * omega
    yield n, omega, m, al, be, p
    p.close()


@pytest.mark.parametrize("orient,l", [(0, 1), (1, 1), (0, 0), (1, 15)])
def test_slab_solve_at_bench_shape(bench_shape, orient, l):
    """Full-size slab solves (n = 1024, q = 74..84) in the launch
    configuration the benchmark times, against SuperLU on the oracle's slab
    matrix."""
    import scipy.sparse.linalg as spla
    n, omega, m, al, be, p = bench_shape
    a_, b_ = (al, be) if orient == 0 else (al.transpose(1, 0, 3, 2), be.transpose(1, 0, 3, 2))
    mm = m if orient == 0 else m.T.copy()
    parts = slabs.layer_partition(n, 16, 10)
    assert p.slab_info(orient, l) == parts[l]
    Cl = slabs.assemble_slab(a_, b_, mm, omega, parts[l], 10, 0.0)
    q = parts[l][3] - parts[l][2] + 1
    b = li.random_complex((n, q), seed=100 + 10 * l + orient)
    x = host(p.slab_solve(orient, l, dev(b)))
    x_ref = spla.spsolve(Cl.tocsc(), b.T.reshape(-1)).reshape(q, n).T
    e = rel(x, x_ref)
    banner(f"bench-shape slab orient={orient} l={l} q={q} rel err {e:.3e}")
    # both sides carry ~ eps * cond(C^l) at q = 84 (measured 2.8e-11 - 3.7e-11)
    assert e < 4e-10


def test_zero_right_hand_side_gives_zero():
    n = 48
    m = li.gaussian_disk_medium(n)
    p, _ = make_plan(n, 4.8, m, slabs=2, ext=6, max_batch=2)
    f = torch.zeros((2, n, n), dtype=torch.complex128, device="cuda")
    f[1] = dev(li.random_complex((n, n), 3))
    u, info = p.solve(f, tol=1e-8)
    banner(f"zero rhs: {info[0]} / nonzero: {info[1]}")
    assert torch.count_nonzero(u[0]).item() == 0 and info[0]["converged"] == 1
    assert info[1]["converged"] == 1
    p.close()


def test_single_slab_is_the_exact_local_solve():
    """L = 1: the one slab is the whole grid, C^1 = C, so Alg. 2 solves the
    sparsified system exactly and the inner GMRES stops after one iteration."""
    n = 64
    m = li.gaussian_disk_medium(n)
    p, omega = make_plan(n, 6.0, m, slabs=1, ext=10)
    P = solver.Problem(n, 1.0 / n, omega, m, slabs_L=1, ext=10, precond="exact")
    r = li.random_complex((n, n), 4)
    z = host(p.precond_apply(dev(r)))
    e = rel(z, P.precond_apply(r))
    banner(f"L=1 precond vs exact C^-1 A r: {e:.3e}")
    assert e < 1e-9
    p.close()


def test_batch_larger_than_max_batch_is_chunked():
    n = 64
    m, _ = li.gaussian_bumps_medium(n, seed=8)
    p, omega = make_plan(n, 6.4, m, slabs=2, ext=6, max_batch=2)
    uI = np.stack([li.plane_wave(n, omega, 0.5 * k) for k in range(5)])
    # ls_apply / ls_rhs_from_incident take at most max_batch vectors; ls_solve
    # takes any batch and works through it max_batch at a time
    f = torch.cat([p.rhs_from_incident(dev(uI[k:k + 2])) for k in range(0, 5, 2)])
    u, infos = p.solve(f, tol=1e-9)
    for k in range(5):
        uk, _ = p.solve(f[k].contiguous(), tol=1e-9)
        e = rel(host(u[k]), host(uk))
        banner(f"chunked batch k={k}: vs single {e:.2e} info {infos[k]}")
        assert infos[k]["converged"] == 1 and e < 1e-7
    p.close()


def test_too_thick_layer_is_refused():
    from paper_1602_07652_amd import LSError
    n = 200
    with pytest.raises(LSError) as ei:
        make_plan(n, 20.0, np.zeros((n, n)), slabs=2, ext=10)     # q = 120 > 96
    banner(f"refused: {ei.value}")
    assert "96" in str(ei.value)


def test_decoupled_sweep_at_bench_shape(bench_shape):
    """1024^2, 16 layers: the decoupled sweep against the sequential one of
    the bench plan, and the full bench solve with it (same iterations, same
    solution to the tolerance)."""
    from paper_1602_07652_amd import LS_SWEEP_DECOUPLED
    n, omega, m, al, be, p = bench_shape
    pd, _ = make_plan(n, omega / (2 * np.pi), m, slabs=16, ext=10, sweep=LS_SWEEP_DECOUPLED)
    g = dev(li.random_complex((n, n), 71))
    for orient in (0, 1):
        e = rel(host(pd.sweep(orient, g)), host(p.sweep(orient, g)))
        banner(f"bench-shape decoupled vs sequential sweep orient={orient}: {e:.3e}")
        assert e < 1e-10
    cfg = li.config_inputs("c2_1024_bumps")
    f = p.rhs_from_incident(dev(cfg["uI"]))
    us, i_s = p.solve(f, tol=1e-8)
    ud, i_d = pd.solve(f, tol=1e-8)
    e = rel(host(ud), host(us))
    banner(f"bench solve sequential {i_s[0]} decoupled {i_d[0]}: {e:.3e}")
    assert i_d[0]["converged"] == 1 and i_d[0]["outer_its"] == i_s[0]["outer_its"]
    assert e < 1e-8
    pd.close()


def test_apply_properties_at_bench_shape(bench_shape):
    """Properties of H that hold at any size, checked on the 1024^2 bench
    plan: linearity; D H complex symmetric (w is even, so
    v^T D H w = w^T D H v with D = diag(m)); f(u_I) = -(H - I) u_I; and
    outputs sampled against the O(N) direct sum (H v)_k = v_k +
    w^2 sum_p w_{k-p} m_p v_p."""
    n, omega, m, al, be, p = bench_shape
    v = li.random_complex((n, n), 61)
    w = li.random_complex((n, n), 62)
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    Hv = host(p.apply(dev(v)))
    Hw = host(p.apply(dev(w)))
    Hl = host(p.apply(dev(a * v + b * w)))
    e_lin = rel(Hl, a * Hv + b * Hw)
    lhs, rhs = np.sum(v * m * Hw), np.sum(w * m * Hv)
    e_sym = abs(lhs - rhs) / abs(lhs)
    f = host(p.rhs_from_incident(dev(v)))
    e_rhs = rel(f, -(Hv - v))
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    rng = np.random.default_rng(63)
    pts = rng.integers(0, n, size=(24, 2))
    mv = m * v
    worst = 0.0
    for j, i in pts:
        # W[n-1 + dj, n-1 + di] = w at offset (dj, di) = (j - jp, i - ip)
        Wk = W[n - 1 + j - np.arange(n)[:, None], n - 1 + i - np.arange(n)[None, :]]
        direct = v[j, i] + omega**2 * np.sum(Wk * mv)
        worst = max(worst, abs(Hv[j, i] - direct) / np.max(np.abs(Hv)))
    banner(f"bench-shape H: linearity {e_lin:.2e}, D H symmetry {e_sym:.2e}, rhs identity {e_rhs:.2e}, "
           f"direct-sum samples {worst:.2e}")
    assert e_lin < 1e-14 and e_sym < 1e-12 and e_rhs < 1e-14 and worst < 1e-13


def test_batch8_apply_at_bench_shape(bench_shape):
    """ls_apply on 8 right-hand sides at 1024^2, the batch the benchmark
    times (run in chunks whose intermediates stay cache-resident): every
    right-hand side equals its own one-right-hand-side apply bit for bit,
    twice in a row (the chunks' work areas and streams are reused), and
    sampled outputs of two of them match the O(N) direct sum of the oracle's
    kernel samples."""
    n, omega, m, al, be, p = bench_shape
    B = 8
    v = li.random_complex((B, n, n), 71)
    vd = dev(v)
    y1 = host(p.apply(vd))
    y2 = host(p.apply(vd))
    assert np.array_equal(y1, y2)
    for k in range(B):
        yk = host(p.apply(dev(v[k:k + 1])))[0]
        assert np.array_equal(yk, y1[k]), f"right-hand side {k} differs from its single apply"
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    rng = np.random.default_rng(72)
    worst = 0.0
    for k in (0, B - 1):
        mv = m * v[k]
        for j, i in rng.integers(0, n, size=(8, 2)):
            Wk = W[n - 1 + j - np.arange(n)[:, None], n - 1 + i - np.arange(n)[None, :]]
            direct = v[k, j, i] + omega**2 * np.sum(Wk * mv)
            worst = max(worst, abs(y1[k, j, i] - direct) / np.max(np.abs(y1[k])))
    banner(f"batch-8 apply at 1024^2: equal to single applies, direct-sum samples {worst:.2e}")
    assert worst < 1e-13
