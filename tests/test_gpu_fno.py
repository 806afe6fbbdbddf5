"""GPU parity of the learned preconditioner (bf16 MFMA network) against the
FP64 oracle in oracle/fno.py, and its use inside the solver.

Tolerances.  The MFMA products round both operands to bf16 (8 significant
bits, unit roundoff u = 2^-9 with round-to-nearest) and accumulate in FP32.
A product therefore carries a relative error of about 2u = 4e-3 per
operand pair; the network chains 4 spectral layers of 4 products each plus
lift and projection, so output errors of order sqrt(16) * 2u ~ 1.6e-2
relative (times the conditioning of the layer maps) are expected.  Outputs
and gradients are compared in relative L2 norm at 4e-2; the GEMM utility
itself is exact on bf16-representable integers and compared bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import fno as ofno, kernel
import ls_inputs as li
from gpu_helpers import dev, host, rel, banner

pytestmark = pytest.mark.gpu
TOL = 4e-2


def small_ints(shape, seed, lo=-8, hi=8):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=shape).astype(np.float32) * 0.25


@pytest.mark.parametrize("M,N,K,batch,ta,tb", [
    (37, 70, 45, 1, False, False),      # ragged tiles, 64x64 shape
    (16, 300, 64, 2, False, True),      # M <= 16 shape, transposed B
    (30, 500, 32, 3, True, False),      # 32 x 128 shape, transposed A
    (25, 20, 96, 2, False, False),      # 32 x 32 shape
    (200, 12, 64, 2, True, True),       # 64 x 16 shape
    (300, 30, 128, 1, False, False),    # 128 x 32 shape
    (64, 32, 5000, 1, False, False),    # split K with atomics
    (80, 30, 40, 2, False, False),      # 64 x 32 shape
])
def test_bf16_gemm_exact_on_representable_inputs(M, N, K, batch, ta, tb):
    from paper_1602_07652_amd import bf16_gemm
    A = small_ints((batch, M, K), 1)
    B = small_ints((batch, K, N), 2)
    C0 = small_ints((batch, M, N), 3)
    Ad = torch.from_numpy(np.ascontiguousarray(A.transpose(0, 2, 1) if ta else A)).cuda()
    Bd = torch.from_numpy(np.ascontiguousarray(B.transpose(0, 2, 1) if tb else B)).cuda()
    Cd = torch.from_numpy(C0.copy()).cuda()
    sa = (1, M, M * K) if ta else (K, 1, M * K)
    sb = (1, K, K * N) if tb else (N, 1, K * N)
    banner(f"gemm M={M} N={N} K={K} batch={batch} ta={ta} tb={tb}")
    bf16_gemm(Ad, Bd, Cd, M, N, K, batch, sa, sb, (N, 1, M * N), alpha=0.5, beta=2.0)
    torch.cuda.synchronize()
    ref = 0.5 * np.einsum("bmk,bkn->bmn", A.astype(np.float64), B.astype(np.float64)) + 2.0 * C0
    assert np.array_equal(Cd.cpu().numpy().astype(np.float64), ref)


def _params(seed=7, last_scale=30.0):
    vec = li.fno_initial_parameters(seed)
    p = ofno.unflatten(vec)
    p["proj2_w"] = p["proj2_w"] * last_scale      # a visible output for the comparison
    p["proj2_b"] = p["proj2_b"] * last_scale
    flat = ofno.flatten(p).astype(np.float32)
    return ofno.unflatten(flat.astype(np.float64)), torch.from_numpy(flat).cuda()


def _inputs(n, S, seed):
    ms, uIs, rs = [], [], []
    for k in range(S):
        m, th = li.fno_sample_recipe(seed + k, n)
        ms.append(m)
        uIs.append(li.plane_wave(n, 2 * np.pi * n / 10, th))
        rs.append(li.random_complex((n, n), seed + 100 + k))
    return np.stack(ms), np.stack(uIs), np.stack(rs)


def _make_x(ms, uIs, rs):
    xs, ss = zip(*[ofno.make_inputs(m, u, r) for m, u, r in zip(ms, uIs, rs)])
    return np.stack(xs), np.array(ss)


@pytest.fixture(scope="module")
def net():
    from paper_1602_07652_amd import Fno
    f = Fno(max_batch=3, max_n=96)
    yield f
    f.close()


@pytest.mark.parametrize("n,S", [(32, 2), (48, 3), (96, 1)])
def test_inputs_and_forward_match_oracle(net, n, S):
    p, flat = _params()
    net.set_params(flat)
    ms, uIs, rs = _inputs(n, S, 1000 + n)
    x_ref, s_ref = _make_x(ms, uIs, rs)
    x, s = net.make_inputs(dev(ms, torch.float64), dev(uIs), dev(rs), shared_medium=False)
    assert np.max(np.abs(host(s) - s_ref)) <= 1e-12 * np.max(s_ref)
    assert np.max(np.abs(host(x) - x_ref)) <= 1e-6 * np.max(np.abs(x_ref))
    y = host(net.forward(x))
    y_ref, _ = ofno.forward(p, x_ref)
    e = rel(y, y_ref)
    banner(f"fno forward n={n} S={S} rel err {e:.3e} (|y| {np.linalg.norm(y_ref):.3e})")
    assert e < TOL


def test_loss_gradients_match_oracle(net):
    n, S = 48, 2
    p, flat = _params(seed=11)
    net.set_params(flat)
    ms, uIs, rs = _inputs(n, S, 2000)
    x_ref, _ = _make_x(ms, uIs, rs)
    target = np.random.default_rng(3).standard_normal((S, 2, n, n)).astype(np.float32)
    y = net.forward(dev(x_ref, torch.float32), keep=True)
    L, dy = net.loss(y, dev(target, torch.float32))
    y_ref, cache = ofno.forward(p, x_ref)
    L_ref, gy_ref = ofno.loss_rel(y_ref, target.astype(np.float64))
    banner(f"loss gpu {L:.6e} oracle {L_ref:.6e}")
    assert abs(L - L_ref) <= TOL * L_ref
    assert rel(host(dy), gy_ref) < TOL
    g = host(net.backward(dy))
    g_ref = ofno.backward(p, cache, gy_ref)
    gv = ofno.unflatten(g.astype(np.float64))
    worst = 0.0
    for k, _ in ofno.param_shapes():
        e = rel(gv[k], g_ref[k])
        worst = max(worst, e)
        banner(f"grad {k:10s} rel err {e:.3e} |g| {np.linalg.norm(g_ref[k]):.3e}")
        assert e < TOL, k
    flat_ref = ofno.flatten(g_ref)
    cos = float(np.dot(g, flat_ref) / (np.linalg.norm(g) * np.linalg.norm(flat_ref)))
    banner(f"gradient cosine {cos:.6f}, worst block {worst:.3e}")
    assert cos > 0.999


def test_adam_step_matches_oracle(net):
    _, flat = _params(seed=5)
    net.set_params(flat)
    rng = np.random.default_rng(9)
    g1 = rng.standard_normal(flat.numel()).astype(np.float32)
    g2 = rng.standard_normal(flat.numel()).astype(np.float32)
    net.adam(dev(g1, torch.float32), lr=1e-3, t=1)
    net.adam(dev(g2, torch.float32), lr=1e-3, t=2)
    got = host(net.get_params()).astype(np.float64)
    p0 = host(flat).astype(np.float64)
    m1 = m2 = np.zeros_like(p0)
    p1, m1, m2 = ofno.adam_step(p0, g1.astype(np.float64), m1, m2, 1, 1e-3)
    p2, _, _ = ofno.adam_step(p1, g2.astype(np.float64), m1, m2, 2, 1e-3)
    e = np.max(np.abs(got - p2)) / 1e-3
    banner(f"adam two steps: max |diff| / lr = {e:.3e}")
    assert e < 1e-3


def test_training_steps_reduce_the_loss(net):
    """A few Adam steps on one fixed batch lower the relative loss: the
    gradient is a descent direction through every kernel of the pass."""
    n, S = 32, 3
    _, flat = _params(seed=3, last_scale=1.0)
    net.set_params(flat)
    ms, uIs, rs = _inputs(n, S, 3000)
    x, _ = _make_x(ms, uIs, rs)
    xd = dev(x, torch.float32)
    target = dev(0.5 * x[:, 3:5], torch.float32)   # a map the network can represent
    losses = []
    for t in range(1, 31):
        y = net.forward(xd, keep=True)
        L, dy = net.loss(y, target)
        losses.append(L)
        net.adam(net.backward(dy), lr=2e-3, t=t)
    banner(f"training losses {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.7 * losses[0]


@pytest.mark.parametrize("n", [33, 40, 48, 64])
def test_apply_is_the_residual_map(net, n):
    """ls_fno_apply runs the inference path (bf16 activations, lift from the
    raw inputs, fused output head): n = 33 has rows and a grid off 16-byte
    boundaries (element-wise loads and stores, the generic x product),
    n = 40 leaves ragged last pixel tiles (P = 1600), n = 48 takes the
    z-transform as two products (n not a multiple of 32), n = 64 as one."""
    p, flat = _params(seed=13)
    net.set_params(flat)
    ms, uIs, rs = _inputs(n, 3, 4000 + n)
    z = host(net.apply(dev(ms[0], torch.float64), dev(uIs), dev(rs)))
    for k in range(3):
        z_ref = ofno.apply(p, ms[0], uIs[k], rs[k])
        # the correction z - r carries the network's error; r passes exactly
        e = rel(z[k] - rs[k], z_ref - rs[k])
        banner(f"apply n={n} k={k} correction rel err {e:.3e}")
        assert e < TOL


@pytest.mark.parametrize("n", [36, 64])
def test_inference_path_is_the_training_forward(net, n):
    """The inference path and the training forward (FP32 activations kept
    for backward, lift and projection as bf16 products) evaluate the same
    network: the corrections agree to the bf16 rounding of the products
    (measured ~3e-3), and the FP64 residual r passes unchanged."""
    p, flat = _params(seed=19)
    net.set_params(flat)
    ms, uIs, rs = _inputs(n, 3, 4500 + n)
    md, uId, rd = dev(ms[0], torch.float64), dev(uIs), dev(rs)
    z = host(net.apply(md, uId, rd))
    x, s = net.make_inputs(md, uId, rd)
    y = host(net.forward(x))
    sh = host(s)
    for k in range(3):
        corr = sh[k] * (y[k, 0].astype(np.float64) + 1j * y[k, 1].astype(np.float64))
        e = rel(z[k] - rs[k], corr)
        banner(f"inference vs training forward n={n} k={k}: correction rel diff {e:.3e}")
        assert e < 1.5e-2


def _solve_problem(n=64, seed=5000, batch=2):
    m, _ = li.fno_sample_recipe(seed, n)
    omega = 2 * np.pi * n / 10
    uI = np.stack([li.plane_wave(n, omega, 0.4 + 1.3 * k) for k in range(batch)])
    return m, omega, uI


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_fno_converges_and_reports(net, precision):
    """With an untrained network the solver still reaches tol (the oracle's
    residual decides), whatever the flags say about the network's passes."""
    from paper_1602_07652_amd import Plan
    n = 64
    _, flat = _params(seed=17, last_scale=1.0)
    net.set_params(flat)
    m, omega, uI = _solve_problem(n)
    plan = Plan(n, 1.0 / n, omega, dev(m, torch.float64), slabs=2, max_batch=2, precision=precision)
    f = plan.rhs_from_incident(dev(uI))
    u, infos = plan.solve_fno(net, dev(uI), f, tol=1e-8, mode=3)
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    for k in range(2):
        fr = kernel.rhs_from_incident(W, m, uI[k], omega)
        res = np.linalg.norm(fr - kernel.apply_H(W, m, host(u[k]), omega)) / np.linalg.norm(fr)
        banner(f"solve_fno prec={precision} k={k} info={infos[k]} oracle residual {res:.3e}")
        assert infos[k]["converged"] == 1 and res < 2e-8
        fl = infos[k]["fno_flags"]
        assert (fl & 1) != (fl & 2) >> 1          # warm start either kept or dropped
        assert ((fl & 4) != 0) != ((fl & 8) != 0)   # network pass either kept or dropped
    plan.close()


def test_poisoned_network_falls_back_to_the_plain_preconditioner(net):
    from paper_1602_07652_amd import Plan
    n = 64
    flat = torch.full((net.nparams,), float("nan"), dtype=torch.float32, device="cuda")
    net.set_params(flat)
    m, omega, uI = _solve_problem(n, seed=5001, batch=1)
    plan = Plan(n, 1.0 / n, omega, dev(m, torch.float64), slabs=2, max_batch=1)
    f = plan.rhs_from_incident(dev(uI))
    u, infos = plan.solve_fno(net, dev(uI), f, tol=1e-8, mode=3)
    u0, i0 = plan.solve(f, tol=1e-8)
    banner(f"poisoned: {infos[0]} plain: {i0[0]}")
    assert infos[0]["fno_flags"] == 2 | 8
    assert infos[0]["converged"] == 1 and infos[0]["relres_true"] <= 1e-8
    assert np.all(np.isfinite(host(u)))
    assert rel(host(u), host(u0)) < 1e-6
    plan.close()
