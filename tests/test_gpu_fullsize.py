"""Full-size workloads checked by the FP64 oracle's residual (a property that
holds at any size): the plain 1024^2 solve as bench.py times it, and the
64-wave batched FP32 + refinement solve at 1024^2 on sampled waves."""
import numpy as np
import pytest
import torch

from oracle import kernel
import ls_inputs as li
from gpu_helpers import dev, host, banner

pytestmark = pytest.mark.gpu


def _oracle_residual(W, Gh, m, omega, uI, u):
    fr = kernel.rhs_from_incident(W, m, uI, omega)
    return np.linalg.norm(fr - kernel.apply_H(W, m, u, omega, Gh)) / np.linalg.norm(fr)


@pytest.mark.parametrize("sweep,inner", [(1, 1), (1, 0), (0, 0)])
def test_plain_solve_at_bench_size(sweep, inner):
    """1024^2, 8 Gaussian bumps (seed 0), 16 layers, ext 10, FP64, tol 1e-8:
    the solve bench.py times (decoupled sweeps, sweep=1, one inner
    iteration per outer iteration: Section 6's relaxed inner solve), the same
    with Alg. 3 as printed (inner tolerance 1e-3), and that with the
    sequential sweeps.  The oracle's own run of this workload takes 5 outer
    iterations with 2 inner each and reaches 1.7e-9."""
    from paper_1602_07652_amd import Plan
    cfg = li.config_inputs("c2_1024_bumps")
    n, omega = cfg["n"], cfg["omega"]
    p = Plan(n, 1.0 / n, omega, dev(cfg["m"], torch.float64), slabs=cfg["slabs"], ext=10, sweep=sweep,
             inner_fixed_iters=inner)
    f = p.rhs_from_incident(dev(cfg["uI"][None]))
    u, info = p.solve(f, tol=1e-8)
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    Gh = kernel.circulant_spectrum(W)
    res = _oracle_residual(W, Gh, cfg["m"], omega, cfg["uI"], host(u[0]))
    banner(f"bench workload (sweep={sweep}, inner_fixed_iters={inner}): {info[0]}, oracle residual {res:.3e}")
    assert info[0]["converged"] == 1 and res < 1e-8
    assert abs(res - info[0]["relres_true"]) <= 1e-3 * res + 1e-14
    assert info[0]["outer_its"] <= 6 and info[0]["inner_its_total"] <= 12
    if inner:
        assert info[0]["inner_its_total"] == info[0]["outer_its"]
    p.close()


@pytest.mark.parametrize("inner", [0, 1])
def test_batched_64_waves_at_1024(inner):
    """64 plane waves theta_k = 2 pi k / 64 on the 1024^2 8-bump medium (seed
    3, omega = 2 pi n / 10), FP32 operator and slab solves with FP64
    refinement, matrix-core level steps and top operator, with Alg. 3 as
    printed and (inner 1) one inner iteration per outer iteration, the form
    bench.py times: every wave reaches 1e-8 by the library's FP64 residual,
    and the oracle agrees on samples."""
    from paper_1602_07652_amd import Plan, LS_FP32_REFINE
    n, B = 1024, 64
    omega = 2 * np.pi * n / 10
    m, _ = li.gaussian_bumps_medium(n, seed=3)
    p = Plan(n, 1.0 / n, omega, dev(m, torch.float64), slabs=n // 64, ext=10, max_batch=B,
             precision=LS_FP32_REFINE, inner_fixed_iters=inner)
    uI = np.stack([li.plane_wave(n, omega, 2 * np.pi * k / B) for k in range(B)])
    f = p.rhs_from_incident(dev(uI))
    u, infos = p.solve(f, tol=1e-8)
    assert all(i["converged"] == 1 and i["relres_true"] <= 1e-8 for i in infos)
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    Gh = kernel.circulant_spectrum(W)
    uh = host(u)
    for k in (0, 17, 63):
        res = _oracle_residual(W, Gh, m, omega, uI[k], uh[k])
        banner(f"64 waves at 1024^2, wave {k}: {infos[k]}, oracle residual {res:.3e}")
        assert res < 1e-8
        assert abs(res - infos[k]["relres_true"]) <= 1e-3 * res + 1e-14
    p.close()
