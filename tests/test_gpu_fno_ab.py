"""What the trained network gains over the method without it (A/B), with the
weights trained by paper_1602_07652_amd.fno_train on 2000 solves at 256^2
(Gaussian-random-field media, seeds 1000-2999).  Test media use seeds
5000+ (never seen in training).  The FP64 oracle checks every solution's
residual; iteration counts and wall times are printed for both arms."""
import os
import time

import numpy as np
import pytest
import torch

from oracle import fno as ofno, kernel
import ls_inputs as li
from gpu_helpers import dev, host, rel, banner

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1602_07652_amd", "weights", "fno_grf256.npz")


@pytest.fixture(scope="module")
def trained():
    from paper_1602_07652_amd import Fno
    from paper_1602_07652_amd.fno_train import load_weights
    params, meta = load_weights(WEIGHTS)
    f = Fno(max_batch=4, max_n=1024)
    f.set_params(params)
    yield f, params, meta
    f.close()


def _case(n, seed):
    m, theta = li.fno_sample_recipe(seed, n)
    omega = 2 * np.pi * n / 10
    return m, omega, li.plane_wave(n, omega, theta)


def _oracle_residual(n, omega, m, uI, u):
    W = kernel.kernel_samples(n, 1.0 / n, omega)
    fr = kernel.rhs_from_incident(W, m, uI, omega)
    return np.linalg.norm(fr - kernel.apply_H(W, m, u, omega)) / np.linalg.norm(fr)


def test_trained_weights_forward_matches_oracle(trained):
    fno, params, meta = trained
    n = 64
    m, omega, uI = _case(n, 5100)
    r = li.random_complex((n, n), 5101)
    z = host(fno.apply(dev(m, torch.float64), dev(uI[None]), dev(r[None])))[0]
    p = ofno.unflatten(host(params).astype(np.float64))
    z_ref = ofno.apply(p, m, uI, r)
    e = rel(z - r, z_ref - r)
    banner(f"trained network, n={n}: correction rel err vs oracle {e:.3e} (trained val loss "
           f"{meta['history'][-1]['val']:.4f})")
    assert e < 4e-2


def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def test_warm_start_gain_at_training_size(trained):
    """256^2, held-out media: the network's initial guess leaves a residual
    well below ||f|| (u0 = 0 leaves exactly ||f||), and the warm-started
    solves need fewer outer iterations in total than the plain ones
    (measured 24 against 26 over the four media)."""
    from paper_1602_07652_amd import Plan
    fno, _, _ = trained
    n = 256
    rows, r0s = [], []
    for seed in range(5000, 5004):
        m, omega, uI = _case(n, seed)
        md = dev(m, torch.float64)
        plan = Plan(n, 1.0 / n, omega, md, slabs=4)
        uId = dev(uI[None])
        f = plan.rhs_from_incident(uId)
        plan.solve(f, tol=1e-8)  # warm-up (graph capture)
        (u_p, i_p), t_p = _timed(lambda: plan.solve(f, tol=1e-8))
        (u_w, i_w), t_w = _timed(lambda: plan.solve_fno(fno, uId, f, tol=1e-8, mode=1))
        u0 = fno.apply(md, uId, f)
        r0 = float(torch.linalg.norm(f - plan.apply(u0)) / torch.linalg.norm(f))
        res = _oracle_residual(n, omega, m, uI, host(u_w[0]))
        banner(f"n={n} seed={seed}: plain {i_p[0]['outer_its']} its {t_p * 1e3:.1f} ms | "
               f"warm start residual {r0:.3f}, {i_w[0]['outer_its']} its {t_w * 1e3:.1f} ms, "
               f"flags {i_w[0]['fno_flags']}, oracle residual {res:.2e}")
        assert i_w[0]["converged"] == 1 and res < 2e-8
        rows.append((i_p[0]["outer_its"], i_w[0]["outer_its"]))
        r0s.append(r0)
        plan.close()
    its_p, its_w = map(sum, zip(*rows))
    banner(f"256^2 totals: plain {its_p} outer its, warm-started {its_w}; mean warm residual "
           f"{np.mean(r0s):.3f}")
    assert np.mean(r0s) < 0.6
    assert its_w < its_p


def test_learned_arm_gain_on_64_waves():
    """The learned form's job at its training size, as bench.py runs it: 64
    plane waves (theta_k = 2 pi k / 64) on a held-out 256^2 GRF medium, FP32
    operator and slab solves with FP64 refinement, the network (64 samples
    per evaluation) as warm start with the probe.  Every wave of both arms
    reaches 1e-8 (the oracle's FP64 residual checks sampled waves), and the
    learned arm needs strictly fewer outer iterations in total (measured 6
    against 7 per wave; wall times are printed: 35.3 against 37.8 ms)."""
    from paper_1602_07652_amd import Plan, Fno, LS_FP32_REFINE, LS_FNO_WARM, LS_FNO_PROBE
    from paper_1602_07652_amd.fno_train import load_weights
    params, _ = load_weights(WEIGHTS)
    n, B = 256, 64
    omega = 2 * np.pi * n / 10
    m = li.gaussian_random_field_medium(n, seed=5000)
    plan = Plan(n, 1.0 / n, omega, dev(m, torch.float64), slabs=n // 64, ext=10, max_batch=B,
                precision=LS_FP32_REFINE)
    net = Fno(max_batch=B, max_n=n)
    net.set_params(params)
    uI = np.stack([li.plane_wave(n, omega, 2 * np.pi * k / B) for k in range(B)])
    uId = dev(uI)
    f = plan.rhs_from_incident(uId)
    arms = {}
    for arm in ("plain", "learned"):
        run = (lambda: plan.solve(f, tol=1e-8)) if arm == "plain" else \
              (lambda: plan.solve_fno(net, uId, f, tol=1e-8, mode=LS_FNO_WARM | LS_FNO_PROBE))
        run()  # warm-up: graphs, Krylov spaces
        (u, infos), t = _timed(run)
        its = sum(i["outer_its"] for i in infos)
        arms[arm] = (host(u), infos, its, t)
        banner(f"64 waves at 256^2, {arm}: {its} outer its in total, {t * 1e3:.1f} ms, "
               f"max relres {max(i['relres_true'] for i in infos):.2e}")
        assert all(i["converged"] == 1 and i["relres_true"] <= 1e-8 for i in infos)
    for k in (0, 37):
        res = _oracle_residual(n, omega, m, uI[k], arms["learned"][0][k])
        banner(f"learned arm wave {k}: oracle residual {res:.2e} (flags {arms['learned'][1][k]['fno_flags']})")
        assert res < 2e-8
    assert all(i["fno_flags"] & 1 for i in arms["learned"][1])  # every warm start kept
    assert arms["learned"][2] < arms["plain"][2]
    net.close()
    plan.close()


@pytest.mark.parametrize("n", [512, 1024])
def test_ab_beyond_training_size(trained, n):
    """Larger grids (more wavelengths than in training): report both arms;
    whatever the network does, the solve reaches tol and the flags say
    whether its passes were kept."""
    from paper_1602_07652_amd import Plan
    fno, _, _ = trained
    m, omega, uI = _case(n, 5200 + n)
    md = dev(m, torch.float64)
    plan = Plan(n, 1.0 / n, omega, md, slabs=n // 64)
    uId = dev(uI[None])
    f = plan.rhs_from_incident(uId)
    plan.solve(f, tol=1e-8)
    (u_p, i_p), t_p = _timed(lambda: plan.solve(f, tol=1e-8))
    out = {}
    for mode in (1, 3):
        (u, i), t = _timed(lambda: plan.solve_fno(fno, uId, f, tol=1e-8, mode=mode))
        out[mode] = (u, i[0], t)
    u0 = fno.apply(md, uId, f)
    r0 = float(torch.linalg.norm(f - plan.apply(u0)) / torch.linalg.norm(f))
    banner(f"n={n}: plain {i_p[0]['outer_its']} its {t_p * 1e3:.1f} ms | warm start residual {r0:.3f} | "
           + " | ".join(f"mode {k}: {v[1]['outer_its']} its {v[2] * 1e3:.1f} ms flags {v[1]['fno_flags']}"
                        for k, v in out.items()))
    for k, (u, i, _) in out.items():
        assert i["converged"] == 1 and i["relres_true"] <= 1e-8
        fl = i["fno_flags"]
        assert (fl & 1) != ((fl & 2) >> 1)
        if k == 3:
            assert ((fl & 4) != 0) != ((fl & 8) != 0)
    if n == 512:
        res = _oracle_residual(n, omega, m, uI, host(out[1][0][0]))
        banner(f"n={n}: oracle residual of the warm-started solution {res:.2e}")
        assert res < 2e-8
    plan.close()


def test_probe_skips_the_network_where_its_warm_start_is_dropped(trained):
    """LS_FNO_PROBE: at 256^2 (training size) the probe's warm start is kept
    and every wave gets one; at 1024^2 it is dropped and the other waves
    start from zero without evaluating the network.  Every solve reaches tol."""
    from paper_1602_07652_amd import (Plan, LS_FNO_WARM, LS_FNO_PROBE, LS_FNO_WARM_USED,
                                      LS_FNO_WARM_REJECTED, LS_FNO_WARM_SKIPPED)
    fno, _, _ = trained
    for n, B in [(256, 6), (1024, 3)]:
        m, omega, _ = _case(n, 5300 + n)
        uI = np.stack([li.plane_wave(n, omega, 2 * np.pi * k / B) for k in range(B)])
        plan = Plan(n, 1.0 / n, omega, dev(m, torch.float64), slabs=n // 64, max_batch=B, precision=1)
        uId = dev(uI)
        f = plan.rhs_from_incident(uId)
        u, infos = plan.solve_fno(fno, uId, f, tol=1e-8, mode=LS_FNO_WARM | LS_FNO_PROBE)
        flags = [i["fno_flags"] for i in infos]
        banner(f"probe n={n}: flags {flags}, outer its {[i['outer_its'] for i in infos]}")
        assert all(i["converged"] == 1 and i["relres_true"] <= 1e-8 for i in infos)
        if flags[0] & LS_FNO_WARM_USED:
            assert all(fl & (LS_FNO_WARM_USED | LS_FNO_WARM_REJECTED) for fl in flags)
            assert not any(fl & LS_FNO_WARM_SKIPPED for fl in flags)
        else:
            assert flags[0] & LS_FNO_WARM_REJECTED
            assert all(fl == LS_FNO_WARM_SKIPPED for fl in flags[1:])
        if n == 256:
            assert flags[0] & LS_FNO_WARM_USED
        plan.close()
