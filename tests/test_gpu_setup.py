"""The off-line stage (Section 4.1): stage timers, and a plan for a second
medium made from a first plan of the same (n, h, omega) by copying what does
not depend on the medium (kernel samples, spectrum, stencils; Section 2)."""
import numpy as np
import pytest
import torch

import ls_inputs as li
from gpu_helpers import dev, host, rel, banner

pytestmark = pytest.mark.gpu


def _plans(n, **kw):
    from paper_1602_07652_amd import Plan
    omega = 2 * np.pi * n / 10
    m1, _ = li.gaussian_bumps_medium(n, seed=31)
    m2, _ = li.gaussian_bumps_medium(n, seed=32)
    a = Plan(n, 1.0 / n, omega, dev(m1, torch.float64), slabs=max(1, n // 64), ext=10, **kw)
    b = Plan(n, 1.0 / n, omega, dev(m2, torch.float64), slabs=max(1, n // 64), ext=10, like=a, **kw)
    c = Plan(n, 1.0 / n, omega, dev(m2, torch.float64), slabs=max(1, n // 64), ext=10, **kw)
    return a, b, c, omega


@pytest.mark.parametrize("precision", [0, 1])
def test_plan_made_like_another_equals_a_fresh_plan(precision):
    """Same spectrum and stencils bit for bit, so the same operator, slab
    factors and solutions as a plan built from scratch for that medium."""
    n = 256
    a, b, c, omega = _plans(n, autotune=0, precision=precision)
    assert np.array_equal(host(b.spectrum()), host(c.spectrum()))
    ab, bb = b.stencils(), c.stencils()
    assert np.array_equal(ab[0], bb[0]) and np.array_equal(ab[1], bb[1])
    v = dev(li.random_complex((n, n), 5))
    assert np.array_equal(host(b.apply(v)), host(c.apply(v)))
    lims = b.slab_info(0, 1)
    q = lims[3] - lims[2] + 1
    r = dev(li.random_complex((n, q), 6))
    assert np.array_equal(host(b.slab_solve(0, 1, r)), host(c.slab_solve(0, 1, r)))
    f = b.rhs_from_incident(dev(li.plane_wave(n, omega, 0.2)))
    ub, ib = b.solve(f, tol=1e-9)
    uc, ic = c.solve(f, tol=1e-9)
    e = rel(host(ub), host(uc))
    banner(f"like-plan n={n} prec={precision}: solve {ib[0]} vs fresh {ic[0]}: {e:.3e}")
    assert ib[0]["outer_its"] == ic[0]["outer_its"] and e == 0.0
    for p in (a, b, c):
        p.close()


def test_stage_timers_and_what_the_copy_skips():
    n = 512
    a, b, c, omega = _plans(n)
    ta, tb = a.timings(), b.timings()
    banner(f"setup n={n}: fresh {ta}; like {tb}")
    for t in (ta, tb):
        assert all(v >= 0.0 for v in t.values())
        parts = sum(v for k, v in t.items() if k != "total")
        assert parts <= t["total"] * 1.01 + 1.0
    assert ta["samples"] > 0 and ta["stencils"] > 0 and ta["factorisation"] > 0
    # the copy runs no kernel sampling, stencil construction or autotuning
    assert tb["samples"] == 0.0 and tb["stencils"] == 0.0 and tb["autotune"] == 0.0
    assert tb["total"] < ta["total"]
    # the autotuned FFT of the copy is the source's: same operator bits
    v = dev(li.random_complex((n, n), 8))
    assert rel(host(b.apply(v)), host(c.apply(v))) < 1e-14
    for p in (a, b, c):
        p.close()


def test_like_plan_checks_its_source():
    from paper_1602_07652_amd import Plan
    n = 64
    m = dev(li.gaussian_disk_medium(n), torch.float64)
    a = Plan(n, 1.0 / n, 2 * np.pi * 6, m, slabs=2)
    with pytest.raises(ValueError):
        Plan(n, 1.0 / n, 2 * np.pi * 7, m, slabs=2, like=a)
    a.close()
