"""The allocation-free slab solve (ls_slab_solve_noalloc) against the slab
solve it is a variant of (ls_slab_solve): same kernels, so the same bits.

Both are called through the C ABI.  The static scratch is shared by every
call on the GPU and keeps the last call's contents, so the cases run back to
back with a smaller slab after a larger one, then in place, then on an FP32
plan (whose solve converts b and x through the scratch too)."""
import numpy as np
import pytest
import torch

import ls_inputs as li
from gpu_helpers import dev, host, banner

pytestmark = pytest.mark.gpu


def _plan(n, L, **kw):
    from paper_1602_07652_amd import Plan
    m, _ = li.gaussian_bumps_medium(n, seed=n + 7)
    banner(f"no-alloc plan n={n} L={L} {kw}")
    return Plan(n, 1.0 / n, 2 * np.pi * n / 10, dev(m, torch.float64), slabs=L, ext=10, **kw)


def _case(p, orient, l, seed):
    a, b, z0, z1 = p.slab_info(orient, l)
    q = z1 - z0 + 1
    rhs = dev(li.random_complex((p.n, q), seed=seed))
    ref = host(p.slab_solve(orient, l, rhs))
    got = host(p.slab_solve_noalloc(orient, l, rhs))
    banner(f"n={p.n} orient={orient} slab={l} q={q}: max |noalloc - slab_solve| "
           f"{np.max(np.abs(got - ref)):.3e}")
    assert np.array_equal(got, ref)
    assert np.all(np.isfinite(got)) and np.max(np.abs(got)) > 0
    return rhs, ref


def test_noalloc_scratch_size():
    from paper_1602_07652_amd import lib
    # two FP64 slab vectors of the largest slab a plan accepts (n = 2048, q = 96)
    assert lib().ls_noalloc_scratch_bytes() == 2 * 2048 * 96 * 16


def test_noalloc_slab_solve_equals_slab_solve():
    big = _plan(512, 8)
    _case(big, 1, 3, 11)                    # interior slab, q = 84
    small = _plan(200, 4)
    rhs, ref = _case(small, 0, 0, 12)       # smaller slab after it: q = 60
    # in place (b == x): the copy of b goes through the scratch as well
    x = rhs.clone()
    small.slab_solve_noalloc(0, 0, x, out=x)
    assert np.array_equal(host(x), ref)
    _case(big, 0, 7, 13)                    # and a larger one again
    big.close()
    small.close()


def test_noalloc_slab_solve_fp32_plan():
    from paper_1602_07652_amd import LS_FP32_REFINE
    p = _plan(256, 4, precision=LS_FP32_REFINE)
    _case(p, 0, 1, 21)
    _case(p, 1, 0, 22)
    p.close()
