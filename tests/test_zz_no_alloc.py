"""The allocation-free CG solve (fkt_cg_solve_noalloc, work vectors in the
library's fixed scratch array) against the allocating one (fkt_cg_solve) on
the same plans: two calls in a row, the second on a smaller problem, plus
its host-side rejections. Both solves run the same kernels; the MVM's
atomic additions make the two iterate sequences agree only to rounding, so
the solutions are compared at a tolerance the solve's own accuracy sets."""
import numpy as np
import pytest

import fkt_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2106_04487_amd as F
    return F


def _solve_both(F, plan, sig2, b, precond, rtol=1e-10, maxit=3000):
    import torch
    xr, itr, rrr = F.fkt_cg_solve(plan, sig2, b, rtol=rtol, maxit=maxit, precond=precond)
    x = torch.zeros_like(b)
    it, rr = F.fkt_cg_solve_noalloc(plan, sig2, b, x, rtol=rtol, maxit=maxit, precond=precond)
    torch.cuda.synchronize()
    return xr, itr, rrr, x, it, rr


def _check(F, plan, sig2, b, x, rtol):
    import torch
    r = b - F.fkt_mvm(plan, x) - sig2 * x
    return float(torch.linalg.norm(r) / torch.linalg.norm(b))


def test_noalloc_matches_allocating_solve_twice(F):
    import torch
    cases = [  # (n, d, kernel, kw, precond, sigma2, nrhs): the second is smaller
        (20000, 3, "matern32", dict(lengthscale=0.1), "none", 1e-1, 2),
        (6000, 4, "matern52", dict(lengthscale=0.2), "block_jacobi", 1e-2, 1),
    ]
    for n, d, kern, kw, pc, sig2, nrhs in cases:
        print(f"noalloc case n={n} d={d} {kern} precond={pc} nrhs={nrhs}", flush=True)
        X = W.uniform_cube(n, d, 700 + d) if d == 3 else W.gaussian_mixture(n, d, 8, 0.15, 700 + d)
        plan = F.fkt_plan(X, kern, 128, 6, theta=0.4, **kw)
        bh = W.normal_rhs(n, nrhs, 710 + d)
        b = torch.as_tensor(bh if nrhs > 1 else bh[:, 0], device="cuda").contiguous()
        xr, itr, rrr, x, it, rr = _solve_both(F, plan, sig2, b, pc)
        assert rr <= 1e-10 and rrr <= 1e-10
        # the MVM's atomic sums round differently from run to run; at rtol
        # 1e-10 a solve of ~1,200 iterations has shifted by up to 8
        assert abs(it - itr) <= max(2, 0.01 * itr), (it, itr)
        # both are solutions of the same system to 1e-10; their difference is
        # bounded by the condition number times that
        err = float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr))
        print(f"  iterations {it} / {itr}, relres {rr:.2e} / {rrr:.2e}, solution difference {err:.2e}", flush=True)
        assert err <= 1e-6, err
        assert _check(F, plan, sig2, b, x, 1e-10) <= 1e-9
        plan.close()


def test_noalloc_rejections(F):
    import torch
    n = 20000
    X = W.uniform_cube(n, 3, 720)
    plan = F.fkt_plan(X, "gaussian", 128, 4, theta=0.5, lengthscale=0.1)
    b = torch.ones((n, 64), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    # 64 columns of 20000 rows need more than the 64 MiB scratch array
    with pytest.raises(F.FktError) as e:
        F.fkt_cg_solve_noalloc(plan, 1.0, b, x, rtol=1e-6, maxit=10)
    assert e.value.status == 1 and "scratch" in str(e.value)
    # block-Jacobi factors are built by the allocating solve only
    b1 = torch.ones(n, dtype=torch.float64, device="cuda")
    x1 = torch.zeros_like(b1)
    with pytest.raises(F.FktError) as e:
        F.fkt_cg_solve_noalloc(plan, 0.5, b1, x1, rtol=1e-6, maxit=10, precond="block_jacobi")
    assert e.value.status == 1 and "block-Jacobi" in str(e.value)
    torch.cuda.synchronize()
    plan.close()
