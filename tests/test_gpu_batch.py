"""Batched uneven instances (fkt_plan_batch), HIP-graph replay and the
leaf-size autotuner, against the oracle run on each instance alone."""
import numpy as np
import pytest

import fkt_workloads as W
import oracle

pytestmark = pytest.mark.gpu

KW = dict(lengthscale=0.2, alpha=1.0)
OKW = dict(lengthscale=0.2, shape=1.0)


@pytest.fixture(scope="module")
def F():
    import paper_2106_04487_amd as F
    return F


def _oracle_batch(X, off, x, leaf, p, theta):
    out = np.zeros_like(x)
    for i in range(len(off) - 1):
        a, b = off[i], off[i + 1]
        if b > a:
            out[a:b] = oracle.fkt_alg1(oracle.Tree(X[a:b], leaf), x[a:b], "ratquad", theta, p, **OKW)
    return out


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_batch_mvm_matches_oracle_per_instance(F, prec, tol):
    import torch
    sizes = [1500, 1, 64, 3000, 0, 777]
    X, off = W.batched_instances(sizes, 3, 900)
    x = W.normal_rhs(X.shape[0], 4, 901)
    leaf, p, theta = 64, 5, 0.5
    plan = F.fkt_plan_batch((X, off), "ratquad", leaf, p, theta=theta, prec=prec, **KW)
    dt = torch.float32 if prec == "f32" else torch.float64
    y = F.fkt_mvm(plan, torch.as_tensor(x, dtype=dt, device="cuda")).double().cpu().numpy()
    zref = _oracle_batch(X, off, x, leaf, p, theta)
    for i in range(len(sizes)):
        a, b = off[i], off[i + 1]
        if b > a:
            e = np.linalg.norm(y[a:b] - zref[a:b]) / np.linalg.norm(zref[a:b])
            assert e <= tol, (i, sizes[i], e)
    plan.close()


def test_batch_many_rhs_matches_oracle_per_instance(F):
    """32 columns on the matrix cores over a forest: the far pairs of groups
    of consecutive target blocks are packed together and the near and far
    units add into one buffer, so groups and units span instance borders;
    every instance must still match the oracle run on it alone (FP32 MFMA
    near field, bf16 x3 far field: the FP32 bar)."""
    import torch
    sizes = [1500, 1, 64, 3000, 0, 777, 2500]
    X, off = W.batched_instances(sizes, 3, 902)
    x = W.normal_rhs(X.shape[0], 32, 903)
    leaf, p, theta = 32, 5, 0.5
    plan = F.fkt_plan_batch((X, off), "ratquad", leaf, p, theta=theta, prec="f32", mrhs="f32", **KW)
    y = F.fkt_mvm(plan, torch.as_tensor(x, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    zref = _oracle_batch(X, off, x, leaf, p, theta)
    for i in range(len(sizes)):
        a, b = off[i], off[i + 1]
        if b > a:
            e = np.linalg.norm(y[a:b] - zref[a:b]) / np.linalg.norm(zref[a:b])
            assert e <= 1e-5, (i, sizes[i], e)


@pytest.mark.parametrize("prec,mrhs,nrhs", [("f64", None, 4), ("f32", None, 4), ("f32", "bf16", 32)])
def test_graph_replays_match_eager(F, prec, mrhs, nrhs):
    import torch
    X, off = W.batched_instances([2000, 300, 4000], 3, 910)
    plan = F.fkt_plan_batch((X, off), "ratquad", 64, 4, theta=0.5, prec=prec, mrhs=mrhs, **KW)
    dt = torch.float32 if prec == "f32" else torch.float64
    x = torch.as_tensor(W.normal_rhs(X.shape[0], nrhs, 911), dtype=dt, device="cuda").contiguous()
    y_eager = F.fkt_mvm(plan, x).clone()
    y = torch.zeros_like(x)
    g = F.Graph(plan, x, y)
    tol = 1e-12 if prec == "f64" else 2e-6
    other = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        y.zero_()
        g.launch()
        torch.cuda.synchronize()
        e = (torch.linalg.norm(y.double() - y_eager.double()) / torch.linalg.norm(y_eager.double())).item()
        assert e <= tol, (rep, e)
        # eager work between replays, on the same buffers' neighbours
        other.mul_(1.0001)
        F.fkt_mvm(plan, x, torch.empty_like(x))
        torch.cuda.synchronize()
    g.close()
    plan.close()


@pytest.mark.parametrize("prec,true_tol", [("f64", 1e-5), ("f32", 1e-4), ("mixed", 1e-4)])
@pytest.mark.parametrize("precond", ["none", "block_jacobi"])
def test_batch_cg_solves_every_instance(F, prec, true_tol, precond):
    """The operator of a batched plan is block diagonal: each instance (and
    column) is its own CG system. Every instance must meet rtol on its own
    rows (checked against the oracle's operator), and the batched solve must
    take no more iterations than the slowest instance solved alone ("mixed":
    FP32 plan, FP64 b and x through fkt_cg_solve64). The
    operator is made accurate (theta 0.35, p 6) so that CG's recurrences
    hold for K~, which is symmetric only up to the expansion error."""
    import torch
    sizes = [1500, 1, 64, 3000, 0, 777]
    X, off = W.batched_instances(sizes, 3, 930)
    leaf, p, theta, sig2, rtol = 64, 6, 0.35, 0.1, 1e-6
    b = W.normal_rhs(X.shape[0], 2, 931)
    dt = torch.float32 if prec == "f32" else torch.float64
    pprec = "f64" if prec == "f64" else "f32"
    solve = F.fkt_cg_solve64 if prec == "mixed" else F.fkt_cg_solve
    plan = F.fkt_plan_batch((X, off), "ratquad", leaf, p, theta=theta, prec=pprec, **KW)
    xb, itb, rrb = solve(plan, sig2, torch.as_tensor(b, dtype=dt, device="cuda"), rtol=rtol, maxit=2000,
                         precond=precond)
    plan.close()
    xb = xb.double().cpu().numpy()
    assert rrb <= rtol
    its = []
    for i in range(len(sizes)):
        a0, a1 = off[i], off[i + 1]
        if a1 == a0:
            continue
        Xi, bi, xi = X[a0:a1], b[a0:a1], xb[a0:a1]
        Kx = oracle.fkt_alg1(oracle.Tree(Xi, leaf), xi, "ratquad", theta, p, **OKW)
        res = np.linalg.norm(bi - Kx - sig2 * xi, axis=0) / np.linalg.norm(bi, axis=0)
        assert res.max() <= true_tol, (i, sizes[i], res)
        pi = F.fkt_plan(Xi, "ratquad", leaf, p, theta=theta, prec=pprec, **KW)
        xs, it, _ = solve(pi, sig2, torch.as_tensor(bi, dtype=dt, device="cuda"), rtol=rtol, maxit=2000,
                          precond=precond)
        pi.close()
        its.append(it)
        xs = xs.double().cpu().numpy()
        e = np.linalg.norm(xi - xs) / np.linalg.norm(xs)
        assert e <= 100 * true_tol, (i, sizes[i], e)
    print("batched iterations", itb, "per instance", its)
    assert itb <= max(its) + 2 + max(its) // 20


def test_batch_refined_solve_meets_fp64_residual(F):
    """Mixed-precision CG on a batched plan: FP32 MVMs, residual replaced by
    the FP64 plan's. Every instance meets 1e-6 under the oracle's operator (the
    same truncation as the FP64 plan), where FP32 CG alone stops near the
    FP32 operator's error."""
    import torch
    sizes = [1500, 1, 64, 3000, 0, 777]
    X, off = W.batched_instances(sizes, 3, 930)
    leaf, p, theta, sig2, rtol = 64, 6, 0.35, 0.1, 1e-6
    b = W.normal_rhs(X.shape[0], 2, 931)
    p64 = F.fkt_plan_batch((X, off), "ratquad", leaf, p, theta=theta, prec="f64", **KW)
    p32 = F.fkt_plan_batch((X, off), "ratquad", leaf, p, theta=theta, prec="f32", **KW)
    bt = torch.as_tensor(b, device="cuda")
    x, it, outer, rr = F.fkt_cg_solve_refined(p64, p32, sig2, bt, rtol=rtol, maxit=2000, precond="block_jacobi")
    print(f"refined: {it} FP32 iterations, {outer} FP64 residual replacements, FP64 relres {rr:.2e}")
    assert rr <= rtol and 1 <= outer <= 40
    x = x.cpu().numpy()
    for i in range(len(sizes)):
        a0, a1 = off[i], off[i + 1]
        if a1 == a0:
            continue
        Xi, bi, xi = X[a0:a1], b[a0:a1], x[a0:a1]
        Kx = oracle.fkt_alg1(oracle.Tree(Xi, leaf), xi, "ratquad", theta, p, **OKW)
        res = np.linalg.norm(bi - Kx - sig2 * xi, axis=0) / np.linalg.norm(bi, axis=0)
        assert res.max() <= 1.1 * rtol, (i, sizes[i], res)
    # the second plan must be the FP32 one
    with pytest.raises(F.FktError):
        F.fkt_cg_solve_refined(p64, p64, sig2, bt)
    p64.close()
    p32.close()


def test_autotuner_picks_a_candidate(F):
    X, off = W.batched_instances([3000, 500, 8000], 3, 920)
    best, ms = F.fkt_autotune_leaf((X, off), "ratquad", 4, [32, 64, 128, 256], nrhs=4, reps=2, theta=0.5,
                                   prec="f32", batch=True, **KW)
    print("autotune ms per MVM:", ms, "best", best)
    assert best in ms and all(v > 0.0 for v in ms.values())
    assert ms[best] == min(ms.values())


def test_autotune_over_leaf_and_far_schedule(F):
    """fkt_autotune times every (leaf, far-field schedule) pair and returns
    the fastest; the pair it returns builds a plan whose MVM matches the
    oracle on every instance."""
    X, off = W.batched_instances(W.instance_sizes(6, 500, 4000, 140), 3, 141)
    (leaf, mode), table = F.fkt_autotune((X, off), "ratquad", 4, [32, 64, 128], ("block", "node"), nrhs=2, reps=1,
                                         theta=0.5, batch=True, **KW)
    assert len(table) == 6 and all(v > 0 for v in table.values())
    assert table[(leaf, mode)] == min(table.values())
    plan = F.fkt_plan_batch((X, off), "ratquad", leaf, 4, theta=0.5, far_mode=mode, **KW)
    x = W.normal_rhs(X.shape[0], 2, 142)
    import torch
    y = F.fkt_mvm(plan, torch.as_tensor(x, device="cuda")).cpu().numpy()
    ref = _oracle_batch(X, off, x, leaf, 4, 0.5)
    assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref)
    plan.close()
