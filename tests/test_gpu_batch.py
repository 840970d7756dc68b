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


def test_autotuner_picks_a_candidate(F):
    X, off = W.batched_instances([3000, 500, 8000], 3, 920)
    best, ms = F.fkt_autotune_leaf((X, off), "ratquad", 4, [32, 64, 128, 256], nrhs=4, reps=2, theta=0.5,
                                   prec="f32", batch=True, **KW)
    print("autotune ms per MVM:", ms, "best", best)
    assert best in ms and all(v > 0.0 for v in ms.values())
    assert ms[best] == min(ms.values())
