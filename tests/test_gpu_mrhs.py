"""Many right-hand sides on the matrix cores (FP32 plans, groups of 32
columns): the near field by MFMA in FP32 or bf16, the moments by FP32 MFMA
and the far field by bf16 x3 MFMA. Checked against the oracle's Algorithm 1
(FP64) and against the same plan's column-at-a-time FP32 path."""
import numpy as np
import pytest

import fkt_workloads as W
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2106_04487_amd as F
    return F


CASES = [
    # name, points, kind, kw, leaf, p, theta, nrhs
    ("d3_gauss", lambda: W.uniform_cube(3001, 3, 71), "gaussian", dict(lengthscale=0.1), 64, 4, 0.5, 32),
    ("d5_gauss_p8", lambda: W.gaussian_mixture(4000, 5, 10, 0.1, 72), "gaussian", dict(lengthscale=0.2), 128, 8, 0.5,
     32),
    ("d4_matern52_64rhs", lambda: W.gaussian_mixture(2500, 4, 8, 0.15, 73), "matern52", dict(lengthscale=0.3), 100, 5,
     0.5, 64),
    ("d3_laplace_dups", lambda: W.clustered_duplicates(2000, 3, 300, 74), "laplace", dict(), 50, 4, 0.5, 32),
    ("ragged_n77", lambda: W.uniform_cube(77, 3, 75), "matern32", dict(lengthscale=0.2), 16, 3, 0.5, 32),
]


def _okind(kind, kw):
    if kind == "laplace":
        return "power", dict(shape=1.0)
    return kind, kw


def _run(F, X, x, kind, kw, leaf, p, theta, mrhs):
    import torch
    plan = F.fkt_plan(X, kind, leaf, p, theta=theta, prec="f32", mrhs=mrhs, **kw)
    xd = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
    y = F.fkt_mvm(plan, xd)
    torch.cuda.synchronize()
    plan.close()
    return y.double().cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_mrhs_matches_oracle_and_column_path(F, case):
    name, gen, kind, kw, leaf, p, theta, nrhs = case
    X = gen()
    x = W.normal_rhs(X.shape[0], nrhs, 76)
    T = oracle.Tree(X, leaf)
    ok, okw = _okind(kind, kw)
    zref = np.concatenate([oracle.fkt_alg1(T, x[:, c:c + 32], ok, theta, p, **okw) for c in range(0, nrhs, 32)], 1)
    zcol = _run(F, X, x, kind, kw, leaf, p, theta, None)
    zf32 = _run(F, X, x, kind, kw, leaf, p, theta, "f32")
    zbf = _run(F, X, x, kind, kw, leaf, p, theta, "bf16")
    e = lambda z: np.linalg.norm(z - zref) / np.linalg.norm(zref)
    print(f"{name}: rel err vs oracle: columns {e(zcol):.2e}, mrhs f32 {e(zf32):.2e}, mrhs bf16 {e(zbf):.2e}")
    # FP32 rounding (see the FP32 parity tolerance); bf16 kernel values and
    # weights: 2^-9 relative per product, summed with random signs
    assert e(zcol) <= 1e-5 and e(zf32) <= 1e-5
    assert np.linalg.norm(zf32 - zcol) / np.linalg.norm(zcol) <= 1e-5
    assert e(zbf) <= 1e-2


def test_mrhs_other_column_counts_use_the_column_path(F):
    X = W.uniform_cube(2000, 3, 77)
    x = W.normal_rhs(2000, 5, 78)
    zf = _run(F, X, x, "gaussian", dict(lengthscale=0.1), 64, 4, 0.5, "bf16")
    zc = _run(F, X, x, "gaussian", dict(lengthscale=0.1), 64, 4, 0.5, None)
    assert np.array_equal(zf, zc) or np.linalg.norm(zf - zc) / np.linalg.norm(zc) <= 1e-6


def test_mrhs_needs_fp32_plan(F):
    X = W.uniform_cube(500, 3, 79)
    with pytest.raises(F.FktError):
        F.fkt_plan(X, "gaussian", 64, 4, theta=0.5, prec="f64", mrhs="bf16", lengthscale=0.1)


def test_mrhs_split_nodes_match_column_path(F):
    """Nodes with a far set and more than 1024 points are split over several
    moment work units whose partial moments are summed afterwards; the
    matrix-core moments of 32 columns must agree with the column-at-a-time
    path there too (which the oracle checks elsewhere)."""
    n, theta = 60000, 0.5
    X = W.uniform_cube(n, 3, 80)
    x = W.normal_rhs(n, 32, 81)
    # the case has such nodes: far from some target whose walk reaches them
    T = oracle.Tree(X, 128)
    big = [b for b in range(T.nnodes) if T.end[b] - T.start[b] > 1024 and T.parent[b] >= 0]
    far_somewhere = False
    for b in big:
        pb = T.parent[b]
        d2b = np.sum((X - T.ctr[b]) ** 2, axis=1)
        d2p = np.sum((X - T.ctr[pb]) ** 2, axis=1)
        if np.any((T.rho2[b] < theta * theta * d2b) & ~(T.rho2[pb] < theta * theta * d2p)):
            far_somewhere = True
            break
    assert far_somewhere
    zcol = _run(F, X, x, "gaussian", dict(lengthscale=0.1), 128, 4, theta, None)
    zf32 = _run(F, X, x, "gaussian", dict(lengthscale=0.1), 128, 4, theta, "f32")
    rel = np.linalg.norm(zf32 - zcol) / np.linalg.norm(zcol)
    print(f"split nodes: mrhs f32 vs columns {rel:.2e}")
    assert rel <= 1e-5
