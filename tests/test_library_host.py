"""Host-side checks of libfkt.so (no GPU needed).

* The library loads and exports every entry point include/fkt.h declares.
* A host-only plan (device = -1) builds the same tree and the same per-target
  partition as the oracle (eq. accparam and the near sets of Sec. 3.2):
  identical point sets per leaf and identical per-target far/near counts.
* Invalid arguments are rejected with the documented status codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import fkt_workloads as W
import oracle

F = pytest.importorskip("paper_2106_04487_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "fkt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fkt_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = _declared_functions()
    assert "fkt_plan" in names and "fkt_mvm" in names and "fkt_cg_solve" in names
    lib = ctypes.CDLL(F.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(F.EXPORTED) == names


CASES = [
    ("cube3_n2k", lambda: W.uniform_cube(2000, 3, 1001), 128, 0.5),
    ("cube3_n30k", lambda: W.uniform_cube(30000, 3, 7), 256, 0.35),
    ("gmm4", lambda: W.gaussian_mixture(8000, 4, 8, 0.15, 9), 100, 0.5),
    ("gmm5", lambda: W.gaussian_mixture(6000, 5, 10, 0.1, 10), 64, 0.6),
    ("dups", lambda: W.clustered_duplicates(3000, 3, 40, 11), 32, 0.5),
    ("tiny", lambda: W.uniform_cube(5, 3, 12), 1, 0.5),
]


@pytest.mark.parametrize("name,gen,leaf,theta", CASES, ids=[c[0] for c in CASES])
def test_host_plan_matches_oracle_partition(name, gen, leaf, theta):
    X = gen()
    p = F.fkt_plan(X, "gaussian", leaf, 3, lengthscale=0.2, theta=theta, device=None, max_depth=30)
    T = oracle.Tree(X, leaf, max_depth=30)
    info = p.info()
    assert info["nnodes"] == T.nnodes
    assert info["nleaves"] == sum(T.is_leaf(b) for b in range(T.nnodes))
    perm = p.perm()
    for b in range(T.nnodes):
        if T.is_leaf(b):
            s, e = T.start[b], T.end[b]
            assert sorted(perm[s:e].tolist()) == sorted(T.perm[s:e].tolist())
    for mine, ref in zip(p.target_counts(), T.counts(theta)):
        np.testing.assert_array_equal(mine, ref)
    # work counters agree with the per-target counts
    fn, fp, nl, npt = p.target_counts()
    assert info["near_pairs"] == int(npt.sum())
    assert info["far_pairs"] == int(fn.sum())
    assert int(fp.sum() + npt.sum()) == X.shape[0] ** 2   # every (t, s) pair exactly once


LIST_CASES = [
    ("cube3_n2k_t0.25", lambda: W.uniform_cube(2000, 3, 1001), 128, 0.25),
    ("cube3_n2k_t0.5", lambda: W.uniform_cube(2000, 3, 1001), 128, 0.5),
    ("cube3_n2k_t0.75", lambda: W.uniform_cube(2000, 3, 1001), 128, 0.75),
    ("cube3_n30k", lambda: W.uniform_cube(30000, 3, 7), 256, 0.35),
    ("gmm4", lambda: W.gaussian_mixture(8000, 4, 8, 0.15, 9), 100, 0.5),
    ("gmm5", lambda: W.gaussian_mixture(6000, 5, 10, 0.1, 10), 64, 0.6),
    ("dups", lambda: W.clustered_duplicates(3000, 3, 40, 11), 32, 0.5),
]


@pytest.mark.parametrize("name,gen,leaf,theta", LIST_CASES, ids=[c[0] for c in LIST_CASES])
def test_host_plan_lists_equal_oracle_walk(name, gen, leaf, theta):
    """The plan's far nodes and near leaves of every target are the oracle
    walk's (eq. accparam, Sec. 3.2), node for node: the mismatch count is 0."""
    X = gen()
    p = F.fkt_plan(X, "gaussian", leaf, 3, lengthscale=0.2, theta=theta, device=None, max_depth=30)
    T = oracle.Tree(X, leaf, max_depth=30)
    fo, fnode, no, nleaf = p.lists()
    mismatched = 0
    for t in range(X.shape[0]):
        far, near = T.walk(X[t], theta)
        mine_f, mine_n = fnode[fo[t]:fo[t + 1]], nleaf[no[t]:no[t + 1]]
        if not (np.array_equal(mine_f, np.sort(far)) and np.array_equal(mine_n, np.sort(near))):
            mismatched += 1
    assert mismatched == 0, f"{mismatched} of {X.shape[0]} targets differ"
    assert fo[-1] == p.info()["far_pairs"]


def test_rank_is_binomial():
    from math import comb
    X = W.uniform_cube(500, 3, 1)
    for d, p in ((3, 0), (3, 4), (3, 6), (3, 8), (4, 5), (5, 4)):
        Xd = W.uniform_cube(300, d, 2)
        plan = F.fkt_plan(Xd, "matern32", 32, p, lengthscale=0.3, device=None)
        assert plan.info()["rank"] == comb(p + d, d)


def _expect(status, fn):
    with pytest.raises(F.FktError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)


def test_invalid_arguments():
    X = W.uniform_cube(100, 3, 3)
    EINVAL, EUNSUP, EDEVICE = 1, 4, 3
    _expect(EINVAL, lambda: F.fkt_plan(X, "gaussian", 0, 4, device=None))
    _expect(EINVAL, lambda: F.fkt_plan(X, "gaussian", 16, -1, device=None))
    _expect(EINVAL, lambda: F.fkt_plan(X, "gaussian", 16, 4, theta=1.0, device=None))
    _expect(EINVAL, lambda: F.fkt_plan(X, "gaussian", 16, 4, theta=0.0, device=None))
    _expect(EINVAL, lambda: F.fkt_plan(X, "gaussian", 16, 4, lengthscale=-1.0, device=None))
    _expect(EINVAL, lambda: F.fkt_plan(X, "ratquad", 16, 4, alpha=0.0, device=None))
    _expect(EINVAL, lambda: F.fkt_plan(X, "gaussian", 16, 4, variance=0.0, device=None))
    _expect(EINVAL, lambda: F.fkt_plan(X, "gaussian", 16, 4, max_depth=0, device=None))
    Xn = X.copy(); Xn[7, 1] = np.nan
    _expect(EINVAL, lambda: F.fkt_plan(Xn, "gaussian", 16, 4, device=None))
    Xi = X.copy(); Xi[3, 0] = np.inf
    _expect(EINVAL, lambda: F.fkt_plan(Xi, "gaussian", 16, 4, device=None))
    _expect(EUNSUP, lambda: F.fkt_plan(W.uniform_cube(50, 2, 1), "gaussian", 16, 4, device=None))
    _expect(EUNSUP, lambda: F.fkt_plan(W.uniform_cube(50, 6, 1), "gaussian", 16, 4, device=None))
    _expect(EUNSUP, lambda: F.fkt_plan(X, "gaussian", 16, 40, device=None))
    with pytest.raises(ValueError):
        F.fkt_plan(X[:, :2].ravel(), "gaussian", 16, 4, device=None)
    # a host-only plan cannot multiply
    p = F.fkt_plan(X, "gaussian", 16, 4, device=None)
    lib = ctypes.CDLL(F.LIB_PATH)
    lib.fkt_mvm.restype = ctypes.c_int
    lib.fkt_mvm.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int]
    buf = (ctypes.c_double * 100)()
    out = (ctypes.c_double * 100)()
    assert lib.fkt_mvm(p.handle, ctypes.addressof(buf), ctypes.addressof(out), 1) == EDEVICE
    assert "host-only" in F.last_error()


def test_solve_entry_points_reject_host_plans():
    """The FP64-in/out and refinement solves check their plans before any
    device work: NULL plans are invalid, host-only plans cannot solve."""
    EINVAL, EDEVICE = 1, 3
    X = W.uniform_cube(100, 3, 5)
    p = F.fkt_plan(X, "gaussian", 16, 4, device=None)
    q = F.fkt_plan(X, "gaussian", 16, 4, device=None, prec="f32")
    lib = ctypes.CDLL(F.LIB_PATH)
    P, D, I = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    lib.fkt_cg_solve64.restype = I
    lib.fkt_cg_solve64.argtypes = [P, D, P, P, I, D, I, I, P, P]
    lib.fkt_cg_solve_refined.restype = I
    lib.fkt_cg_solve_refined.argtypes = [P, P, D, P, P, I, D, I, I, P, P, P]
    b = (ctypes.c_double * 100)()
    x = (ctypes.c_double * 100)()
    ab, ax = ctypes.addressof(b), ctypes.addressof(x)
    assert lib.fkt_cg_solve64(p.handle, 0.1, ab, ax, 1, 1e-6, 10, 0, None, None) == EDEVICE
    assert "host-only" in F.last_error()
    assert lib.fkt_cg_solve_refined(None, q.handle, 0.1, ab, ax, 1, 1e-6, 10, 0, None, None, None) == EINVAL
    assert lib.fkt_cg_solve_refined(p.handle, q.handle, 0.1, ab, ax, 1, 1e-6, 10, 0, None, None, None) == EDEVICE
    assert "host-only" in F.last_error()
    p.close()
    q.close()


def test_duplicate_points_hit_depth_cap():
    X = np.repeat(W.uniform_cube(3, 3, 4), 200, axis=0)
    p = F.fkt_plan(X, "gaussian", 8, 2, lengthscale=0.3, device=None, max_depth=20)
    assert p.info()["depth"] <= 20
    T = oracle.Tree(X, 8, max_depth=20)
    for mine, ref in zip(p.target_counts(), T.counts(0.5)):
        np.testing.assert_array_equal(mine, ref)


def test_batch_plan_is_a_forest_of_oracle_trees():
    """fkt_plan_batch: each instance partitioned exactly as the oracle's own
    tree of that instance alone; no (target, source) pair crosses instances."""
    sizes = [700, 1, 0, 64, 2500, 129]
    X, off = W.batched_instances(sizes, 3, 500)
    theta = 0.45
    p = F.fkt_plan_batch((X, off), "gaussian", 50, 3, lengthscale=0.2, theta=theta, device=None)
    counts = p.target_counts()
    perm = p.perm()
    nnodes = 0
    for i, m in enumerate(sizes):
        if m == 0:
            continue
        a, b = off[i], off[i + 1]
        T = oracle.Tree(X[a:b], 50)
        nnodes += T.nnodes
        for mine, ref in zip(counts, T.counts(theta)):
            np.testing.assert_array_equal(mine[a:b], ref)
        assert int(counts[1][a:b].sum() + counts[3][a:b].sum()) == m * m
        assert sorted(perm[a:b].tolist()) == list(range(a, b))   # tree positions stay in the instance
    assert p.info()["nnodes"] == nnodes


def test_batch_plan_rejects_bad_offsets():
    X = W.uniform_cube(10, 3, 1)
    with pytest.raises(F.FktError):
        F.fkt_plan_batch((X, np.array([0, 6, 4, 10])), "gaussian", 8, 2, lengthscale=0.2, device=None)
    with pytest.raises(F.FktError):
        F.fkt_plan_batch((X, np.array([1, 10])), "gaussian", 8, 2, lengthscale=0.2, device=None)


@pytest.mark.parametrize("kernel,kw,d", [("laplace", {}, 3), ("laplace", {}, 4), ("laplace", {}, 5),
                                         ("exponential", dict(lengthscale=0.3), 3),
                                         ("exponential", dict(lengthscale=0.3), 5),
                                         ("gaussian", dict(lengthscale=0.3), 3)])
def test_radial_compression_equals_oracle(kernel, kw, d):
    """The library's ranks R_k (exact, modular) and interpolative
    coefficients equal the oracle's exact-fraction ones (oracle/radial.py,
    pinned by the paper's Table "ranks" and e^-r decomposition), p = 0..8."""
    from oracle import radial as R
    q = R.LAURENT_Q[{"laplace": "power1", "exponential": "exponential", "gaussian": "gaussian"}[kernel]]
    for p in range(9):
        rk, keep, coef = F.fkt_radial_compression(kernel, d, p, **kw)
        assert rk == R.ranks(q, d, p), (p, rk)
        built = {("laplace", 3): 1, ("exponential", 3): 2}.get((kernel, d), 0)
        assert keep == built
        if keep:
            for k in range(p + 1):
                n = min(keep, (p - k) // 2 + 1)
                c = R.interpolative(q, d, k, p, n)
                for jj, row in enumerate(c):
                    for i, v in enumerate(row):
                        assert coef[k, jj, i] == pytest.approx(float(v), rel=1e-15, abs=1e-300), (p, k, jj, i)
        else:
            assert coef is None


def test_radial_compression_plan_rank_and_rejections():
    X = W.uniform_cube(3000, 3, 5)
    for kernel, kw, want in [("laplace", {}, 49), ("exponential", dict(lengthscale=0.2), 74),
                             ("gaussian", dict(lengthscale=0.2), 84)]:
        pl = F.fkt_plan(X, kernel, 64, 6, theta=0.5, device=None, compress=True, **kw)
        i = pl.info()
        assert i["rank"] == 84 and i["radial_rank"] == want, (kernel, i["radial_rank"])
        pl.close()
    pl = F.fkt_plan(X, "laplace", 64, 6, theta=0.5, device=None)
    assert pl.info()["radial_rank"] == 84
    pl.close()
    with pytest.raises(F.FktError, match="FKT_EINVAL"):
        F.fkt_plan(X, "matern32", 64, 6, theta=0.5, device=None, compress=True, lengthscale=0.2)
    with pytest.raises(F.FktError, match="FKT_EUNSUPPORTED"):
        F.fkt_plan(X, "laplace", 64, 6, theta=0.5, device=None, compress=True, far_mode="block")
    with pytest.raises(F.FktError, match="FKT_EINVAL"):
        F.fkt_radial_compression("matern52", 3, 6, lengthscale=0.2)


def test_fuse_option_validation():
    """The persistent launch is refused where it is not built (d = 4, 5) or
    cannot run (block-major far field, radial compression)."""
    X3, X4 = W.uniform_cube(2000, 3, 8), W.uniform_cube(2000, 4, 9)
    pl = F.fkt_plan(X3, "gaussian", 64, 4, theta=0.5, device=None, fuse=True, lengthscale=0.2)
    pl.close()
    for X, kw in ((X4, {}), (X3, dict(far_mode="block")), (X3, dict(compress=True))):
        with pytest.raises(F.FktError, match="FKT_EUNSUPPORTED"):
            F.fkt_plan(X, "gaussian", 64, 4, theta=0.5, device=None, fuse=True, lengthscale=0.2, **kw)
