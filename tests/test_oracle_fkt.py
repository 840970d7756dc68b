"""Pins of the oracle's dense sum (eq. nbody) and of Algorithm 1.

* Dense: an explicit FP64 kernel matrix (scipy cdist) times x.
* Algorithm 1 with everything near (theta tiny) equals the dense sum.
* Algorithm 1 node-major equals the same operator row by row.
* The relative error against the dense sum falls as p rises (theta fixed),
  for the Gaussian and for 1/r (closed forms above pin each pair).
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import fkt_workloads as W
import oracle


def _kmat(X, kind, **kw):
    R = cdist(X, X)
    ell = kw.get("lengthscale", 1.0)
    if kind == "gaussian":
        return np.exp(-R ** 2 / (2 * ell ** 2))
    if kind == "matern32":
        a = np.sqrt(3.0) / ell
        return (1 + a * R) * np.exp(-a * R)
    if kind == "matern52":
        a = np.sqrt(5.0) / ell
        return (1 + a * R + a * a * R * R / 3) * np.exp(-a * R)
    if kind == "exponential":
        return np.exp(-R / ell)
    if kind == "ratquad":
        al = kw["shape"]
        return (1 + R ** 2 / (2 * al * ell ** 2)) ** (-al)
    if kind == "cauchy":
        return 1.0 / (1 + R ** 2 / ell ** 2)
    if kind == "power":
        with np.errstate(divide="ignore"):
            K = R ** (-kw["shape"])
        K[R == 0] = 0.0
        return K
    raise KeyError(kind)


KS = [("gaussian", dict(lengthscale=0.1)), ("matern32", dict(lengthscale=0.05)),
      ("matern52", dict(lengthscale=0.3)), ("exponential", dict(lengthscale=0.2)),
      ("ratquad", dict(lengthscale=0.2, shape=1.0)), ("cauchy", dict(lengthscale=0.3)),
      ("power", dict(shape=1.0))]


@pytest.mark.parametrize("kind,kw", KS, ids=[k[0] for k in KS])
def test_dense_matches_explicit_matrix(kind, kw):
    X = W.uniform_cube(400, 3, 21)
    x = W.normal_rhs(400, 2, 22)
    z = oracle.dense_mvm(X, x, kind, **kw)
    ref = _kmat(X, kind, **kw) @ x
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("kind,kw", KS, ids=[k[0] for k in KS])
def test_all_near_equals_dense(kind, kw):
    X = W.uniform_cube(700, 3, 31)
    x = W.normal_rhs(700, 1, 32)
    T = oracle.Tree(X, 32)
    z = oracle.fkt_alg1(T, x, kind, 1e-3, 4, **kw)
    zd = oracle.dense_mvm(X, x, kind, **kw)
    assert oracle.rel_err(z, zd) < 1e-13


@pytest.mark.parametrize("d", [3, 4, 5])
def test_rows_equal_algorithm1(d):
    X = W.gaussian_mixture(900, d, 4, 0.15, 40 + d)
    x = W.normal_rhs(900, 3, 50)
    T = oracle.Tree(X, 40)
    z = oracle.fkt_alg1(T, x, "matern52", 0.6, 4, lengthscale=0.4)
    tg = W.subsample(900, 150, 60)
    zr = oracle.fkt_rows(T, x, "matern52", 0.6, 4, tg, lengthscale=0.4)
    np.testing.assert_allclose(zr, z[tg], rtol=0, atol=1e-13 * np.abs(z).max())


def test_error_falls_with_p_gaussian_small_case():
    """2000 uniform points, Gaussian l=0.1, leaf 128, theta = 0.5."""
    X = W.uniform_cube(2000, 3, 1001)
    x = W.normal_rhs(2000, 1, 2001)
    T = oracle.Tree(X, 128)
    zd = oracle.dense_mvm(X, x, "gaussian", lengthscale=0.1)
    errs = [oracle.rel_err(oracle.fkt_alg1(T, x, "gaussian", 0.5, p, lengthscale=0.1), zd) for p in (0, 2, 4, 8, 12)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[2] < 3e-3  # p = 4


def test_error_falls_with_p_laplace():
    X = W.uniform_cube(3000, 3, 77)
    x = W.normal_rhs(3000, 1, 78)
    T = oracle.Tree(X, 64)
    zd = oracle.dense_mvm(X, x, "power", shape=1.0)
    errs = [oracle.rel_err(oracle.fkt_alg1(T, x, "power", 0.5, p, shape=1.0), zd) for p in (0, 2, 4, 6, 8)]
    assert all(b < 0.7 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4
