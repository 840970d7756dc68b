"""Pins of the oracle's factorised FKT (Cartesian moments, ``fkt_cart``).

The factorised oracle reads Theorem 3.1 as the degree-p Taylor polynomial of
y -> K(|r - y|) about the node centre (the j-group of eq. finaltrunc is its
homogeneous degree-j part), and builds the Taylor coefficients from the
rho-derivatives of h(rho) = K(sqrt(rho)). Its pins do not use its own
arithmetic:

* the rho-derivatives (closed forms per kernel) against mpmath's
  high-precision differentiation of K(sqrt(rho));
* one pair against mpmath's Taylor polynomial in t of K(|r - t r'|);
* the whole operator against the pairwise Gegenbauer form of Algorithm 1
  (``fkt_alg1``, itself pinned by tests/test_oracle_expansion.py and
  tests/test_oracle_fkt.py) on small inputs, for several kernels, d and p,
  with two right-hand sides;
* selected rows equal the corresponding rows of the full product.
"""
import mpmath as mp
import numpy as np
import pytest

import fkt_workloads as W
import oracle
from test_oracle_expansion import KERNELS, _taylor_in_t


@pytest.mark.parametrize("name,kw,f", KERNELS)
def test_rho_derivatives_against_mpmath(name, kw, f):
    """d^n/drho^n K(sqrt(rho)) by mpmath's numerical differentiation, also
    at small r / l where a chain rule through the radial derivatives would
    cancel badly."""
    mp.mp.dps = 50
    for r in (0.05, 0.3, 0.9, 2.2):
        ours = oracle.rho_derivs(name, r, 8, **kw)
        ref = [float(mp.diff(lambda q: f(mp.sqrt(q)), mp.mpf(r) ** 2, n)) for n in range(9)]
        np.testing.assert_allclose(ours, ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("name,kw,f", KERNELS)
@pytest.mark.parametrize("d", [3, 4, 5])
def test_cartesian_pair_equals_taylor_polynomial(name, kw, f, d):
    mp.mp.dps = 40
    rng = np.random.default_rng(300 + d)
    for p in (0, 1, 3, 6, 8):
        rp = rng.standard_normal(d); rp *= rng.uniform(0.1, 0.6) / np.linalg.norm(rp)
        r = rng.standard_normal(d); r *= rng.uniform(1.0, 2.0) / np.linalg.norm(r)
        ours = oracle.cart_pair(d, p, name, rp, r, **kw)
        ref = _taylor_in_t(f, rp, r, p)
        assert abs(ours - ref) <= 1e-12 * max(1.0, abs(ref)), (name, d, p, ours, ref)


CASES = [("gaussian", dict(lengthscale=0.15), 3, 5, 0.5), ("matern32", dict(lengthscale=0.1), 3, 6, 0.4),
         ("power", dict(shape=1.0), 3, 6, 0.5), ("matern52", dict(lengthscale=0.3), 4, 8, 0.4),
         ("ratquad", dict(lengthscale=0.2, shape=1.0), 4, 4, 0.6), ("exponential", dict(lengthscale=0.3), 5, 4, 0.5),
         ("cauchy", dict(lengthscale=0.2), 5, 3, 0.6)]


@pytest.mark.parametrize("name,kw,d,p,theta", CASES)
def test_factorised_equals_pairwise_algorithm1(name, kw, d, p, theta):
    n = 1500 if d == 3 else 1200
    X = W.uniform_cube(n, d, 900 + d)
    x = W.normal_rhs(n, 2, 901)
    T = oracle.Tree(X, 48)
    z1 = oracle.fkt_alg1(T, x, name, theta, p, **kw)
    z2 = oracle.fkt_cart(T, x, name, theta, p, **kw)
    far = sum(c.sum() for c in T.counts(theta)[1:2])
    assert far > 0, "the case must exercise the far field"
    err = np.abs(z1 - z2).max() / np.abs(z1).max()
    assert err <= 1e-13, err


def test_selected_rows_equal_full_product():
    X = W.gaussian_mixture(2000, 4, 5, 0.15, 7)
    x = W.normal_rhs(2000, 1, 8)
    T = oracle.Tree(X, 64)
    z = oracle.fkt_cart(T, x, "matern52", 0.45, 6, lengthscale=0.3)
    tg = W.subsample(2000, 37, 9)
    zr = oracle.fkt_cart(T, x, "matern52", 0.45, 6, targets=tg, lengthscale=0.3)
    np.testing.assert_array_equal(zr, z[tg])
