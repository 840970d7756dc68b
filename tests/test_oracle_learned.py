"""Pins of the learned-preconditioner reference (oracle/learned.py).

* o = 0 (zero last layer) must give the exact inverse of every leaf block
  K_ll + sigma2 I: the block-Jacobi closed form.
* The analytic gradient must match central differences of the loss when the
  operator is an exactly symmetric matrix (the dense K + sigma2 I), for
  coordinates in every parameter block.
"""
import numpy as np
import pytest

import fkt_workloads as W
import oracle
from oracle import learned as LR


def _small(n=240, d=3, leaf=60, seed=11):
    X = W.gaussian_mixture(n, d, 4, 0.15, seed)
    return X, oracle.Tree(X, leaf)


def test_zero_output_is_block_jacobi():
    X, T = _small()
    sp = LR.leaf_spectra(T, X, "matern52", 1e-2, 60, lengthscale=0.3)
    theta = np.random.default_rng(0).normal(0.0, 0.5, LR.NPARAMS)
    p = LR.unpack(theta)
    p["w3"][:] = 0.0
    p["b3"] = np.zeros(())
    theta = LR.pack(p)
    hs, _ = LR.filters(sp, theta)
    for L, h in zip(sp, hs):
        M = L["V"].T @ np.diag(h) @ L["V"]
        assert np.abs(M @ L["A"] - np.eye(len(h))).max() < 1e-9


def test_leaf_block_is_the_kernel_matrix():
    X, T = _small(n=80, leaf=40)
    s, e = LR.leaf_ranges(T)[0]
    idx = T.perm[s:e]
    A = LR.leaf_block(X[idx], "gaussian", 0.5, lengthscale=0.2)
    D = np.linalg.norm(X[idx][:, None] - X[idx][None], axis=-1)
    assert np.allclose(A, np.exp(-D ** 2 / (2 * 0.2 ** 2)) + 0.5 * np.eye(len(idx)), rtol=1e-13, atol=1e-14)


def test_gradient_matches_central_differences():
    X, T = _small(n=200, leaf=50, seed=12)
    sig2 = 5e-2
    sp = LR.leaf_spectra(T, X, "matern52", sig2, 50, lengthscale=0.3)
    A = LR.leaf_block(X, "matern52", sig2, lengthscale=0.3)  # exactly symmetric n x n
    op = lambda x: A @ x
    rng = np.random.default_rng(1)
    theta = rng.normal(0.0, 0.2, LR.NPARAMS)
    v = rng.normal(size=(X.shape[0], 3))
    L0, g = LR.loss_grad(sp, theta, v, op)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in LR.SIZES])
    coords = []
    for b in range(len(LR.SIZES)):
        coords += list(rng.integers(offs[b], offs[b + 1], size=2))
    eps = 1e-6
    for k in coords:
        tp = theta.copy(); tp[k] += eps
        tm = theta.copy(); tm[k] -= eps
        fd = (LR.loss_grad(sp, tp, v, op)[0] - LR.loss_grad(sp, tm, v, op)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-7 * np.abs(g).max(), (k, fd, g[k])
    assert L0 > 0.0
