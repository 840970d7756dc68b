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


def test_loss_closed_form_two_single_point_leaves():
    """Two leaves of one point each: A = [[a, c], [c, a]] with a = K(0) +
    sigma2 and c = K(r12). With any outputs o, M = diag(e^o1 / a, e^o2 / a),
    so for v = e_1, u = A M v is parallel to (1, c / a) and the loss, the
    squared sine of the angle between u and v, is t^2 / (1 + t^2) with
    t = c / a; for v = (1, 1) and o1 = o2, u is parallel to v and L = 0."""
    X = np.array([[0.1, 0.2, 0.3], [0.35, 0.1, 0.4]])
    T = oracle.Tree(X, 1)
    sig2, ell = 0.3, 0.4
    sp = LR.leaf_spectra(T, X, "gaussian", sig2, 1, lengthscale=ell)
    assert len(sp) == 2
    r = np.linalg.norm(X[0] - X[1])
    a, c = 1.0 + sig2, np.exp(-r * r / (2 * ell * ell))
    A = np.array([[a, c], [c, a]])
    op = lambda x: A @ x
    rng = np.random.default_rng(4)
    theta = rng.normal(0.0, 0.3, LR.NPARAMS)
    t = c / a
    L1, _ = LR.loss_grad(sp, theta, np.array([[1.0], [0.0]]), op)
    assert abs(L1 - t * t / (1 + t * t)) <= 1e-14
    p = LR.unpack(theta)
    p["w3"][:] = 0.0  # o = b3 for every eigenvalue
    p["b3"] = np.array(0.7)
    L2, g2 = LR.loss_grad(sp, LR.pack(p), np.array([[1.0], [1.0]]), op)
    assert L2 <= 1e-28 and np.abs(g2).max() <= 1e-13


def test_single_leaf_block_jacobi_is_exact():
    """One leaf holding every point and o = 0: M is the inverse of the whole
    operator, so A M v = v for every v: loss 0 and (a minimum) gradient 0."""
    X = W.gaussian_mixture(60, 4, 2, 0.2, 5)
    T = oracle.Tree(X, 60)
    sig2 = 1e-2
    sp = LR.leaf_spectra(T, X, "matern52", sig2, 60, lengthscale=0.3)
    A = LR.leaf_block(X, "matern52", sig2, lengthscale=0.3)
    theta = np.random.default_rng(6).normal(0.0, 0.3, LR.NPARAMS)
    p = LR.unpack(theta)
    p["w3"][:] = 0.0
    p["b3"] = np.zeros(())
    v = np.random.default_rng(7).normal(size=(60, 2))
    L, g = LR.loss_grad(sp, LR.pack(p), v, lambda x: A @ x)
    assert L <= 1e-16 and np.abs(g).max() <= 1e-9


def test_two_level_single_leaf_is_exact():
    """One leaf and o = 0: D is the residual block A - L L^T itself, so
    P = (L L^T + A - L L^T)^-1 = A^-1 and the loss is 0."""
    X = W.gaussian_mixture(80, 4, 2, 0.2, 8)
    T = oracle.Tree(X, 80)
    sig2 = 1e-2
    Lf = LR.nystrom_factor(X, W.subsample(80, 12, 9), "matern52", sig2, lengthscale=0.3)
    sp = LR.leaf_spectra(T, X, "matern52", sig2, 80, coarse=Lf, lengthscale=0.3)
    A = LR.leaf_block(X, "matern52", sig2, lengthscale=0.3)
    p = LR.unpack(np.random.default_rng(10).normal(0.0, 0.3, LR.NPARAMS))
    p["w3"][:] = 0.0
    p["b3"] = np.zeros(())
    v = np.random.default_rng(11).normal(size=(80, 2))
    L, g = LR.loss_grad(sp, LR.pack(p), v, lambda x: A @ x, coarse=Lf)
    assert L <= 1e-14 and np.abs(g).max() <= 1e-7


def test_nystrom_factor_reproduces_landmark_columns():
    """L L^T on the landmark columns equals K(X, X_J) (K_JJ + s2 I)^-1 K_JJ,
    and the residual K + s2 I - L L^T is positive definite (>= s2 I)."""
    X = W.gaussian_mixture(150, 3, 3, 0.2, 12)
    J = W.subsample(150, 20, 13)
    sig2 = 0.05
    Lf = LR.nystrom_factor(X, J, "gaussian", sig2, lengthscale=0.3)
    D = np.linalg.norm(X[:, None] - X[None], axis=-1)
    K = np.exp(-D ** 2 / (2 * 0.3 ** 2))
    ref = K[:, J] @ np.linalg.solve(K[np.ix_(J, J)] + sig2 * np.eye(len(J)), K[J][:, J])
    assert np.abs(Lf @ Lf[J].T - ref).max() <= 1e-12
    assert np.linalg.eigvalsh(K + sig2 * np.eye(150) - Lf @ Lf.T).min() >= sig2 * (1 - 1e-9)


def test_two_level_gradient_matches_central_differences():
    X, T = _small(n=120, leaf=40, seed=14)
    sig2 = 5e-2
    Lf = LR.nystrom_factor(X, W.subsample(120, 16, 15), "matern52", sig2, lengthscale=0.3)
    sp = LR.leaf_spectra(T, X, "matern52", sig2, 40, coarse=Lf, lengthscale=0.3)
    A = LR.leaf_block(X, "matern52", sig2, lengthscale=0.3)
    op = lambda x: A @ x
    rng = np.random.default_rng(16)
    theta = rng.normal(0.0, 0.2, LR.NPARAMS)
    v = rng.normal(size=(X.shape[0], 2))
    L0, g = LR.loss_grad(sp, theta, v, op, coarse=Lf)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in LR.SIZES])
    coords = []
    for b in range(len(LR.SIZES)):
        coords += list(rng.integers(offs[b], offs[b + 1], size=2))
    eps = 1e-6
    for k in coords:
        tp = theta.copy(); tp[k] += eps
        tm = theta.copy(); tm[k] -= eps
        fd = (LR.loss_grad(sp, tp, v, op, coarse=Lf)[0] - LR.loss_grad(sp, tm, v, op, coarse=Lf)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-7 * np.abs(g).max(), (k, fd, g[k])
    assert L0 > 0.0


@pytest.mark.parametrize("two_level", [False, True])
def test_cond_gradient_matches_central_differences(two_level):
    """d log kappa(P A) / d theta against central differences of log kappa
    from scipy's dense generalized eigenvalues (one- and two-level P)."""
    import scipy.linalg
    X, T = _small(n=120, leaf=40, seed=18)
    sig2 = 5e-2
    Lf = LR.nystrom_factor(X, W.subsample(120, 12, 19), "matern52", sig2, lengthscale=0.3) if two_level else None
    sp = LR.leaf_spectra(T, X, "matern52", sig2, 40, coarse=Lf, lengthscale=0.3)
    A = LR.leaf_block(X, "matern52", sig2, lengthscale=0.3)
    rng = np.random.default_rng(20)
    theta = rng.normal(0.0, 0.2, LR.NPARAMS)

    def logk(th):
        hs, _ = LR.filters(sp, th)
        D = np.zeros_like(A)
        for Sl, h in zip(sp, hs):
            D[np.ix_(Sl["idx"], Sl["idx"])] = Sl["V"].T @ np.diag(1.0 / h) @ Sl["V"]
        Pinv = D if Lf is None else Lf @ Lf.T + D
        lam = scipy.linalg.eigvalsh(A, 0.5 * (Pinv + Pinv.T))
        return np.log(lam[-1] / lam[0])

    kappa, g = LR.cond_grad(sp, theta, A, coarse=Lf)
    assert abs(np.log(kappa) - logk(theta)) <= 1e-10
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in LR.SIZES])
    coords = []
    for b in range(len(LR.SIZES)):
        coords += list(rng.integers(offs[b], offs[b + 1], size=2))
    eps = 1e-6
    for k in coords:
        tp = theta.copy(); tp[k] += eps
        tm = theta.copy(); tm[k] -= eps
        fd = (logk(tp) - logk(tm)) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-5 * max(1.0, abs(g[k])) + 1e-6 * np.abs(g).max(), (k, fd, g[k])


def test_cond_lanczos_estimate_converges_to_exact():
    """PCG run as long as the problem (n = 120 steps) resolves the extreme
    eigenpairs of P A: the Lanczos estimate equals the exact cond_grad."""
    X, T = _small(n=120, leaf=40, seed=22)
    sig2 = 0.1
    sp = LR.leaf_spectra(T, X, "gaussian", sig2, 40, lengthscale=0.4)
    A = LR.leaf_block(X, "gaussian", sig2, lengthscale=0.4)
    theta = np.random.default_rng(23).normal(0.0, 0.1, LR.NPARAMS)
    b = np.random.default_rng(24).normal(size=120)
    k_ex, g_ex = LR.cond_grad(sp, theta, A)
    k_la, g_la = LR.cond_grad_lanczos(sp, theta, lambda x: A @ x, b, 119)
    assert abs(k_la - k_ex) <= 1e-8 * k_ex
    assert np.linalg.norm(g_la - g_ex) <= 1e-6 * np.linalg.norm(g_ex)
