"""Learned per-leaf spectral preconditioner: plain FP64 CPU reference.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/`` may
use it. Shares no code with the HIP path.

Not part of the paper (the paper solves Gaussian-process systems through
kernel MVMs only, Sec. 5.3 and eq. gp_posterior); it is the preconditioner
this project adds for CG on A = K~ + sigma2 I. Definitions:

* leaf block  A_l = K(X_l, X_l) + sigma2 I = V_l^T diag(lam_l) V_l
  (``numpy.linalg.eigh``; rows of V_l are eigenvectors, lam ascending);
* features of eigenvalue i of leaf l (m points):
  [log(lam_i / sigma2) / 8, log(lam_max / sigma2) / 8, m / leaf_size, (i + 1/2) / m];
* network (per feature row f): h1 = tanh(f W1 + b1), h2 = tanh(h1 W2 + b2),
  o = h2 . w3 + b3;
* filter   h_{l,i} = exp(o_{l,i}) / lam_{l,i},  M_l = V_l^T diag(h_l) V_l;
* loss     L = (1/B) sum_b min_a |a A M v_b - v_b|^2 / |v_b|^2, the optimal
  a_b = <u_b, v_b> / |u_b|^2 with u_b = A M v_b (PCG does not see the scale
  of M, so neither does L; without the minimisation over a the loss is
  lowered by shrinking M towards zero, which changes no CG iterate);
* gradient through the chain rule with A taken as symmetric (a_b is
  stationary, so it is held fixed): dL/dw_b = (2 a_b / (B |v_b|^2)) A
  (a_b A M v_b - v_b), dL/dh_{l,i} = sum_b (V_l dL/dw_b)_i (V_l v_b)_i,
  dL/do = h dL/dh, then back through the MLP.

Two-level form (``nystrom_factor``, ``two_level_matrix``): with landmark
points J, L = K(X, X_J) chol(K(X_J, X_J) + sigma2 I)^-T approximates K by
L L^T; the leaf blocks become the residual blocks A_l - L_l L_l^T and the
preconditioner is P = (L L^T + D)^-1 with D^-1 the block filter above, taken
here by its definition as a dense inverse (small n).

The parameter vector is ordered W1 [4][256], b1, W2 [256][256], b2, w3, b3.
Pins (tests/test_oracle_learned.py): with o = 0 the filter is the exact
inverse of every leaf block (block-Jacobi); the loss has the closed form of
two single-point leaves and is exactly 0 for one leaf holding every point
(one-level, and two-level, where P = (L L^T + A - L L^T)^-1 = A^-1); the
analytic gradient matches central differences of L when A is an exactly
symmetric matrix, in the one-level and the two-level form; the gradient of
the condition-number objective (``cond_grad``) matches central differences
of log kappa from dense eigenvalues, and its Lanczos estimate
(``cond_grad_lanczos``, the device's algorithm) matches ``cond_grad`` when
the Lanczos run is long enough to resolve the extreme eigenpairs.
"""
from __future__ import annotations

import numpy as np

from . import dense_mvm

H = 256
F = 4
SIZES = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", ())]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAMS,)
    out, k = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = theta[k:k + size].reshape(shape)
        k += size
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.ravel(np.asarray(p[name], dtype=np.float64)) for name, _ in SIZES])


def leaf_ranges(tree):
    """(start, end) tree positions of the leaves, in preorder."""
    return [(int(tree.start[b]), int(tree.end[b])) for b in range(tree.nnodes) if tree.is_leaf(b)]


def leaf_block(Xl, kind, sigma2, **kw) -> np.ndarray:
    """K(X_l, X_l) + sigma2 I from the oracle's dense sum (identity columns)."""
    m = Xl.shape[0]
    A = np.zeros((m, m))
    for c0 in range(0, m, 64):
        c1 = min(m, c0 + 64)
        E = np.zeros((m, c1 - c0))
        E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
        A[:, c0:c1] = dense_mvm(Xl, E, kind, **kw)
    A = 0.5 * (A + A.T)
    return A + sigma2 * np.eye(m)


def nystrom_factor(X, landmarks, kind, sigma2, **kw) -> np.ndarray:
    """Two-level coarse factor L = K(X, X_J) chol(K(X_J, X_J) + sigma2 I)^-T
    (n x k, original order), so that K ~ L L^T (regularised Nystrom)."""
    X = np.asarray(X, dtype=np.float64)
    J = np.asarray(landmarks, dtype=np.int64)
    n, k = X.shape[0], len(J)
    KnJ = np.zeros((n, k))
    for c0 in range(0, k, 64):
        c1 = min(k, c0 + 64)
        E = np.zeros((n, c1 - c0))
        E[J[c0:c1], np.arange(c1 - c0)] = 1.0
        KnJ[:, c0:c1] = dense_mvm(X, E, kind, **kw)
    KJJ = KnJ[J]
    Lc = np.linalg.cholesky(0.5 * (KJJ + KJJ.T) + sigma2 * np.eye(k))
    return np.linalg.solve(Lc, KnJ.T).T


def leaf_spectra(tree, X, kind, sigma2, leaf_size, coarse=None, **kw):
    """Per leaf: dict(idx = original indices, lam, V (rows), feat [m][4]);
    with the coarse factor L (n x k), of the residual blocks
    K_ll + sigma2 I - L_l L_l^T."""
    X = np.asarray(X, dtype=np.float64)
    out = []
    for s, e in leaf_ranges(tree):
        idx = tree.perm[s:e].copy()
        A = leaf_block(X[idx], kind, sigma2, **kw)
        if coarse is not None:
            A = A - coarse[idx] @ coarse[idx].T
            A = 0.5 * (A + A.T)
        lam, U = np.linalg.eigh(A)
        m = e - s
        feat = np.stack([np.log(lam / sigma2) / 8.0, np.full(m, np.log(lam[-1] / sigma2) / 8.0),
                         np.full(m, m / leaf_size), (np.arange(m) + 0.5) / m], axis=1)
        out.append(dict(idx=idx, lam=lam, V=U.T.copy(), feat=feat, A=A))
    return out


def mlp_forward(theta, feat):
    p = unpack(theta)
    h1 = np.tanh(feat @ p["W1"] + p["b1"])
    h2 = np.tanh(h1 @ p["W2"] + p["b2"])
    o = h2 @ p["w3"] + p["b3"]
    return o, (feat, h1, h2)


def mlp_backward(theta, cache, go) -> np.ndarray:
    """Gradient of sum_s go[s] o[s] with respect to theta."""
    p = unpack(theta)
    feat, h1, h2 = cache
    d2 = np.outer(go, p["w3"]) * (1.0 - h2 ** 2)
    d1 = (d2 @ p["W2"].T) * (1.0 - h1 ** 2)
    g = dict(W1=feat.T @ d1, b1=d1.sum(0), W2=h1.T @ d2, b2=d2.sum(0), w3=h2.T @ go, b3=np.sum(go))
    return pack(g)


def filters(spectra, theta):
    """h for every leaf (list of arrays) and the MLP cache over all leaves."""
    feat = np.concatenate([L["feat"] for L in spectra], axis=0)
    o, cache = mlp_forward(theta, feat)
    hs, k = [], 0
    for L in spectra:
        m = len(L["lam"])
        hs.append(np.exp(o[k:k + m]) / L["lam"])
        k += m
    return hs, cache


def apply_filter(spectra, hs, v) -> np.ndarray:
    """M v for v (n x B) in the original order."""
    v = np.asarray(v, dtype=np.float64)
    w = np.zeros_like(v)
    for L, h in zip(spectra, hs):
        c = L["V"] @ v[L["idx"]]
        w[L["idx"]] = L["V"].T @ (h[:, None] * c)
    return w


def two_level_matrix(spectra, hs, L) -> np.ndarray:
    """P = (L L^T + D)^-1 with D^-1 = blockdiag(V_l^T diag(h_l) V_l), as a
    dense n x n matrix (small n): the two-level preconditioner by its
    definition (the device applies it through the Woodbury identity)."""
    n = L.shape[0]
    D = np.zeros((n, n))
    for Sl, h in zip(spectra, hs):
        ix = Sl["idx"]
        D[np.ix_(ix, ix)] = Sl["V"].T @ np.diag(1.0 / h) @ Sl["V"]
    P = np.linalg.inv(L @ L.T + D)
    return 0.5 * (P + P.T)


def cond_grad(spectra, theta, A, coarse=None):
    """(kappa, d log kappa / d theta) of the preconditioned operator P A, by
    the dense generalized eigenproblem A u = lam P^-1 u (small n): with
    u^T P^-1 u = 1, d lam / d h_i = lam (V u)_i^2 / h_i^2 because P^-1 =
    L L^T + D(h) and dD = V^T diag(-dh / h^2) V; so d log kappa / d o_i =
    (V u_max)_i^2 / h_i - (V u_min)_i^2 / h_i, then back through the MLP."""
    import scipy.linalg
    hs, cache = filters(spectra, theta)
    n = sum(len(Sl["lam"]) for Sl in spectra)
    D = np.zeros((n, n))
    for Sl, h in zip(spectra, hs):
        ix = Sl["idx"]
        D[np.ix_(ix, ix)] = Sl["V"].T @ np.diag(1.0 / h) @ Sl["V"]
    Pinv = D if coarse is None else coarse @ coarse.T + D
    lam, U = scipy.linalg.eigh(A, 0.5 * (Pinv + Pinv.T))
    umax, umin = U[:, -1], U[:, 0]
    go = []
    for Sl, h in zip(spectra, hs):
        a = Sl["V"] @ umax[Sl["idx"]]
        b = Sl["V"] @ umin[Sl["idx"]]
        go.append((a * a - b * b) / h)
    return float(lam[-1] / lam[0]), mlp_backward(theta, cache, np.concatenate(go))


def cond_grad_lanczos(spectra, theta, op, b, T, coarse=None):
    """The device's estimate of cond_grad, step by step: T PCG iterations
    from zero on b with the current preconditioner P (dense here), the
    Lanczos tridiagonal of P A from the step lengths (diagonal 1/alpha_j +
    beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j), the Ritz
    vectors of its extreme eigenvalues from the Lanczos vectors (-1)^j z_j /
    sqrt(r_j . z_j), and the gradient formula of cond_grad with them.
    op(x) = A x for a vector x."""
    hs, cache = filters(spectra, theta)
    n = sum(len(Sl["lam"]) for Sl in spectra)
    if coarse is None:
        Pm = np.zeros((n, n))
        for Sl, h in zip(spectra, hs):
            Pm[np.ix_(Sl["idx"], Sl["idx"])] = Sl["V"].T @ np.diag(h) @ Sl["V"]
    else:
        Pm = two_level_matrix(spectra, hs, coarse)
    r = np.array(b, dtype=np.float64)
    z = Pm @ r
    p = z.copy()
    rho = r @ z
    Z, al, be = [z / np.sqrt(rho)], [], []
    for j in range(T):
        q = op(p)
        a = rho / (p @ q)
        r = r - a * q
        z = Pm @ r
        rn = r @ z
        al.append(a)
        be.append(rn / rho)
        if j + 1 < T:
            Z.append((-1.0) ** (j + 1) * z / np.sqrt(rn))
        p = z + (rn / rho) * p
        rho = rn
    Tm = np.zeros((T, T))
    for j in range(T):
        Tm[j, j] = 1.0 / al[j] + (be[j - 1] / al[j - 1] if j else 0.0)
        if j + 1 < T:
            Tm[j, j + 1] = Tm[j + 1, j] = np.sqrt(be[j]) / al[j]
    w, S = np.linalg.eigh(Tm)
    Z = np.array(Z)
    umax, umin = S[:, -1] @ Z, S[:, 0] @ Z
    go = []
    for Sl, h in zip(spectra, hs):
        a = Sl["V"] @ umax[Sl["idx"]]
        c = Sl["V"] @ umin[Sl["idx"]]
        go.append((a * a - c * c) / h)
    return float(w[-1] / w[0]), mlp_backward(theta, cache, np.concatenate(go))


def loss_grad(spectra, theta, v, op, coarse=None):
    """(L, dL/dtheta) for the batch v (n x B); op(x) = A x for n x B x. With
    the coarse factor L the preconditioner is the two-level P(h) =
    (L L^T + D)^-1, D^-1 = M = blockdiag filter; then dP = (P D) dM (D P)
    (the derivative of the inverse), so the spectral projections of v and
    of the back-propagated residual are taken after D P."""
    v = np.asarray(v, dtype=np.float64)
    if v.ndim == 1:
        v = v[:, None]
    B = v.shape[1]
    hs, cache = filters(spectra, theta)
    if coarse is None:
        w = apply_filter(spectra, hs, v)
        pre = lambda x: x
    else:
        P = two_level_matrix(spectra, hs, coarse)
        w = P @ v
        Dm = np.linalg.inv(P) - coarse @ coarse.T     # D = M^-1
        pre = lambda x: Dm @ (P @ x)
    u = op(w)
    vv = np.sum(v * v, axis=0)
    a = np.sum(u * v, axis=0) / np.sum(u * u, axis=0)
    r = a[None, :] * u - v
    loss = float(np.mean(np.sum(r * r, axis=0) / vv))
    g = op(r) * (2.0 * a / (B * vv))[None, :]
    vp, gp = pre(v), pre(g)
    go = []
    for L, h in zip(spectra, hs):
        c = L["V"] @ vp[L["idx"]]
        q = L["V"] @ gp[L["idx"]]
        go.append(h * np.sum(c * q, axis=1))
    return loss, mlp_backward(theta, cache, np.concatenate(go))
