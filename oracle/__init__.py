"""CPU oracle for the Fast Kernel Transform MVM (FP64).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's ``cpu_baseline`` leg may import this package. It shares no
code with the HIP product path and never imports it.

Parts:
  * ``coeffs``   -- exact-rational tables A, B, Tbar (Appendix A.2).
  * ``radial``   -- exact ranks R_k and interpolative coefficients of the
    compressed radial expansion for K' = q K kernels (Appendix A.4).
  * ``fkt_ref.c`` -- plain C (FP64, OpenMP): dense direct sum (eq. nbody),
    the space-partition tree (Sec. 3.1), far/near sets (eq. accparam), and
    Algorithm 1 with the compressed blocks evaluated pairwise through the
    Gegenbauer form of eq. (finaltrunc) (``fkt_alg1``, ``fkt_rows``); and
    the same operator factorised through Cartesian monomial moments and the
    Taylor coefficients of the kernel about each far node's centre
    (``fkt_cart``), fast enough for every row at N = 10^6.

Every function is pinned by tests in ``tests/test_oracle_*.py`` against
values or identities that do not come from this code (see the docstrings
there). Parity of the tree *shape* against the paper is unpinned: the
paper's Figure 1 is not available and the split rule is a reading.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import coeffs

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fkt_ref.c")
LIB = os.path.join(HERE, "_fkt_ref.so")

# kernel kinds of the oracle (its own numbering)
KINDS = {"gaussian": 0, "exponential": 1, "matern32": 2, "matern52": 3,
         "ratquad": 4, "cauchy": 5, "power": 6}
SINGULAR = {"power"}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    # -O3 without -march: the library may run on another host than the one
    # that built it; no FMA contraction, so the far test is evaluated as the
    # readings state (multiply, then add)
    cmd = ["gcc", "-O3", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.ref_tree_new.restype = P
        L.ref_tree_new.argtypes = [i64, i32, P, i32, i32]
        L.ref_tree_nnodes.restype = i64
        L.ref_tree_nnodes.argtypes = [P]
        L.ref_tree_export.argtypes = [P] * 11
        L.ref_tree_free.argtypes = [P]
        L.ref_walk.restype = i32
        L.ref_walk.argtypes = [P, P, dbl, P, i64, P, P, i64, P]
        L.ref_dense.argtypes = [i64, i32, P, i32, P, P, i32, i64, P, P]
        L.ref_fkt_rows.argtypes = [P, dbl, i32, P, i32, P, P, i32, i64, P, P]
        L.ref_fkt_alg1.argtypes = [P, dbl, i32, P, i32, P, P, i32, P]
        L.ref_expansion.restype = dbl
        L.ref_expansion.argtypes = [i32, i32, P, i32, P, P, P]
        L.ref_kernel_derivs.argtypes = [i32, P, dbl, i32, P]
        L.ref_kernel_value.restype = dbl
        L.ref_kernel_value.argtypes = [i32, P, dbl]
        L.ref_counts.argtypes = [P, dbl, P, P, P, P]
        L.ref_fkt_cart.argtypes = [P, dbl, i32, i32, P, P, i32, i64, P, P]
        L.ref_cart_pair.restype = dbl
        L.ref_cart_pair.argtypes = [i32, i32, i32, P, P, P]
        L.ref_rho_derivs.argtypes = [i32, i32, P, dbl, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def kernel_params(kind: str, lengthscale: float = 1.0, shape: float = 1.0, variance: float = 1.0):
    """(kind id, parameter vector [lengthscale, shape, variance]).

    shape is alpha for the rational quadratic and the exponent q for r^-q.
    """
    return KINDS[kind], np.array([lengthscale, shape, variance], dtype=np.float64)


def kernel_derivs(kind: str, r: float, p: int, **kw) -> np.ndarray:
    k, prm = kernel_params(kind, **kw)
    out = np.zeros(p + 1)
    lib().ref_kernel_derivs(k, _ptr(prm), float(r), p, _ptr(out))
    return out


def dense_mvm(X, x, kind: str, targets=None, **kw) -> np.ndarray:
    """O1: z[t] = sum_j K(|X_t - X_j|) x_j for the given targets (all if None)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    n, d = X.shape
    nrhs = x.shape[1]
    assert nrhs <= 64
    tg = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    out = np.zeros((len(tg), nrhs))
    k, prm = kernel_params(kind, **kw)
    lib().ref_dense(n, d, _ptr(X), k, _ptr(prm), _ptr(x), nrhs, len(tg), _ptr(tg), _ptr(out))
    return out


class Tree:
    """The oracle's binary space-partition tree (owns a copy of the points)."""

    def __init__(self, X, leaf_size: int, max_depth: int = 48):
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.n, self.d = self.X.shape
        self.leaf_size = leaf_size
        self.h = lib().ref_tree_new(self.n, self.d, _ptr(self.X), leaf_size, max_depth)
        nn = lib().ref_tree_nnodes(self.h)
        self.nnodes = nn
        self.perm = np.zeros(self.n, dtype=np.int64)
        self.lo = np.zeros((nn, self.d)); self.side = np.zeros((nn, self.d)); self.ctr = np.zeros((nn, self.d))
        self.rho2 = np.zeros(nn)
        self.start = np.zeros(nn, dtype=np.int64); self.end = np.zeros(nn, dtype=np.int64)
        self.child = np.zeros((nn, 2), dtype=np.int64); self.parent = np.zeros(nn, dtype=np.int64)
        self.depth = np.zeros(nn, dtype=np.int32)
        lib().ref_tree_export(self.h, *[_ptr(a) for a in (self.perm, self.lo, self.side, self.ctr, self.rho2,
                                                          self.start, self.end, self.child, self.parent, self.depth)])

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ref_tree_free(self.h)
                self.h = None
        except Exception:
            pass

    def is_leaf(self, b):
        return self.child[b, 0] < 0 and self.child[b, 1] < 0

    def walk(self, t, theta):
        """(far node ids, near leaf ids) of target point t, in visit order."""
        t = np.ascontiguousarray(t, dtype=np.float64)
        fo = np.zeros(self.nnodes, dtype=np.int64); no = np.zeros(self.nnodes, dtype=np.int64)
        nf = ctypes.c_int64(0); nq = ctypes.c_int64(0)
        rc = lib().ref_walk(self.h, _ptr(t), float(theta), _ptr(fo), self.nnodes, ctypes.byref(nf),
                            _ptr(no), self.nnodes, ctypes.byref(nq))
        assert rc == 0
        return fo[:nf.value].copy(), no[:nq.value].copy()

    def counts(self, theta):
        """Per-target (far nodes, far points, near leaves, near points)."""
        out = [np.zeros(self.n, dtype=np.int64) for _ in range(4)]
        lib().ref_counts(self.h, float(theta), *[_ptr(a) for a in out])
        return tuple(out)


def tbar(d: int, p: int) -> np.ndarray:
    return np.ascontiguousarray(coeffs.tbar_table(d, p))


def expansion(d: int, p: int, kind: str, rp, r, Tb=None, **kw) -> float:
    """Truncated expansion K~_p(r', r) about a centre at the origin."""
    Tb = tbar(d, p) if Tb is None else Tb
    k, prm = kernel_params(kind, **kw)
    rp = np.ascontiguousarray(rp, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    return lib().ref_expansion(d, p, _ptr(Tb), k, _ptr(prm), _ptr(rp), _ptr(r))


def fkt_alg1(tree: Tree, x, kind: str, theta: float, p: int, **kw) -> np.ndarray:
    """O2 (Algorithm 1, node-major) applied to x; output in original order."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    Tb = tbar(tree.d, p)
    k, prm = kernel_params(kind, **kw)
    out = np.zeros((tree.n, x.shape[1]))
    lib().ref_fkt_alg1(tree.h, float(theta), p, _ptr(Tb), k, _ptr(prm), _ptr(x), x.shape[1], _ptr(out))
    return out


def fkt_rows(tree: Tree, x, kind: str, theta: float, p: int, targets, **kw) -> np.ndarray:
    """O2, selected output rows only (original indices)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    tg = np.ascontiguousarray(targets, dtype=np.int64)
    Tb = tbar(tree.d, p)
    k, prm = kernel_params(kind, **kw)
    out = np.zeros((len(tg), x.shape[1]))
    lib().ref_fkt_rows(tree.h, float(theta), p, _ptr(Tb), k, _ptr(prm), _ptr(x), x.shape[1], len(tg),
                       _ptr(tg), _ptr(out))
    return out


def fkt_cart(tree: Tree, x, kind: str, theta: float, p: int, targets=None, **kw) -> np.ndarray:
    """O2b: the FKT operator at the same tree, partition and truncation,
    factorised through Cartesian moments (Theorem 3.1 read as the degree-p
    Taylor polynomial about the node centre); rows for the given original
    indices, or all rows in original order."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    k, prm = kernel_params(kind, **kw)
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = tree.n if tg is None else len(tg)
    out = np.zeros((nt, x.shape[1]))
    lib().ref_fkt_cart(tree.h, float(theta), p, k, _ptr(prm), _ptr(x), x.shape[1], nt,
                       None if tg is None else _ptr(tg), _ptr(out))
    return out


def cart_pair(d: int, p: int, kind: str, rp, r, **kw) -> float:
    """Cartesian (Taylor) form of the truncated expansion for one pair."""
    k, prm = kernel_params(kind, **kw)
    rp = np.ascontiguousarray(rp, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    return lib().ref_cart_pair(d, p, k, _ptr(prm), _ptr(rp), _ptr(r))


def rho_derivs(kind: str, r: float, p: int, **kw) -> np.ndarray:
    """d^n/drho^n K(sqrt(rho)) at rho = r^2, n = 0..p."""
    k, prm = kernel_params(kind, **kw)
    out = np.zeros(p + 1)
    lib().ref_rho_derivs(p, k, _ptr(prm), float(r), _ptr(out))
    return out


def rel_err(z, zref) -> float:
    """||z - zref||_2 / ||zref||_2 over all entries (the paper never defines it)."""
    z = np.asarray(z, dtype=np.float64); zref = np.asarray(zref, dtype=np.float64)
    return float(np.linalg.norm(z - zref) / np.linalg.norm(zref))
