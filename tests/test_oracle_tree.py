"""Pins of the oracle's space-partition tree (Sec. 3.1) and near/far sets
(eq. accparam, Sec. 3.2).

The paper fixes only properties, not a shape (its Figure 1 is unavailable),
so the tree is pinned by invariants and by a brute-force re-derivation in
Python of every rule the reading fixes; the tree shape itself is "parity
unpinned" against the paper. The partition is pinned by brute force over all
(target, node) pairs from its definition.
"""
import numpy as np
import pytest

import fkt_workloads as W
import oracle


def _far(tree, b, t, theta):
    # FP64, axis order, multiply then add -- Python floats are IEEE doubles
    s = 0.0
    for a in range(tree.d):
        u = float(t[a]) - float(tree.ctr[b, a])
        s = s + u * u
    return float(tree.rho2[b]) < (theta * theta) * s


def _ancestors(tree, b):
    out = []
    while tree.parent[b] >= 0:
        b = tree.parent[b]
        out.append(b)
    return out


CASES = [
    ("cube3", lambda: W.uniform_cube(300, 3, 1), 16),
    ("cube4", lambda: W.uniform_cube(200, 4, 2), 8),
    ("gmm5", lambda: W.gaussian_mixture(250, 5, 3, 0.1, 3), 10),
    ("dups", lambda: W.clustered_duplicates(120, 3, 7, 4), 5),
    ("tiny", lambda: W.uniform_cube(3, 3, 5), 1),
]


@pytest.mark.parametrize("name,gen,leaf", CASES, ids=[c[0] for c in CASES])
def test_tree_invariants(name, gen, leaf):
    X = gen()
    T = oracle.Tree(X, leaf, max_depth=24)
    n, d = X.shape
    # the permutation is a permutation, ranges contiguous and nested
    assert sorted(T.perm.tolist()) == list(range(n))
    assert T.start[0] == 0 and T.end[0] == n
    for b in range(T.nnodes):
        pts = X[T.perm[T.start[b]:T.end[b]]]
        assert len(pts) > 0
        lo, side = T.lo[b], T.side[b]
        # points inside the (closed) box; lo is exact (a min or a split
        # plane), lo + side may round down by an ulp
        assert np.all(pts >= lo) and np.all(pts <= (lo + side) * (1 + 4e-16) + 4e-16)
        # aspect ratio <= 2
        assert side.max() <= 2 * side.min() or side.max() == 0
        # centre = box centre; rho2 = max squared distance of the node's points
        np.testing.assert_array_equal(T.ctr[b], lo + 0.5 * side)
        r2 = max(sum((p[a] - T.ctr[b, a]) ** 2 for a in range(d)) for p in pts)
        assert abs(T.rho2[b] - r2) <= 1e-15 * max(1, r2)
        kids = [c for c in T.child[b] if c >= 0]
        if not kids:
            assert T.end[b] - T.start[b] <= leaf or T.depth[b] == 24
            continue
        assert T.end[b] - T.start[b] > leaf
        # preorder, left first
        assert kids[0] == b + 1
        # children tile the parent's range
        assert T.start[kids[0]] == T.start[b] and T.end[kids[-1]] == T.end[b]
        if len(kids) == 2:
            assert T.end[kids[0]] == T.start[kids[1]]
        # one longest side halved; the best-balanced longest axis chosen
        smax = side.max()
        cand = [a for a in range(d) if side[a] == smax]
        c0 = kids[0]
        halved = [a for a in range(d) if T.side[c0, a] != side[a]]
        assert len(halved) == 1 and halved[0] in cand
        ax = halved[0]
        assert T.side[c0, ax] == 0.5 * side[ax]
        mid = lo[ax] + 0.5 * side[ax]
        scores = {a: abs(2 * int(np.sum(pts[:, a] < lo[a] + 0.5 * side[a])) - len(pts)) for a in cand}
        best = min(cand, key=lambda a: (scores[a], a))
        assert ax == best
        left = X[T.perm[T.start[b]:T.start[b] + int(np.sum(pts[:, ax] < mid))]]
        assert np.all(left[:, ax] < mid)
        # stable order inside each child
        for c in kids:
            seg = T.perm[T.start[c]:T.end[c]]
            parent_seg = T.perm[T.start[b]:T.end[b]].tolist()
            pos = [parent_seg.index(i) for i in seg]
            assert pos == sorted(pos)


@pytest.mark.parametrize("name,gen,leaf", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("theta", [0.3, 0.6, 0.9])
def test_partition_brute_force(name, gen, leaf, theta):
    """t in F_b iff far(t,b) and no ancestor of b is far; t in N_l iff l is a
    leaf and nothing on the root-to-l path is far; and for every t the far
    nodes and near leaves cover every source exactly once."""
    X = gen()
    T = oracle.Tree(X, leaf, max_depth=24)
    n = X.shape[0]
    anc = [_ancestors(T, b) for b in range(T.nnodes)]
    for t in range(n):
        far_bf = [b for b in range(T.nnodes)
                  if _far(T, b, X[t], theta) and not any(_far(T, a, X[t], theta) for a in anc[b])]
        near_bf = [b for b in range(T.nnodes) if T.is_leaf(b)
                   and not _far(T, b, X[t], theta) and not any(_far(T, a, X[t], theta) for a in anc[b])]
        fo, no = T.walk(X[t], theta)
        assert sorted(fo.tolist()) == far_bf
        assert sorted(no.tolist()) == near_bf
        cover = np.zeros(n, dtype=int)
        for b in list(fo) + list(no):
            cover[T.perm[T.start[b]:T.end[b]]] += 1
        assert np.all(cover == 1)
        # a target is never far from a node containing it; self is near
        own = [b for b in no if t in T.perm[T.start[b]:T.end[b]]]
        assert len(own) == 1
    # the root has no far set
    assert all(0 not in T.walk(X[t], theta)[0] for t in range(n))


def test_walk_visits_cfg1_tree_counts():
    """The small Gaussian workload: 2000 uniform points, leaf 128."""
    X = W.uniform_cube(2000, 3, 1001)
    T = oracle.Tree(X, 128)
    leaves = sum(T.is_leaf(b) for b in range(T.nnodes))
    assert T.nnodes == 41 and leaves == 21
