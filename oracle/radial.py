"""Exact compression of the radial expansion (Appendix A.4, eq. f_g).

TEST INFRASTRUCTURE ONLY. Part of the CPU oracle: only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it.

For a kernel with K'(r) = q(r) K(r), q a Laurent polynomial, every
derivative is K^(m) = K P_m with P_0 = 1 and P_{m+1} = P_m' + q P_m (Laurent
polynomials). The order-p radial function of harmonic degree k is then

    Kk(r', r) = sum_j r'^j F_kj(r),   F_kj(r) = K(r) L_j(r),
    L_j(r) = r^-j ( [j = 0] + sum_{m=1..j} Tbar_{k,j,m} P_m(r) r^m ),

over j = k, k+2, ..., <= p (Appendix A.2, eq. finaltrunc with the
derivatives of Lemma A.2). The L_j are Laurent polynomials with rational
coefficients, so the smallest R_k of eq. (f_g) is the rank of their
coefficient matrix over the rationals; everything here is computed with
``fractions.Fraction``, so ranks and coefficients are exact.

The decomposition kept is the interpolative one: the first n of the L_j
(n = the rank) are the functions F_ki, and every other L_j is written
exactly as sum_i c_ji L_{k+2i}, which turns into the G_ki(r') as the
combinations of r'^j. A kernel K(r / l) has the same L_j in u = r / l.
"""
from __future__ import annotations

from fractions import Fraction

from .coeffs import Tbar, alpha_of

# q of K' = q K, as {power: coefficient}, in the scaled variable u = r / l
# (u = r for the scale-free powers)
LAURENT_Q = {
    "power1": {-1: Fraction(-1)},               # 1/r
    "power2": {-1: Fraction(-2)},               # 1/r^2
    "power3": {-1: Fraction(-3)},               # 1/r^3
    "exponential": {0: Fraction(-1)},           # e^-u
    "exp_over_r": {-1: Fraction(-1), 0: Fraction(-1)},   # e^-u / u
    "r_exp": {-1: Fraction(1), 0: Fraction(-1)},         # u e^-u
    "gaussian": {1: Fraction(-1)},              # e^(-u^2 / 2)
    "exp_inv_r": {-2: Fraction(1)},             # e^(-1/u)
    "exp_inv_r2": {-3: Fraction(2)},            # e^(-1/u^2)
}


def _mul(a, b):
    out = {}
    for i, x in a.items():
        for j, y in b.items():
            out[i + j] = out.get(i + j, Fraction(0)) + x * y
    return {e: v for e, v in out.items() if v != 0}


def _add(a, b):
    out = dict(a)
    for e, v in b.items():
        out[e] = out.get(e, Fraction(0)) + v
    return {e: v for e, v in out.items() if v != 0}


def _deriv(a):
    return {e - 1: v * e for e, v in a.items() if e != 0}


def derivative_polys(q, mmax: int):
    """[P_0, ..., P_mmax] with K^(m) = K P_m (Laurent dicts)."""
    P = [{0: Fraction(1)}]
    for _ in range(mmax):
        P.append(_add(_deriv(P[-1]), _mul(q, P[-1])))
    return P


def radial_rows(q, d: int, k: int, p: int):
    """[L_j for j = k, k+2, ..., <= p] as Laurent dicts (see module doc)."""
    al = alpha_of(d)
    P = derivative_polys(q, p)
    rows = []
    for j in range(k, p + 1, 2):
        L = {0: Fraction(1)} if j == 0 else {}
        for m in range(1, j + 1):
            t = Tbar(k, j, m, al)
            if t != 0:
                L = _add(L, _mul(P[m], {m: t}))
        rows.append({e - j: v for e, v in L.items()})
    return rows


def _matrix(rows):
    cols = sorted({e for r in rows for e in r})
    return [[r.get(c, Fraction(0)) for c in cols] for r in rows]


def exact_rank(rows) -> int:
    """Rank over the rationals (Gaussian elimination on exact fractions)."""
    M = _matrix(rows)
    rk = 0
    ncol = len(M[0]) if M else 0
    for c in range(ncol):
        piv = next((i for i in range(rk, len(M)) if M[i][c] != 0), None)
        if piv is None:
            continue
        M[rk], M[piv] = M[piv], M[rk]
        for i in range(len(M)):
            if i != rk and M[i][c] != 0:
                f = M[i][c] / M[rk][c]
                M[i] = [a - f * b for a, b in zip(M[i], M[rk])]
        rk += 1
    return rk


def ranks(q, d: int, p: int):
    """R_k of eq. (f_g) for k = 0..p."""
    return [exact_rank(radial_rows(q, d, k, p)) for k in range(p + 1)]


def radial_function(q, d: int, k: int, p: int):
    """Kk(r', r) / K(r) as {(power of r, power of r'): coefficient}."""
    out = {}
    for idx, L in enumerate(radial_rows(q, d, k, p)):
        j = k + 2 * idx
        for e, v in L.items():
            out[(e, j)] = out.get((e, j), Fraction(0)) + v
    return {key: v for key, v in out.items() if v != 0}


def interpolative(q, d: int, k: int, p: int, n: int):
    """Exact coefficients c[jj][i] with L_{k+2jj} = sum_{i<n} c[jj][i] L_{k+2i}
    for every jj, or None when the first n rows do not span all rows or are
    dependent. Solved on n columns where the first n rows are independent."""
    rows = radial_rows(q, d, k, p)
    n = min(n, len(rows))
    lead = rows[:n]
    if exact_rank(lead) != n or exact_rank(rows) != n:
        return None
    cols = sorted({e for r in rows for e in r})
    # columns where the leading rows are independent (greedy)
    chosen = []
    for c in cols:
        trial = chosen + [c]
        sub = [{cc: r.get(cc, Fraction(0)) for cc in trial} for r in lead]
        if exact_rank(sub) == len(trial):
            chosen = trial
        if len(chosen) == n:
            break
    A = [[lead[i].get(c, Fraction(0)) for i in range(n)] for c in chosen]  # n x n, A c = b
    coef = []
    for r in rows:
        b = [r.get(c, Fraction(0)) for c in chosen]
        coef.append(_solve(A, b))
    return coef


def _solve(A, b):
    n = len(b)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        piv = next(i for i in range(c, n) if M[i][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for i in range(n):
            if i != c and M[i][c] != 0:
                f = M[i][c] / M[c][c]
                M[i] = [a - f * x for a, x in zip(M[i], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def expansion_size(d: int, rk):
    """Size of the compressed expansion: sum_k |H_k| R_k, with |H_k| the
    number of degree-k harmonics in d dimensions (Appendix A.3)."""
    from math import comb
    total = 0
    for k, r in enumerate(rk):
        hk = comb(k + d - 1, d - 1) - (comb(k + d - 3, d - 1) if k >= 2 else 0)
        total += hk * r
    return total
