"""Pins of the exact radial compression (oracle/radial.py, Appendix A.4).

Against values the paper prints and closed forms:
  * Table "ranks": R_k for 1/r, 1/r^2, 1/r^3, e^-r / r, e^-r and r e^-r in
    d = 3..9 (a dash: no reduction below floor((p - k) / 2) + 1).
  * Table "exp_decomp": the two-term decomposition of e^-r for k = 0, 1, 2
    equals the oracle's radial function exactly (up to the factor
    r^(k+1) / r'^k of the paper's normalisation), at p = 7.
  * Newton kernels: 1/r^(d-2) in d = 3, 4, 5 has the Gegenbauer generating
    function as its expansion, so its radial function is r'^k / r^(k+d-2)
    exactly and R_k = 1.
The interpolative coefficients are checked by exact reconstruction.
"""
from fractions import Fraction
from math import comb

import pytest

from oracle import radial as R

# Table "ranks": kernel -> {d: R} (None for a dash)
TABLE_RANKS = {
    "power1": {3: 1, 4: None, 5: 2, 6: None, 7: 3, 8: None, 9: 4},
    "power2": {3: None, 4: 1, 5: None, 6: 2, 7: None, 8: 3, 9: None},
    "power3": {3: None, 4: None, 5: 1, 6: None, 7: 2, 8: None, 9: 3},
    "exp_over_r": {3: 1, 4: None, 5: 2, 6: None, 7: 3, 8: None, 9: 4},
    "exponential": {3: 2, 4: None, 5: 3, 6: None, 7: 4, 8: None, 9: 5},
    "r_exp": {3: 3, 4: None, 5: 4, 6: None, 7: 5, 8: None, 9: 6},
}


def _full(p):
    return [len(range(k, p + 1, 2)) for k in range(p + 1)]


@pytest.mark.parametrize("kernel", sorted(TABLE_RANKS))
def test_ranks_match_table(kernel):
    """At p = 12 (full rank 7 for k = 0, above every table entry): each
    R_k is min(table value, full), and a dash is the full rank."""
    p = 12
    full = _full(p)
    for d, want in TABLE_RANKS[kernel].items():
        got = R.ranks(R.LAURENT_Q[kernel], d, p)
        expect = full if want is None else [min(want, f) for f in full]
        assert got == expect, (kernel, d, got)


def test_gaussian_has_no_reduction():
    """The paper finds no reduction for the squared exponential."""
    for d in (3, 4, 5):
        assert R.ranks(R.LAURENT_Q["gaussian"], d, 8) == _full(8)


# Table "exp_decomp" (K = e^-r): F_ki(r) / e^-r and G_ki(r') as {power: coefficient}
EXP_F = {0: [{1: Fraction(1)}, {0: Fraction(-1, 3)}],
         1: [{2: Fraction(1)}, {1: Fraction(-1, 5), 0: Fraction(-1, 5)}],
         2: [{2: Fraction(1, 3), 3: Fraction(1, 3)},
             {1: Fraction(-1, 7), 2: Fraction(-1, 42), 3: Fraction(1, 42), 0: Fraction(-1, 7)}]}
EXP_G = {0: [{0: Fraction(1), 2: Fraction(1, 6), 4: Fraction(1, 120), 6: Fraction(1, 5040)},
             {2: Fraction(1), 4: Fraction(1, 10), 6: Fraction(1, 280)}],
         1: [{0: Fraction(1), 2: Fraction(1, 10), 4: Fraction(1, 280), 6: Fraction(1, 15120)},
             {2: Fraction(1), 4: Fraction(1, 14), 6: Fraction(1, 504)}],
         2: [{0: Fraction(1), 4: Fraction(-1, 504)}, {2: Fraction(1), 4: Fraction(1, 18)}]}


@pytest.mark.parametrize("k", [0, 1, 2])
def test_exponential_decomposition_matches_table(k):
    paper = {}
    for f, g in zip(EXP_F[k], EXP_G[k]):
        for a, x in f.items():
            for b, y in g.items():
                key = (a - k - 1, b + k)  # times r'^k / r^(k+1)
                paper[key] = paper.get(key, Fraction(0)) + x * y
    paper = {key: v for key, v in paper.items() if v != 0}
    assert R.radial_function(R.LAURENT_Q["exponential"], 3, k, 7) == paper


@pytest.mark.parametrize("d,kernel", [(3, "power1"), (4, "power2"), (5, "power3")])
def test_newton_kernel_closed_form(d, kernel):
    """1/r^(d-2) = sum_k C_k^alpha(cos) r'^k / r^(k+d-2): the radial function
    of degree k is the single term r'^k r^-(k+d-2), i.e. K(r) (r'/r)^k, for
    every p >= k."""
    for p in (4, 9):
        for k in range(p + 1):
            assert R.radial_function(R.LAURENT_Q[kernel], d, k, p) == {(-k, k): Fraction(1)}


@pytest.mark.parametrize("kernel,d,keep", [("power1", 3, 1), ("exponential", 3, 2), ("power1", 5, 2),
                                           ("exponential", 5, 3)])
def test_interpolative_reconstructs_every_row(kernel, d, keep):
    q = R.LAURENT_Q[kernel]
    for p in (2, 6, 8):
        for k in range(p + 1):
            rows = R.radial_rows(q, d, k, p)
            n = min(keep, len(rows))
            c = R.interpolative(q, d, k, p, n)
            assert c is not None
            for jj, row in enumerate(rows):
                rec = {}
                for i in range(n):
                    for e, v in rows[i].items():
                        rec[e] = rec.get(e, Fraction(0)) + c[jj][i] * v
                assert {e: v for e, v in rec.items() if v != 0} == row
                if jj < n:
                    assert c[jj] == [Fraction(int(i == jj)) for i in range(n)]


def test_expansion_size():
    """sum_k |H_k| floor((p-k)/2 + 1) = C(p+d, d) (Appendix A.3), and the
    compressed 1/r in d = 3 has (p+1)^2 terms."""
    for d in (3, 4, 5):
        for p in range(9):
            assert R.expansion_size(d, _full(p)) == comb(p + d, d)
    for p in range(9):
        assert R.expansion_size(3, R.ranks(R.LAURENT_Q["power1"], 3, p)) == (p + 1) ** 2
