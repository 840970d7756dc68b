"""Exact-rational coefficient tables of the generalised multipole expansion.

TEST INFRASTRUCTURE ONLY. This module is part of the CPU oracle: only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
it. The product path never does.

Everything here follows the derivation of Theorem 3.1 in Appendix A.2
("Derivation of the FKT expansion") and is computed with
``fractions.Fraction`` so that it carries no rounding at all:

* ``A(k, i, alpha)``  -- powers of cosine in Gegenbauer polynomials,
  eq. (coschange).  Reading: the printed ``(i-k)/2`` in the denominator is a
  factorial, ``((i-k)/2)!``; without it the k = i entries divide by zero.
* ``B(n, m)``         -- Faa di Bruno coefficients of Lemma A.2, eq. (faa).
* ``Tbar(k, j, m, alpha)`` -- the dimension-only constants that combine the
  two.  Reading: the binomial ``C(n, 2n-j)`` that the binomial expansion of
  eq. (prelemma) produces is restored; the printed formula drops it from the
  re-indexing step on, and without it 1/r in d = 3 does not reduce to the
  Legendre expansion of eq. (electro).
* ``bell_B(n, m)``    -- the same derivative coefficients from the Bell
  polynomial recurrence used in the proof of Lemma A.2 (an independent pin
  for ``B``).

The expansion truncated at order p (eq. finaltrunc) keeps, for each
harmonic degree k <= p, the radial powers j = k, k+2, ..., <= p
(reading of "p-term truncation", fixed by the rank count
floor((p-k)/2 + 1) of Appendix A.3).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial


def rising(a: Fraction, n: int) -> Fraction:
    """Rising factorial (a)_n = a (a+1) ... (a+n-1)."""
    out = Fraction(1)
    for i in range(n):
        out *= a + i
    return out


def double_factorial(n: int) -> int:
    """n!! with the convention (-1)!! = 1 (and 0!! = 1)."""
    if n <= 0:
        return 1
    out = 1
    while n > 0:
        out *= n
        n -= 2
    return out


def alpha_of(d: int) -> Fraction:
    """Gegenbauer index alpha = d/2 - 1 of the addition theorem (Appendix A.1)."""
    return Fraction(d, 2) - 1


@lru_cache(maxsize=None)
def A(k: int, i: int, alpha: Fraction) -> Fraction:
    """cos^i(g) = sum_k A(k,i) C_k^alpha(cos g); zero unless k <= i, k = i mod 2."""
    if k > i or (i - k) % 2:
        return Fraction(0)
    return Fraction(factorial(i)) * (alpha + k) / (
        Fraction(2) ** i * factorial((i - k) // 2) * rising(alpha, (i + k) // 2 + 1))


@lru_cache(maxsize=None)
def B(n: int, m: int) -> Fraction:
    """d^n/de^n K(r sqrt(1+e)) at e=0 equals sum_{m=1}^n B(n,m) K^(m)(r) r^m (n >= 1)."""
    if n == 0 and m == 0:
        return Fraction(1)
    if m < 1 or m > n:
        return Fraction(0)
    return Fraction((-1) ** (n + m) * double_factorial(2 * n - 2 * m - 1) * comb(2 * n - m - 1, m - 1),
                    2 ** n)


@lru_cache(maxsize=None)
def bell_B(n: int, m: int) -> Fraction:
    """Partial Bell polynomial B_{n,m}(g', g'', ...) / r^m for g(e) = r sqrt(1+e).

    Uses the recurrence B_{n,m} = sum_i C(n-1, i-1) g^(i) B_{n-i, m-1} with
    g^(i)(0) = (-1)^(i+1) (2i-3)!! / 2^i * r  (proof of Lemma A.2).
    """
    if n == 0 and m == 0:
        return Fraction(1)
    if n == 0 or m == 0:
        return Fraction(0)
    total = Fraction(0)
    for i in range(1, n - m + 2):
        gi = Fraction((-1) ** (i + 1) * double_factorial(2 * i - 3), 2 ** i)
        total += comb(n - 1, i - 1) * gi * bell_B(n - i, m - 1)
    return total


@lru_cache(maxsize=None)
def Tbar(k: int, j: int, m: int, alpha: Fraction) -> Fraction:
    """Tbar_{k,j,m}: sum over n of A_{k,2n-j} (-2)^{2n-j} C(n,2n-j) B_{n,m} / n!.

    The radial function of harmonic degree k is
      F_kj(r) = [j = 0] K(r) + sum_{m=1}^{j} K^(m)(r) r^(m-j) Tbar_{k,j,m}
    and the truncated kernel is sum_k C_k^alpha(cos g) sum_j r'^j F_kj(r).
    """
    if j < k or (j - k) % 2 or m < 1 or m > j:
        return Fraction(0)
    total = Fraction(0)
    for n in range(max((j + k) // 2, m), j + 1):
        i = 2 * n - j
        total += A(k, i, alpha) * Fraction(-2) ** i * comb(n, i) * B(n, m) / factorial(n)
    return total


def tbar_table(d: int, p: int):
    """Dense (p+1)^3 float64 table T[k][j][m] (zero where undefined), C order."""
    import numpy as np
    alpha = alpha_of(d)
    t = np.zeros((p + 1, p + 1, p + 1))
    for k in range(p + 1):
        for j in range(k, p + 1, 2):
            for m in range(1, j + 1):
                t[k, j, m] = float(Tbar(k, j, m, alpha))
    return t


def gegenbauer_monomial(k: int, alpha: Fraction):
    """Coefficients c[i] with C_k^alpha(x) = sum_i c[i] x^i (from the recurrence)."""
    c0 = [Fraction(1)]
    if k == 0:
        return c0
    c1 = [Fraction(0), 2 * alpha]
    for n in range(2, k + 1):
        nxt = [Fraction(0)] * (n + 1)
        for i, v in enumerate(c1):
            nxt[i + 1] += 2 * (n + alpha - 1) * v / n
        for i, v in enumerate(c0):
            nxt[i] -= (n + 2 * alpha - 2) * v / n
        c0, c1 = c1, nxt
    return c1


def harmonic_count(k: int, d: int) -> int:
    """|H_k| = C(k+d-1, k) - C(k+d-3, k-2) (Appendix A.3)."""
    return comb(k + d - 1, k) - (comb(k + d - 3, k - 2) if k >= 2 else 0)


def expansion_rank(d: int, p: int) -> int:
    """sum_k |H_k| floor((p-k)/2 + 1), eq. (num_multipoles)."""
    return sum(harmonic_count(k, d) * ((p - k) // 2 + 1) for k in range(p + 1))
