"""Pins of the oracle's exact coefficient tables (Appendix A.2, A.3).

Each test compares the oracle against something it does not compute itself:
a library routine (scipy's Gegenbauer polynomials), symbolic differentiation
(sympy), or closed forms fixed by classical expansions (Legendre/Gegenbauer
generating function).
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest
import sympy
from scipy.special import eval_gegenbauer

from oracle import coeffs as C


@pytest.mark.parametrize("d", [3, 4, 5, 6, 9])
def test_cos_powers_in_gegenbauer(d):
    """eq. (coschange): cos^i = sum_k A_ki C_k^alpha(cos), checked with scipy's C_k^alpha."""
    alpha = C.alpha_of(d)
    xs = np.linspace(-1.0, 1.0, 13)
    for i in range(0, 11):
        rhs = sum(float(C.A(k, i, alpha)) * eval_gegenbauer(k, float(alpha), xs) for k in range(i + 1))
        np.testing.assert_allclose(rhs, xs ** i, atol=1e-12)


def test_cos_powers_small_cases():
    """x = C_1/(2 alpha) and x^2 = C_2/(2 alpha (alpha+1)) + C_0/(2(alpha+1))."""
    for d in (3, 4, 5):
        a = C.alpha_of(d)
        assert C.A(1, 1, a) == 1 / (2 * a)
        assert C.A(2, 2, a) == 1 / (2 * a * (a + 1))
        assert C.A(0, 2, a) == 1 / (2 * (a + 1))
        assert C.A(1, 2, a) == 0 and C.A(0, 1, a) == 0


def test_faa_di_bruno_coefficients_symbolic():
    """Lemma A.2: d^n/de^n K(r sqrt(1+e)) at 0 = sum_m B_nm K^(m)(r) r^m.

    With K(s) = exp(c s), K^(m) = c^m exp(c s), so the left side divided by
    exp(c r) is a polynomial in (c r) whose coefficients are B_nm. Computed by
    sympy, independently of the closed form and of the Bell recurrence.
    """
    c, r, e = sympy.symbols("c r e", positive=True)
    f = sympy.exp(c * r * sympy.sqrt(1 + e))
    for n in range(1, 8):
        poly = sympy.expand(sympy.simplify(sympy.diff(f, e, n).subs(e, 0) / sympy.exp(c * r)))
        P = sympy.Poly(poly, c)
        for m in range(0, n + 2):
            coef = P.coeff_monomial(c ** m)
            b = C.B(n, m) if 1 <= m <= n else Fraction(0)
            expect = sympy.Rational(b.numerator, b.denominator) * r ** m
            assert sympy.simplify(coef - expect) == 0, (n, m)


def test_faa_di_bruno_matches_bell_recurrence():
    """The closed form of B_nm equals the Bell-polynomial recurrence of the proof."""
    for n in range(1, 16):
        for m in range(1, n + 1):
            assert C.B(n, m) == C.bell_B(n, m), (n, m)


@pytest.mark.parametrize("d", [3, 4, 5, 6, 7])
def test_newtonian_kernel_is_rank_one(d):
    """|r - r'|^-(d-2) = r^-(d-2) sum_k C_k^alpha(cos g) (r'/r)^k (Gegenbauer
    generating function; eq. electro for d = 3). Hence for K = r^-q, q = 2 alpha:
    F_kj(r) = r^(-q-j) [delta_j0 + sum_m (-1)^m (q)_m Tbar_kjm] must equal
    delta_jk r^(-q-k), exactly in rationals. Fails if the restored binomial
    C(n, 2n-j), the factorial in A, or the m = 0 term were wrong."""
    alpha = C.alpha_of(d)
    q = 2 * alpha
    p = 10
    for k in range(p + 1):
        for j in range(k, p + 1, 2):
            s = Fraction(1 if j == 0 else 0)
            for m in range(1, j + 1):
                s += (-1) ** m * C.rising(q, m) * C.Tbar(k, j, m, alpha)
            assert s == (1 if j == k else 0), (d, k, j, s)


def test_printed_formula_without_binomial_fails_laplace():
    """Guard for the reading: dropping C(n, 2n-j) breaks the d=3 Legendre case."""
    alpha = C.alpha_of(3)
    from math import factorial
    k, j = 0, 4   # n = 3, i = 2 is the first term where C(n, i) != 1
    s = Fraction(0)
    for m in range(1, j + 1):
        t = Fraction(0)
        for n in range(max((j + k) // 2, m), j + 1):
            i = 2 * n - j
            t += C.A(k, i, alpha) * Fraction(-2) ** i * C.B(n, m) / factorial(n)
        s += (-1) ** m * C.rising(Fraction(1), m) * t
    assert s != 0


@pytest.mark.parametrize("d", [3, 4, 5, 6, 8])
def test_term_count_equals_binomial(d):
    """Appendix A.3: sum_k |H_k| floor((p-k)/2 + 1) = C(p+d, d)."""
    for p in range(0, 13):
        assert C.expansion_rank(d, p) == comb(p + d, d)


def test_harmonic_count_small():
    """|H_k| = 2k+1 in d=3 and (k+1)^2 in d=4 (classical)."""
    for k in range(10):
        assert C.harmonic_count(k, 3) == 2 * k + 1
        assert C.harmonic_count(k, 4) == (k + 1) ** 2


@pytest.mark.parametrize("d", [3, 5])
def test_gegenbauer_monomials_match_scipy(d):
    a = C.alpha_of(d)
    xs = np.linspace(-1, 1, 9)
    for k in range(9):
        c = C.gegenbauer_monomial(k, a)
        v = sum(float(ci) * xs ** i for i, ci in enumerate(c))
        np.testing.assert_allclose(v, eval_gegenbauer(k, float(a), xs), atol=1e-12)
