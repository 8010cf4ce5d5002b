"""Pins of the multivariate double-double references (``dd_monomial_sum``,
``monomial_ptilde``) against the plain definition p(x) = sum_m c_m x^m
(Section 1, Definition of evaluation tree: the value of every tree is this
sum) evaluated exactly, and against closed forms.

A plausible mistake in either function fails at least one of these:
 * a transposed variable or a wrong power index: the exact comparisons use
   asymmetric polynomials and distinct coordinates per variable;
 * a dropped low word (plain FP64 instead of double-double): the
   ill-conditioned cases below need far more than FP64 accuracy;
 * a dropped term or a wrong sign: the exact and closed-form values."""
import math
from fractions import Fraction

import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import exact

U = 2.0 ** -53


def _exact_cols(exps, coeffs, pts):
    terms = [(tuple(int(e) for e in m), Fraction(float(c))) for m, c in zip(exps, coeffs)]
    ys, pt = [], []
    for i in range(pts.shape[1]):
        x = [Fraction(float(v)) for v in pts[:, i]]
        ys.append(exact.exact_value(terms, x))
        pt.append(exact.exact_ptilde(terms, x))
    return ys, pt


def _check_dd(exps, coeffs, pts, k_rel=1.0, k_abs=64.0):
    """|dd - exact| <= k_rel u |exact| + k_abs 2^-104 (terms * deg) ptilde:
    rounding the double-double sum once to FP64, plus the double-double
    products and sums (a few 2^-104 relative per operation)."""
    y = exact.dd_monomial_sum(exps, coeffs, pts)
    ye, pe = _exact_cols(exps, coeffs, pts)
    nops = len(coeffs) * (1 + int(np.asarray(exps).sum(axis=1).max()))
    for i in range(pts.shape[1]):
        err = abs(Fraction(float(y[i])) - ye[i])
        bound = Fraction(k_rel * U) * abs(ye[i]) + Fraction(k_abs * nops) * Fraction(2) ** -104 * pe[i]
        assert err <= bound, (i, float(err), float(bound))
    return y


# coordinates 0 or of magnitude in [2^-20, 1.3], coefficients of magnitude
# at least 2^-30: no monomial reaches the subnormal range, where
# double-double loses its low word
_coord = st.one_of(st.just(0.0), st.floats(2.0 ** -20, 1.3), st.floats(-1.3, -(2.0 ** -20)))

poly_multi = st.integers(1, 3).flatmap(lambda v: st.dictionaries(
    st.tuples(*[st.integers(0, 9)] * v),
    st.floats(-1, 1, allow_nan=False, allow_infinity=False).filter(lambda c: abs(c) >= 2.0 ** -30),
    min_size=1, max_size=25))


@settings(max_examples=60, deadline=None)
@given(poly_multi, st.lists(_coord, min_size=9, max_size=9))
def test_dd_monomial_sum_against_exact_definition(d, xs):
    exps = np.array(list(d.keys()), dtype=np.int64)
    coeffs = np.array(list(d.values()))
    v = exps.shape[1]
    pts = np.array(xs[: v * 3], dtype=np.float64).reshape(v, 3)
    _check_dd(exps, coeffs, pts)
    # monomial_ptilde: all terms non-negative, so FP64 gives it to about
    # (terms + degree) u relative
    pt = exact.monomial_ptilde(exps, coeffs, pts)
    _, pe = _exact_cols(exps, coeffs, pts)
    nops = len(coeffs) + int(exps.sum(axis=1).max()) + 1
    for i in range(3):
        assert abs(Fraction(float(pt[i])) - pe[i]) <= Fraction(2 * nops * U) * pe[i]


def _multinomial_terms(k, signs=(1, 1, 1)):
    """(s0 x + s1 y + s2 z)^k expanded: exponent tuples and coefficients."""
    ex, co = [], []
    for a in range(k + 1):
        for b in range(k + 1 - a):
            c = k - a - b
            ex.append((a, b, c))
            co.append(math.factorial(k) // (math.factorial(a) * math.factorial(b) * math.factorial(c))
                      * signs[0] ** a * signs[1] ** b * signs[2] ** c)
    return np.array(ex, dtype=np.int64), np.array(co, dtype=np.float64)


def test_dd_monomial_sum_multinomial_closed_form():
    # (x + y + z)^k at dyadic points whose sum is exact: the value is a
    # dyadic number representable in FP64, so the reference must return it
    # exactly (the terms are much larger than the result: cancellation)
    ex, co = _multinomial_terms(9)
    pts = np.array([[0.75, -1.5, 0.5, 2.0],
                    [-0.5, 1.25, 0.25, -1.0],
                    [0.125, 0.5, -0.625, -0.5]])
    want = (pts[0] + pts[1] + pts[2]) ** 9
    y = exact.dd_monomial_sum(ex, co, pts)
    assert np.array_equal(y, want)
    # p~ = (|x| + |y| + |z|)^k, exact for these dyadics
    assert np.array_equal(exact.monomial_ptilde(ex, co, pts), (np.abs(pts).sum(axis=0)) ** 9)
    # the variables are not interchangeable: (x + y - z)^9
    ex2, co2 = _multinomial_terms(9, signs=(1, 1, -1))
    want2 = (pts[0] + pts[1] - pts[2]) ** 9
    assert np.array_equal(exact.dd_monomial_sum(ex2, co2, pts), want2)


def test_dd_monomial_sum_ill_conditioned_needs_double_double():
    # (x + y - 1)^7 near the plane x + y = 1: the sum of the monomials'
    # magnitudes is ~3^7 while the value is ~1e-70; plain FP64 summation is
    # off by ~1e-13, the double-double reference must be within its bound
    ex, co = _multinomial_terms(7, signs=(1, 1, -1))
    rng = np.random.default_rng(5)
    x = rng.uniform(0.2, 0.8, 6)
    y = 1.0 - x + np.ldexp(rng.integers(1, 64, 6).astype(float), -60)
    pts = np.stack([x, y, np.ones(6)])
    got = _check_dd(ex, co, pts)
    # a plain FP64 evaluation of the same sum fails what the reference meets
    plain = np.zeros(6)
    for m, c in zip(ex, co):
        plain += c * pts[0] ** m[0] * pts[1] ** m[1] * pts[2] ** m[2]
    ye, _ = _exact_cols(ex, co, pts)
    ref = np.array([float(v) for v in ye])
    assert np.max(np.abs(plain - ref)) > 1e3 * np.max(np.abs(got - ref) + 1e-300)


def test_dd_monomial_sum_at_plus_minus_one_is_fsum():
    # at x_j = +-1 every monomial is +-c_m exactly, so the value is the
    # correctly rounded fsum of the signed coefficients
    rng = np.random.default_rng(9)
    ex = np.unique(rng.integers(0, 12, size=(300, 3)), axis=0)
    co = rng.uniform(-1, 1, len(ex))
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                want = math.fsum(c * sx ** m[0] * sy ** m[1] * sz ** m[2] for m, c in zip(ex, co))
                got = exact.dd_monomial_sum(ex, co, np.array([[sx], [sy], [sz]]))[0]
                assert got == want
                pt = exact.monomial_ptilde(ex, co, np.array([[sx], [sy], [sz]]))[0]
                ref = math.fsum(np.abs(co))
                assert abs(pt - ref) <= 2 * len(co) * U * ref


def test_dd_monomial_sum_univariate_matches_exact_on_workload_shape():
    # a sparse univariate polynomial of the benchmark's shape (degree 300,
    # 10 % zeros) at points in [-1.05, 1.05]: within one ulp of the exact
    # value wherever cond < 1e10 (the bar the GPU tests rely on)
    rng = np.random.default_rng(21)
    n = 300
    c = rng.uniform(-1, 1, n + 1)
    c[rng.choice(n, 30, replace=False)] = 0
    ex = np.nonzero(c)[0].reshape(-1, 1)
    pts = rng.uniform(-1.05, 1.05, (1, 12))
    y = exact.dd_monomial_sum(ex, c[ex[:, 0]], pts)
    ye, pe = exact.exact_uni_values(c, pts[0])
    ok = pe / np.abs(ye) < 1e10
    assert ok.sum() >= 8
    assert np.all(np.abs(y[ok] - ye[ok]) <= np.spacing(np.abs(ye[ok])))
