"""The plain definition p(x) = sum_m c_m x^m, computed without any scheme.

Every function scheme reaches this value exactly in exact arithmetic (the
value of an evaluation tree, Section 1 Definition, together with the
uniqueness of the split in Section 1.1), so this is what the oracle checks the
GPU path against.

* ``exact_value``       exact rational value (Fraction), rounded once to FP64
                        by ``float`` (correctly rounded).
* ``exact_ptilde``      sum |c_m| |x|^m, exact, for the condition number
                        cond(p, x) = ptilde / |p(x)|.
* ``modp_value``        sum c_m prod_j x_j^{m_j} mod p with Python integers.
* ``dd_horner``         double-double Hörner (Dekker/Veltkamp split, no fma),
                        vectorised over points: the bulk FP64 reference.
* ``dd_monomial_sum``   double-double sum of monomials for multivariate input.
* ``fsum_at_pm1``       closed forms at x = +1 / -1 by math.fsum.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


# ----------------------------------------------------------------------------
# exact rationals
# ----------------------------------------------------------------------------

def exact_value(terms, x) -> Fraction:
    """sum c_m prod_j x_j^{m_j} over Q (terms: (exponent tuple, coef))."""
    xs = [Fraction(v) for v in (x if hasattr(x, "__len__") else (x,))]
    acc = Fraction(0)
    for m, c in terms:
        t = Fraction(c)
        for xj, e in zip(xs, m):
            t *= xj ** int(e)
        acc += t
    return acc


def exact_ptilde(terms, x) -> Fraction:
    xs = [abs(Fraction(v)) for v in (x if hasattr(x, "__len__") else (x,))]
    acc = Fraction(0)
    for m, c in terms:
        t = abs(Fraction(c))
        for xj, e in zip(xs, m):
            t *= xj ** int(e)
        acc += t
    return acc


def exact_uni_values(coeffs, xs):
    """Exact values of a dense univariate polynomial at FP64 points, rounded
    once; also returns ptilde (rounded).  Hörner over Q is exact, so the order
    of the exact operations does not matter."""
    cf = [Fraction(float(c)) for c in coeffs]
    ys, pts = [], []
    for x in xs:
        xf = Fraction(float(x))
        ax = abs(xf)
        acc = Fraction(0)
        pt = Fraction(0)
        for c in reversed(cf):
            acc = acc * xf + c
            pt = pt * ax + abs(c)
        ys.append(float(acc))
        pts.append(float(pt))
    return np.array(ys), np.array(pts)


# ----------------------------------------------------------------------------
# modular
# ----------------------------------------------------------------------------

def modp_value(terms, x, p: int) -> int:
    acc = 0
    for m, c in terms:
        t = int(c) % p
        for xj, e in zip(x, m):
            t = t * pow(int(xj), int(e), p) % p
        acc = (acc + t) % p
    return acc


# ----------------------------------------------------------------------------
# double-double (Dekker 1971 / Knuth TwoSum), numpy vectorised, no fma
# ----------------------------------------------------------------------------

_SPLIT = 134217729.0  # 2^27 + 1


def _two_sum(a, b):
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def _fast_two_sum(a, b):
    s = a + b
    e = b - (s - a)
    return s, e


def _split(a):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def dd_mul(ah, al, bh, bl):
    p, e = _two_prod(ah, bh)
    e = e + (ah * bl + al * bh)
    return _fast_two_sum(p, e)


def dd_add(ah, al, bh, bl):
    s, e = _two_sum(ah, bh)
    e = e + (al + bl)
    return _fast_two_sum(s, e)


def dd_horner(coeffs, xs):
    """Double-double Hörner of a dense coefficient vector (index = exponent)
    at FP64 points; returns (hi, lo).  Error about 2n 2^-104 ptilde."""
    x = np.asarray(xs, dtype=np.float64)
    c = np.asarray(coeffs, dtype=np.float64)
    hi = np.full_like(x, c[-1])
    lo = np.zeros_like(x)
    zero = np.zeros_like(x)
    for k in range(len(c) - 2, -1, -1):
        hi, lo = dd_mul(hi, lo, x, zero)
        hi, lo = dd_add(hi, lo, np.full_like(x, c[k]), zero)
    return hi, lo


def dd_value(coeffs, xs):
    hi, lo = dd_horner(coeffs, xs)
    return hi + lo


def ptilde_f64(coeffs, xs):
    """sum |c| |x|^m by FP64 Hörner; all terms are >= 0 so the relative error
    is at most about 2n u."""
    x = np.abs(np.asarray(xs, dtype=np.float64))
    c = np.abs(np.asarray(coeffs, dtype=np.float64))
    acc = np.full_like(x, c[-1])
    for k in range(len(c) - 2, -1, -1):
        acc = acc * x + c[k]
    return acc


def dd_monomial_sum(exps, coeffs, pts):
    """Double-double sum_m c_m prod_j x_j^{m_j} at FP64 points (SoA [v, N]).

    Powers are built by repeated double-double multiplication from x_j, so
    each monomial carries an error of a few 2^-104 relative."""
    exps = np.asarray(exps)
    pts = np.asarray(pts, dtype=np.float64)
    v, N = pts.shape
    zero = np.zeros(N)
    maxe = exps.max(axis=0) if len(exps) else np.zeros(v, int)
    pw = []
    for j in range(v):
        tab = [(np.ones(N), zero.copy())]
        for _ in range(int(maxe[j])):
            tab.append(dd_mul(tab[-1][0], tab[-1][1], pts[j], zero))
        pw.append(tab)
    hi = zero.copy()
    lo = zero.copy()
    for m, c in zip(exps, coeffs):
        th = np.full(N, float(c))
        tl = zero.copy()
        for j in range(v):
            if m[j]:
                th, tl = dd_mul(th, tl, pw[j][int(m[j])][0], pw[j][int(m[j])][1])
        hi, lo = dd_add(hi, lo, th, tl)
    return hi + lo


def monomial_ptilde(exps, coeffs, pts):
    pts = np.abs(np.asarray(pts, dtype=np.float64))
    acc = np.zeros(pts.shape[1])
    for m, c in zip(exps, coeffs):
        t = np.full(pts.shape[1], abs(float(c)))
        for j in range(pts.shape[0]):
            t = t * pts[j] ** int(m[j])
        acc = acc + t
    return acc


# ----------------------------------------------------------------------------
# closed forms
# ----------------------------------------------------------------------------

def fsum_at_pm1(coeffs, sign: int) -> float:
    """p(1) = fsum(c), p(-1) = fsum((-1)^m c_m), correctly rounded."""
    return math.fsum(c if (sign > 0 or e % 2 == 0) else -c for e, c in enumerate(coeffs))


def fsum_at_pow2(coeffs, k: int) -> float:
    """p(2^k): every term c_m 2^{km} is exact in FP64 (barring overflow), so
    fsum gives the correctly rounded value."""
    return math.fsum(math.ldexp(float(c), k * e) for e, c in enumerate(coeffs))
