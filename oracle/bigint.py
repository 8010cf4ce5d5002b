"""Exact evaluation over the natural numbers at big-integer points (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's benchmarks evaluate polynomials over multiprecision integers
(Benchmarks section, Figure 1).  The value is the plain definition
p(x) = sum c_m x^m in Python's exact integers; every scheme reaches it
exactly (Section 1, Definition of evaluation tree, over the integers), so the
oracle does not build a tree.  Composition over the integers (p(q(X)), the
title problem with integer coefficients) is likewise its definition,
sum c_m q(X)^m by schoolbook polynomial products.  Big integers cross to the
GPU as arrays of 16-bit limbs, least significant first.
"""
from __future__ import annotations

LIMB_BITS = 16
LIMB_MASK = (1 << LIMB_BITS) - 1


def eval_int(terms, x: int) -> int:
    """sum c * x**e over the (exponent tuple, coefficient) terms."""
    return sum(int(c) * x ** int(e[0]) for e, c in terms)


def to_limbs(v: int, n: int) -> list:
    """The n least significant 16-bit limbs of v >= 0 (v must fit)."""
    if v < 0 or v >> (LIMB_BITS * n):
        raise ValueError("value does not fit the limbs")
    return [(v >> (LIMB_BITS * k)) & LIMB_MASK for k in range(n)]


def from_limbs(limbs) -> int:
    v = 0
    for k, w in enumerate(limbs):
        v |= int(w) << (LIMB_BITS * k)
    return v


def compose_int(terms, q) -> list:
    """The coefficients of p(q(X)) over the integers (Section 1.2: composition,
    the polynomial elements whose size grows with the degree), p given by its
    (exponent tuple, coefficient) terms and q by its coefficient list
    q[0] + q[1] X + ...: the plain definition sum_m c_m q(X)^m, each power
    by schoolbook products of coefficient lists.  Length deg p * deg q + 1."""
    q = [int(c) for c in q]
    dp = max(int(e[0]) for e, _ in terms)
    dq = len(q) - 1
    res = [0] * (dp * dq + 1)

    def mul(a, b):
        r = [0] * (len(a) + len(b) - 1)
        for i, x in enumerate(a):
            if x:
                for j, y in enumerate(b):
                    r[i + j] += x * y
        return r

    powers = {0: [1]}
    for m in range(1, dp + 1):
        powers[m] = mul(powers[m - 1], q)
    for e, c in terms:
        for k, v in enumerate(powers[int(e[0])]):
            res[k] += int(c) * v
    return res
