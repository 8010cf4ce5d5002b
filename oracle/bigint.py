"""Exact evaluation over the natural numbers at big-integer points (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's benchmarks evaluate polynomials over multiprecision integers
(Benchmarks section, Figure 1).  The value is the plain definition
p(x) = sum c_m x^m in Python's exact integers; every scheme reaches it
exactly (Section 1, Definition of evaluation tree, over the integers), so the
oracle does not build a tree.  Big integers cross to the GPU as arrays of
16-bit limbs, least significant first.
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
