"""Interval evaluation of an evaluation tree, in exact rationals (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's library evaluates its trees over any coefficient type with an
addition and a multiplication, intervals among them (Abstract).  This module
takes the value of the tree (Section 1, Definition of evaluation tree) with
interval operations carried out exactly:

* a value is a closed interval (lo, hi) of Fractions;
* a coefficient c is the point interval (c, c);
* a sum of intervals is (a.lo + b.lo, a.hi + b.hi);
* a product of intervals is spanned by the four products of their ends;
* the power x_j^e over X = [l, h] is its exact range: increasing for odd e;
  for even e decreasing on l <= h <= 0, increasing on 0 <= l <= h, and
  [0, max(l^e, h^e)] when 0 lies inside.

Reading (the paper names the interval type but not its power): a partial
degree is applied as the range of the power, not as e repeated interval
products (which would widen x * x over an interval containing 0).  The result
therefore depends on the scheme (interval sums and products do not
distribute), and it contains p(x) for every x in the box.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Sequence

from . import tree as otree


def iv_add(a, b):
    return (a[0] + b[0], a[1] + b[1])


def iv_mul(a, b):
    ps = (a[0] * b[0], a[0] * b[1], a[1] * b[0], a[1] * b[1])
    return (min(ps), max(ps))


def power_range(x, e: int):
    """Exact range of t^e for t in [x[0], x[1]] (e >= 0)."""
    lo, hi = x
    if e == 0:
        return (Fraction(1), Fraction(1))
    if e % 2 == 1:
        return (lo ** e, hi ** e)
    if lo >= 0:
        return (lo ** e, hi ** e)
    if hi <= 0:
        return (hi ** e, lo ** e)
    return (Fraction(0), max(lo ** e, hi ** e))


def tree_interval(nodes, box: Sequence):
    """Interval value of the tree (nodes in <_t order, root last) over the box
    [(lo_j, hi_j)] of Fractions: value(N) = (c(N) + sum value(C)) times the
    range of each x_j^{d_j(N)} (Section 1, Definition of evaluation tree)."""
    val = {}
    powers = {}                          # (j, e) -> range of x_j^e, computed once
    for n in nodes:                      # children come before their parent
        c = Fraction(n.coef)
        acc = (c, c)
        for ch in n.children:
            acc = iv_add(acc, val[ch.index])
        for j, e in enumerate(n.pdeg):
            if e:
                if (j, e) not in powers:
                    powers[(j, e)] = power_range(box[j], e)
                acc = iv_mul(acc, powers[(j, e)])
        val[n.index] = acc
    return val[nodes[-1].index]


def interval_eval(terms, scheme, box):
    """Build T_p^f with the oracle's own builder and take its interval value.
    ``terms`` are (exponent tuple, coefficient) pairs with exact (float or
    Fraction) coefficients; ``box`` one (lo, hi) pair per variable."""
    nodes = otree.build_tree(terms, scheme)
    return tree_interval(nodes, [(Fraction(lo), Fraction(hi)) for lo, hi in box])


def magnitude_bound(terms, box) -> Fraction:
    """sum |c| prod_j max(1, |lo_j|, |hi_j|)^{e_j}: bounds every partial value
    of every tree of p over the box, and every power range (used to size
    rounding slack)."""
    m = [max(Fraction(1), abs(Fraction(lo)), abs(Fraction(hi))) for lo, hi in box]
    tot = Fraction(0)
    for e, c in terms:
        t = abs(Fraction(c))
        for j, ej in enumerate(e):
            t *= m[j] ** int(ej)
        tot += t
    return tot
