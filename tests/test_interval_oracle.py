"""Pins of the interval oracle (oracle/interval.py) against what the
mathematics fixes: thin boxes reduce to the exact value of p (Section 1,
Definition of evaluation tree, with point intervals), a polynomial with
nonnegative coefficients over a nonnegative box is monotone (its interval
value is [p(lo), p(hi)] for every scheme), the exact ranges of single powers,
a hand-computed Hörner / Estrin pair (Section 1.1) and the inclusion property
(p(x) lies in the interval value for every x in the box)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, interval, schemes, tree

SCHEMES = {"horner": schemes.horner, "estrin": schemes.estrin, "balanced": schemes.balanced,
           "direct": schemes.direct}


def uni_terms(coeffs):
    return [((e,), float(c)) for e, c in enumerate(coeffs) if c != 0]


@pytest.mark.parametrize("name", list(SCHEMES))
def test_thin_box_is_the_exact_value(name):
    g = np.random.default_rng(11)
    c = g.uniform(-1, 1, 41)
    c[g.choice(40, 6, replace=False)] = 0.0
    terms = uni_terms(c)
    for x in g.uniform(-1.1, 1.1, 6):
        lo, hi = interval.interval_eval(terms, SCHEMES[name], [(x, x)])
        assert lo == hi == exact.exact_value(terms, [x])


@pytest.mark.parametrize("name", list(SCHEMES))
def test_thin_box_multivariate(name):
    g = np.random.default_rng(12)
    terms = []
    for a in range(4):
        for b in range(4 - a):
            for cc in range(3 - a if a < 3 else 1):
                if g.uniform() < 0.7:
                    terms.append(((a, b, cc), float(g.uniform(-1, 1))))
    x = [float(v) for v in g.uniform(-1, 1, 3)]
    lo, hi = interval.interval_eval(terms, SCHEMES[name], [(v, v) for v in x])
    assert lo == hi == exact.exact_value(terms, x)


@pytest.mark.parametrize("name", list(SCHEMES))
def test_monotone_polynomial_gives_its_end_values(name):
    g = np.random.default_rng(13)
    c = g.uniform(0, 1, 30)
    terms = uni_terms(c)
    l, h = 0.25, 0.875
    lo, hi = interval.interval_eval(terms, SCHEMES[name], [(l, h)])
    assert (lo, hi) == (exact.exact_value(terms, [l]), exact.exact_value(terms, [h]))


def test_power_ranges():
    F = Fraction
    assert interval.power_range((F(-1), F(2)), 2) == (0, 4)
    assert interval.power_range((F(-3), F(-1)), 2) == (1, 9)
    assert interval.power_range((F(-2), F(1)), 3) == (-8, 1)
    assert interval.power_range((F(-2), F(-1)), 3) == (-8, -1)
    assert interval.power_range((F(1, 2), F(3)), 4) == (F(1, 16), 81)
    assert interval.power_range((F(-5), F(3)), 0) == (1, 1)


def test_hand_computed_horner_and_estrin():
    # p = 1 + x + x^2 + x^3 over [-1, 1].  Hörner ((x + 1) x + 1) x + 1:
    # [0, 2] [-1, 1] = [-2, 2]; + 1 = [-1, 3]; times [-1, 1] = [-3, 3]; + 1.
    # Estrin (1 + x) + (1 + x) x^2: [0, 2] [0, 1] = [0, 2], plus 1 + [-1, 1].
    terms = uni_terms([1.0, 1.0, 1.0, 1.0])
    assert interval.interval_eval(terms, schemes.horner, [(-1.0, 1.0)]) == (-2, 4)
    assert interval.interval_eval(terms, schemes.estrin, [(-1.0, 1.0)]) == (0, 4)


@pytest.mark.parametrize("name", list(SCHEMES))
def test_inclusion_property(name):
    g = np.random.default_rng(14)
    c = g.uniform(-1, 1, 25)
    terms = uni_terms(c)
    nodes = tree.build_tree(terms, SCHEMES[name])
    for _ in range(5):
        a, b = sorted(g.uniform(-1.2, 1.2, 2))
        lo, hi = interval.tree_interval(nodes, [(Fraction(a), Fraction(b))])
        for t in np.linspace(a, b, 9):
            assert lo <= exact.exact_value(terms, [float(t)]) <= hi


def test_outward_rounding_rule_encloses_round_to_nearest():
    """The interval walk moves each round-to-nearest result r outward by
    RN(RN(r -/+ |r| 2^-52) -/+ 2^-1074).  For exact values z (random, and at
    binade edges, in the subnormal range and near overflow), with r = RN(z)
    computed exactly: dn(r) <= z <= up(r)."""
    F = Fraction
    tiny = F(2) ** -1074

    def rn(q):                     # correctly rounded (float() of a Fraction)
        return float(q)

    def dn(r):
        return rn(F(rn(F(r) - abs(F(r)) * F(2) ** -52)) - tiny)

    def up(r):
        return rn(F(rn(F(r) + abs(F(r)) * F(2) ** -52)) + tiny)

    g = np.random.default_rng(21)
    zs = []
    for e in (-1074, -1060, -1022, -1000, -52, -1, 0, 1, 52, 500, 1020):
        for _ in range(20):
            m = F(int(g.integers(1, 2 ** 62)), 2 ** 62)        # (0, 1)
            zs.append(m * F(2) ** e)
        zs.append(F(2) ** e)                                   # binade edges
        zs.append(F(2) ** e * (1 - F(1, 2 ** 60)))
    zs += [-z for z in zs] + [F(0)]
    for z in zs:
        r = rn(z)
        assert F(dn(r)) <= z <= F(up(r)), z
