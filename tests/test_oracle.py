"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each value comes from the
paper's worked example, a closed form, brute force, or an independent
formulation (exact rationals vs. double-double vs. plain C)."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import compose as ocomp
from oracle import exact, native, schemes, tree

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
P61 = (1 << 61) - 1
P31 = (1 << 31) - 1


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


def children_by_exp(nodes):
    return {str(n.exps[0]): [c.exps[0] for c in n.children] for n in nodes if n.children}


# ----------------------------------------------------------------------------
# worked example (Section 1.1 Example, Section 1.2 Example, Section 1.3 Example)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["direct", "horner", "estrin", "balanced"])
def test_worked_example_trees(gold, name):
    c = gold["coeffs_by_exponent"]
    nodes = tree.build_tree(tree.dense_terms(c), schemes.BY_NAME[name])
    assert children_by_exp(nodes) == gold["children_by_exponent"][name]
    # the first split p = a x^{f(8)} + b
    sp = gold["first_split"][name]
    assert schemes.BY_NAME[name](8) == sp["f"]
    a = [0] * (len(c) - sp["f"])
    for e in range(sp["f"], len(c)):
        a[e - sp["f"]] = c[e]
    while a and a[0] == 0:
        a.pop(0)
    assert a == sp["a"] or a == sp["a"][-len(a):]
    assert c[: sp["f"]] == sp["b"]


def test_worked_example_lazy_heights(gold):
    c = gold["coeffs_by_exponent"]
    for name, want in gold["lazy_height_printed"].items():
        nodes = tree.build_tree(tree.dense_terms(c), schemes.BY_NAME[name])
        lh = max(tree.lazy_heights(nodes))
        if name in gold["lazy_height_by_definition"]:
            assert lh == gold["lazy_height_by_definition"][name]
        else:
            assert lh == want
    nodes = tree.build_tree(tree.dense_terms(c), schemes.horner)
    assert max(tree.classical_heights(nodes)) == gold["classical_height_printed"]["horner"]


def test_worked_example_balanced_lower_degrees(gold):
    c = gold["coeffs_by_exponent"]
    e = tree.build_tree(tree.dense_terms(c), schemes.estrin)
    b = tree.build_tree(tree.dense_terms(c), schemes.balanced)
    assert max(tree.distinct_partial_degrees(b)) < max(tree.distinct_partial_degrees(e))


def test_worked_example_values(gold):
    c = gold["coeffs_by_exponent"]
    for x in [Fraction(0), Fraction(1), Fraction(-1), Fraction(2), Fraction(-3, 7)]:
        want = (3 * x**8 - x**7 + 2 * x**6 + x**5 - 4 * x**4 + 9 * x**3 - 3 * x**2 - 2 * x + 1)
        assert exact.exact_value(tree.dense_terms(c), [x]) == want
        for name in ["direct", "horner", "estrin", "balanced", "balanced_literal"]:
            nodes = tree.build_tree(tree.dense_terms(c), schemes.BY_NAME[name])
            assert tree.tree_value(nodes, [x]) == want
            assert tree.walk(nodes, [x]) == want


# ----------------------------------------------------------------------------
# Table 1: distinct partial degrees of a dense polynomial of degree n
# ----------------------------------------------------------------------------

def table1_sets(n):
    lg = n.bit_length() - 1
    return {
        "direct": set(range(1, n + 1)),
        "horner": {1},
        "estrin": {1 << k for k in range(lg + 1)},
        "balanced": {n >> k for k in range(lg + 1)} | {(n >> k) + 1 for k in range(lg + 1)},
    }


@pytest.mark.parametrize("n", list(range(1, 130)) + [255, 256, 257, 511, 1000, 1023, 1024, 3000, 5000])
def test_table1_degrees(n):
    c = [1.0] * (n + 1)
    sets = table1_sets(n)
    for name in ["horner", "estrin", "balanced"] + (["direct"] if n <= 300 else []):
        nodes = tree.build_tree(tree.dense_terms(c), schemes.BY_NAME[name])
        got = tree.distinct_partial_degrees(nodes)
        if name in ("direct", "horner"):
            assert got == sets[name], name
        else:
            assert got <= sets[name], (name, sorted(got - sets[name]))
            assert len(got) <= 2 * (n.bit_length())


@pytest.mark.parametrize("m", range(1, 11))
def test_estrin_equals_balanced_at_powers_of_two_terms(m):
    # with 2^m terms the balanced split ceil(n/2) equals 2^floor(log n)
    c = [1.0] * (1 << m)
    e = tree.build_tree(tree.dense_terms(c), schemes.estrin)
    b = tree.build_tree(tree.dense_terms(c), schemes.balanced)
    assert children_by_exp(e) == children_by_exp(b)


@pytest.mark.parametrize("n", [7, 31, 100, 1023, 3000, 5000])
def test_lazy_height_logarithmic_and_equal_safe_slot_on_dense(n):
    c = [1.0] * (n + 1)
    for name in ["horner", "estrin", "balanced", "direct"]:
        if name == "direct" and n > 300:
            continue
        nodes = tree.build_tree(tree.dense_terms(c), schemes.BY_NAME[name])
        lh = tree.lazy_heights(nodes)
        ss = tree.safe_slots(nodes)
        assert max(lh) <= n.bit_length()
        assert lh == ss


# ----------------------------------------------------------------------------
# structure invariants
# ----------------------------------------------------------------------------

def _check_structure(nodes, terms):
    # <_t is topological with the root last (Section 1)
    for n in nodes:
        for ch in n.children:
            assert ch.index < n.index
        # children in <_t order, C_1 biggest
        assert [ch.index for ch in n.children] == sorted(ch.index for ch in n.children)
    # monomial degree = sum of partial degrees along the root path (Section 1)
    for n in nodes:
        s = [0] * len(n.exps)
        m = n
        while m is not None:
            s = [a + b for a, b in zip(s, m.pdeg)]
            m = m.parent
        assert tuple(s) == n.exps
    real = {n.exps: n.coef for n in nodes if not n.junction}
    want = {tuple(m): c for m, c in terms if c != 0}
    assert real == want


poly_uni = st.dictionaries(st.integers(0, 60), st.integers(-9, 9).filter(lambda v: v != 0),
                           min_size=1, max_size=25)


@settings(max_examples=60, deadline=None)
@given(poly_uni, st.sampled_from(["direct", "horner", "estrin", "balanced", "balanced_literal"]),
       st.fractions(min_value=-3, max_value=3, max_denominator=11))
def test_uni_sparse_tree_value_exact(d, name, x):
    terms = [((e,), c) for e, c in d.items()]
    nodes = tree.build_tree(terms, schemes.BY_NAME[name])
    _check_structure(nodes, terms)
    want = exact.exact_value(terms, [x])
    assert tree.tree_value(nodes, [x]) == want
    assert tree.walk(nodes, [x]) == want
    # the same over Z/pZ
    xp = (x.numerator * pow(x.denominator, -1, P61)) % P61
    add = lambda a, b: (a + b) % P61
    mul = lambda a, b: (a * b) % P61
    tp = [(m, c % P61) for m, c in terms]
    nodes_p = tree.build_tree(tp, schemes.BY_NAME[name])
    assert tree.walk(nodes_p, [xp], add=add, mul=mul) == exact.modp_value(tp, [xp], P61)


poly_multi = st.integers(1, 3).flatmap(lambda v: st.dictionaries(
    st.tuples(*[st.integers(0, 6)] * v), st.integers(-5, 5).filter(lambda c: c != 0),
    min_size=1, max_size=30))


@settings(max_examples=60, deadline=None)
@given(poly_multi, st.sampled_from(["horner", "estrin", "balanced", "direct"]),
       st.lists(st.integers(-4, 4), min_size=3, max_size=3))
def test_multi_sparse_tree_value_exact(d, name, xs):
    terms = list(d.items())
    v = len(terms[0][0])
    x = [Fraction(a, 3) for a in xs[:v]]
    nodes = tree.build_tree(terms, schemes.BY_NAME[name])
    _check_structure(nodes, terms)
    # one nonzero variable in every partial degree (nesting, Section 1.1 Remark)
    for n in nodes[:-1]:
        assert sum(1 for e in n.pdeg if e) == 1
    want = exact.exact_value(terms, x)
    assert tree.tree_value(nodes, x) == want
    assert tree.walk(nodes, x) == want


def test_paper_lazy_height_unsafe_on_sparse_but_safe_slots_hold():
    # a sparse case where a non-first child has one child with a deep
    # subtree: the walk with the paper's lazy height clobbers an accumulator
    rng = np.random.default_rng(3)
    bad = 0
    for trial in range(200):
        e = sorted(rng.choice(200, 60, replace=False).tolist())
        terms = [((int(k),), int(rng.integers(1, 9))) for k in e]
        nodes = tree.build_tree(terms, schemes.estrin)
        x = [Fraction(2, 3)]
        want = exact.exact_value(terms, x)
        assert tree.walk(nodes, x) == want
        if tree.walk(nodes, x, slots=tree.lazy_heights(nodes)) != want:
            bad += 1
    assert bad > 0


def test_brute_force_tiny():
    # every support subset of {0..5} with coefficients 1..k, every scheme
    x = Fraction(-5, 3)
    for r in range(1, 7):
        for supp in itertools.combinations(range(6), r):
            terms = [((e,), i + 1) for i, e in enumerate(supp)]
            want = sum(Fraction(c) * x**e[0] for e, c in terms)
            for name in ["direct", "horner", "estrin", "balanced", "balanced_literal"]:
                nodes = tree.build_tree(terms, schemes.BY_NAME[name])
                assert tree.walk(nodes, [x]) == want
                assert tree.tree_value(nodes, [x]) == want


def test_scheme_legality():
    for k in range(1, 2000):
        for f in [schemes.direct, schemes.horner, schemes.estrin, schemes.balanced,
                  schemes.balanced_literal]:
            assert 0 < f(k) <= k
    with pytest.raises(tree.SchemeError):
        tree.build_tree([((0,), 1), ((3,), 1)], lambda k: 0)
    with pytest.raises(ValueError):
        tree.build_tree([((1,), 1), ((1,), 2)], schemes.horner)


def test_nested_dense_trivariate_has_no_junctions():
    # dense polynomials need no junction node; a sparse one does
    ex = [(a, b, c) for a in range(4) for b in range(4) for c in range(4) if a + b + c <= 3]
    nodes = tree.build_tree([(m, 1) for m in ex], schemes.estrin)
    assert not any(n.junction for n in nodes)
    assert len(nodes) == math.comb(3 + 3, 3)
    nodes = tree.build_tree([((2, 1, 0), 1), ((0, 1, 1), 1), ((1, 0, 2), 1)], schemes.horner)
    assert any(n.junction for n in nodes)


# ----------------------------------------------------------------------------
# definition-level values: closed forms
# ----------------------------------------------------------------------------

def test_exact_value_binomial_closed_form():
    k = 12
    terms = [((m,), math.comb(k, m)) for m in range(k + 1)]
    for x in [Fraction(1, 3), Fraction(-7, 5), Fraction(2)]:
        assert exact.exact_value(terms, [x]) == (1 + x) ** k


def test_exact_value_geometric_closed_form():
    n = 40
    terms = [((m,), 1) for m in range(n + 1)]
    for x in [Fraction(3, 4), Fraction(-9, 8)]:
        assert exact.exact_value(terms, [x]) == (x ** (n + 1) - 1) / (x - 1)


def test_dd_and_exact_agree_with_fsum_closed_forms():
    rng = np.random.default_rng(11)
    c = rng.uniform(-1, 1, 301)
    for s in (1, -1):
        want = exact.fsum_at_pm1(c, s)
        assert float(exact.exact_value(tree.dense_terms(c), [s])) == want
        assert exact.dd_value(c, np.array([float(s)]))[0] == want
        assert native.dd_value(c, np.array([float(s)]))[0] == want
    for k in (-3, -1, 1):
        want = exact.fsum_at_pow2(c[:60], k)
        assert exact.dd_value(c[:60], np.array([2.0**k]))[0] == want
        assert native.dd_value(c[:60], np.array([2.0**k]))[0] == want
    # x = 0 gives the constant coefficient
    assert native.dd_value(c, np.array([0.0]))[0] == c[0]


def test_dd_within_one_ulp_of_exact():
    rng = np.random.default_rng(12)
    c = rng.uniform(-1, 1, 1001)
    c[rng.choice(1000, 100, replace=False)] = 0
    x = rng.uniform(-1.05, 1.05, 60)
    ye, pt = exact.exact_uni_values(c, x)
    for impl in (exact.dd_value, native.dd_value):
        y = impl(c, x)
        cond = pt / np.abs(ye)
        ok = cond < 1e10
        ulp = np.spacing(np.abs(ye))
        assert np.all(np.abs(y - ye)[ok] <= ulp[ok])
    assert np.allclose(native.ptilde(c, x), pt, rtol=1e-12)


def _round_fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def test_native_fma_horner_matches_single_rounding_emulation():
    rng = np.random.default_rng(13)
    c = rng.uniform(-1, 1, 40)
    x = rng.uniform(-1, 1, 25)
    y = native.horner_f64(c, x, use_fma=True)
    y2 = native.horner_f64(c, x, use_fma=False)
    for i, xi in enumerate(x):
        acc = float(c[-1])
        acc2 = float(c[-1])
        for k in range(len(c) - 2, -1, -1):
            acc = _round_fma(acc, xi, c[k])
            acc2 = float(Fraction(float(Fraction(acc2) * Fraction(xi))) + Fraction(c[k]))
        assert y[i] == acc
        assert y2[i] == acc2


# ----------------------------------------------------------------------------
# modular definition
# ----------------------------------------------------------------------------

def test_modp_fermat_and_binomial():
    p = 10007
    for x in range(1, 50):
        assert exact.modp_value([((p - 1,), 1)], [x], p) == 1
    k = 30
    terms = [((m,), math.comb(k, m)) for m in range(k + 1)]
    for x in [3, 12345, P61 - 2]:
        assert exact.modp_value(terms, [x], P61) == pow(x + 1, k, P61)
    # native C against the Python definition, multivariate
    rng = np.random.default_rng(5)
    ex = rng.integers(0, 12, size=(40, 3)).astype(np.int32)
    ex = np.unique(ex, axis=0)
    co = rng.integers(0, P61, size=len(ex), dtype=np.uint64)
    pts = rng.integers(0, P61, size=(3, 30), dtype=np.uint64)
    got = native.modp_eval(ex, co, P61, pts)
    terms = [(tuple(int(v) for v in m), int(c)) for m, c in zip(ex, co)]
    for i in range(30):
        assert int(got[i]) == exact.modp_value(terms, [int(pts[j, i]) for j in range(3)], P61)


def test_modp_multivariate_closed_form():
    # (x + y + z)^4 expanded with multinomial coefficients
    p = P61
    terms = []
    for a in range(5):
        for b in range(5 - a):
            c = 4 - a - b
            terms.append(((a, b, c), math.factorial(4) // (math.factorial(a) * math.factorial(b) * math.factorial(c))))
    for pt in [(1, 2, 3), (p - 1, 5, 77), (123456789, 987654321, 42)]:
        assert exact.modp_value(terms, pt, p) == pow(sum(pt), 4, p)
        ex = np.array([m for m, _ in terms], dtype=np.int32)
        co = np.array([c for _, c in terms], dtype=np.uint64)
        got = native.modp_eval(ex, co, p, np.array(pt, dtype=np.uint64).reshape(3, 1))
        assert int(got[0]) == pow(sum(pt), 4, p)


# ----------------------------------------------------------------------------
# composition
# ----------------------------------------------------------------------------

def test_compose_special_cases():
    p = P31
    rng = np.random.default_rng(8)
    pc = [int(v) for v in rng.integers(0, p, 9)]
    # q = x gives p
    assert ocomp.compose(pc, [0, 1], p) == pc
    # q = constant c gives p(c) (and the remaining coefficients are zero)
    r = ocomp.compose(pc, [7, 0], p)
    assert r[0] == ocomp.horner_at(pc, 7, p) and all(v == 0 for v in r[1:])
    # p = x^k gives q^k, checked by evaluation at points
    qc = [int(v) for v in rng.integers(0, p, 4)]
    k = 5
    r = ocomp.compose([0] * k + [1], qc, p)
    for t in [2, 99, p - 3]:
        assert ocomp.horner_at(r, t, p) == pow(ocomp.horner_at(qc, t, p), k, p)
    # (1 + x) o (a + b x) = (1 + a) + b x, by hand
    assert ocomp.compose([1, 1], [5, 6], p) == [6, 6]


def test_compose_schwartz_zippel_and_native():
    p = P31
    rng = np.random.default_rng(9)
    P = rng.integers(0, p, size=(3, 32), dtype=np.uint32)
    Q = rng.integers(0, p, size=(3, 6), dtype=np.uint32)
    got = native.compose_modp(P, Q, p)
    for b in range(3):
        r = ocomp.compose(P[b].tolist(), Q[b].tolist(), p)
        assert got[b].tolist() == r
        for t in [3, 1000003, p - 2]:
            assert ocomp.horner_at(r, t, p) == ocomp.compose_at(P[b].tolist(), Q[b].tolist(), t, p)


def test_bigint_oracle_closed_forms_and_limbs():
    """The big-integer oracle against closed forms: (x + 1)^n by the binomial
    theorem and the geometric sum (x^(n+1) - 1) / (x - 1); limbs round trip."""
    from oracle import bigint
    g = np.random.default_rng(31)
    for n in (1, 7, 64, 255):
        x = int(g.integers(2, 2 ** 62)) * 2 ** 70 + 12345
        binom = [((e,), math.comb(n, e)) for e in range(n + 1)]
        assert bigint.eval_int(binom, x) == (x + 1) ** n
        geo = [((e,), 1) for e in range(n + 1)]
        assert bigint.eval_int(geo, x) * (x - 1) == x ** (n + 1) - 1
        v = bigint.eval_int(geo, x)
        nl = v.bit_length() // 16 + 1
        assert bigint.from_limbs(bigint.to_limbs(v, nl)) == v
