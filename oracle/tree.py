"""Independent builder and evaluator of evaluation trees (oracle side).

Follows the paper's definitions directly:

* evaluation tree and its value: Section 1, Definition of evaluation tree
  (T(x) = c(R) x^{d(R)} for a single node, else (c(R) + sum S_i(x)) x^{d(R)});
* partial degree vs monomial degree: Section 1, the paragraph after the
  definition (the monomial degree is the sum of the partial degrees on the
  path from the root);
* topological order <_t: Section 1 (decreasing lexicographic order of the
  monomials, index 0 is the biggest node, the root is last);
* T_p^f: Section 1.1, Definition of function scheme (p = a x^{f(n)} + b, T_a
  becomes a child of the root of T_b);
* multivariate: Section 1.1, Remark (the scheme applied recursively to each
  variable);
* lazy height: Section 1.3, Definition;
* coefficient walk: Section 2.1.

Readings where the paper is silent (also listed in the design notes):

* f takes the degree n of the current sub-polynomial, measured from the
  exponent origin of that sub-polynomial (a is divided by x^{f(n)}, b is not
  re-based).
* if b = 0 the split adds no node: T_p is T_a with its origin moved by f(n).
* partial degrees are d(N) = exp(N) - exp(parent(N)) componentwise, and
  d(root) = exp(root).
* multivariate nesting: x1 is the outermost variable; the node of an outer
  block whose coefficient polynomial has a constant term is that polynomial's
  own root; otherwise a junction node with coefficient 0 and the block's
  exponent is inserted above it.
* the walk uses the "safe" slot rule 0 if <= 1 child, else
  1 + max_{i >= 2} H(C_i) with H the largest slot in a subtree; the paper's
  lazy height is also computed, and equals the safe slot on dense trees.
"""
from __future__ import annotations

import sys
from dataclasses import dataclass, field
from typing import Callable, Sequence

# Hörner trees are chains as deep as the degree
sys.setrecursionlimit(max(sys.getrecursionlimit(), 200_000))


@dataclass(eq=False)
class Node:
    exps: tuple
    coef: object
    children: list = field(default_factory=list)   # in <_t order, C_1 first
    parent: "Node | None" = None
    junction: bool = False
    index: int = -1
    pdeg: tuple = ()


class SchemeError(ValueError):
    pass


def _split_build(items, origin: int, k: int, f: Callable[[int], int], make_node):
    """Build T_p^f for p = sum_{(e, payload) in items} payload * x_k^(e - origin).

    ``items`` is sorted by exponent, largest first (Section 1.1 Definition)."""
    if len(items) == 1:
        return make_node(items[0])
    n = items[0][0] - origin
    s = f(n)
    if not (0 < s <= n):
        raise SchemeError(f"scheme returned f({n}) = {s}, outside [1, {n}]")
    a = [it for it in items if it[0] >= origin + s]
    b = [it for it in items if it[0] < origin + s]
    if not b:
        # p = a x^{f(n)}: no new node, the origin of a moves by f(n)
        return _split_build(a, origin + s, k, f, make_node)
    ra = _split_build(a, origin + s, k, f, make_node)
    rb = _split_build(b, origin, k, f, make_node)
    rb.children.insert(0, ra)        # T_a is the biggest child of root(T_b)
    ra.parent = rb
    return rb


def build_tree(terms: Sequence, f, nvars: int | None = None, zero=0) -> list:
    """Evaluation tree of a polynomial given as (exponent tuple, coef) pairs.

    Returns the nodes in <_t order (index 0 = biggest monomial, root last),
    each with ``index``, ``parent``, ``children`` and ``pdeg`` set.  Zero
    coefficients are dropped; duplicate monomials are an error."""
    d = {}
    for m, c in terms:
        m = tuple(int(v) for v in (m if hasattr(m, "__len__") else (m,)))
        if any(v < 0 for v in m):
            raise ValueError("negative exponent")
        if m in d:
            raise ValueError(f"duplicate monomial {m}")
        if c != 0:
            d[m] = c
    if not d:
        raise ValueError("empty polynomial")
    if nvars is None:
        nvars = len(next(iter(d)))
    fs = f if isinstance(f, (list, tuple)) else [f] * nvars
    root = _nested_multi(d, nvars, fs)
    nodes = []

    def collect(n):
        nodes.append(n)
        for ch in n.children:
            collect(ch)
    collect(root)
    nodes.sort(key=lambda n: n.exps, reverse=True)
    for i, n in enumerate(nodes):
        n.index = i
    for n in nodes:
        base = n.parent.exps if n.parent is not None else (0,) * nvars
        n.pdeg = tuple(a - b for a, b in zip(n.exps, base))
        if any(v < 0 for v in n.pdeg) or (n.parent is not None and not any(n.pdeg)):
            raise AssertionError("partial degree must be >= 0 and nonzero")
        if n.parent is not None and n.parent.index <= n.index:
            raise AssertionError("<_t is not topological")
    assert nodes[-1] is root
    return nodes


def _nested_multi(d, nvars, fs):
    # the same scheme per variable by default; fs[k] may differ per variable
    return _nested_fs(d, 0, nvars, (), fs)


def _nested_fs(terms, k, nvars, prefix, fs):
    """Tree of sum_{m in terms} c_m x^m where every m starts with ``prefix``
    and ``terms`` maps the remaining exponents (vars k..nvars-1) to c."""
    blocks: dict = {}
    for m, c in terms.items():
        blocks.setdefault(m[0], {})[m[1:]] = c
    items = sorted(blocks.items(), key=lambda t: -t[0])

    def make_node(item):
        e, sub = item
        here = prefix + (e,)
        if k == nvars - 1:
            (c,) = sub.values()
            return Node(exps=here, coef=c)
        inner = _nested_fs(sub, k + 1, nvars, here, fs)
        if all(v == 0 for v in inner.exps[k + 1:]):
            return inner
        j = Node(exps=here + (0,) * (nvars - k - 1), coef=0, junction=True)
        j.children.append(inner)
        inner.parent = j
        return j

    return _split_build(items, 0, k, fs[k], make_node)


def dense_terms(coeffs) -> list:
    """(exponent, coef) pairs of a univariate coefficient list (index = exp)."""
    return [((e,), c) for e, c in enumerate(coeffs) if c != 0]


# ----------------------------------------------------------------------------
# values
# ----------------------------------------------------------------------------

def tree_value(nodes, x: Sequence, add=lambda a, b: a + b, mul=lambda a, b: a * b,
               one=1, zero=0):
    """The recursive value of the tree (Section 1, Definition of evaluation
    tree) over any ring given by add/mul: value(N) = (c(N) + sum value(C))
    * prod_j x_j^{d_j(N)}."""
    def power(v, e):
        r = one
        for _ in range(e):
            r = mul(r, v)
        return r

    val = {}
    for n in nodes:                         # children come first in <_t
        acc = n.coef
        for ch in n.children:
            acc = add(acc, val[ch.index])
        for j, e in enumerate(n.pdeg):
            if e:
                acc = mul(acc, power(x[j], e))
        val[n.index] = acc
    return val[nodes[-1].index]


def lazy_heights(nodes) -> list:
    """lh(N) = 0 with 0 or 1 child, else max_{i >= 2} lh(C_i) + 1 (Section 1.3)."""
    lh = [0] * len(nodes)
    for n in nodes:
        if len(n.children) >= 2:
            lh[n.index] = 1 + max(lh[c.index] for c in n.children[1:])
    return lh


def safe_slots(nodes) -> list:
    """slot(N) = 0 with <= 1 child, else 1 + max_{i >= 2} H(C_i), where H is the
    largest slot in a subtree (the reading used for the walk)."""
    slot = [0] * len(nodes)
    H = [0] * len(nodes)
    for n in nodes:
        i = n.index
        if len(n.children) >= 2:
            slot[i] = 1 + max(H[c.index] for c in n.children[1:])
        H[i] = max([slot[i]] + [H[c.index] for c in n.children])
    return slot


def classical_heights(nodes) -> list:
    h = [0] * len(nodes)
    for n in nodes:
        if n.children:
            h[n.index] = 1 + max(h[c.index] for c in n.children)
    return h


def walk(nodes, x: Sequence, slots=None, add=lambda a, b: a + b,
         mul=lambda a, b: a * b, one=1, zero=0):
    """The coefficient walk of Section 2.1: for i = 0..n,
    p = (m[h] + c) x^d; m[h] = 0; the root returns p, every other node adds p
    into m[h(parent)].  ``slots`` defaults to the safe slots."""
    if slots is None:
        slots = safe_slots(nodes)

    def power(v, e):
        r = one
        for _ in range(e):
            r = mul(r, v)
        return r

    L = max(slots) + 1
    m = [zero] * L
    for n in nodes:
        h = slots[n.index]
        p = add(m[h], n.coef)
        for j, e in enumerate(n.pdeg):
            if e:
                p = mul(p, power(x[j], e))
        m[h] = zero
        if n.parent is None:
            return p
        hp = slots[n.parent.index]
        m[hp] = add(m[hp], p)
    raise AssertionError("root not reached")


def distinct_partial_degrees(nodes, var: int = 0) -> set:
    return {n.pdeg[var] for n in nodes if n.pdeg[var] != 0}
