"""Function schemes f: N -> N with 0 < f(k) <= k (Section 1.1, Definition of
function scheme; Section 1.2 for the balanced scheme).

The argument k is the degree n of the sub-polynomial being split
(p = a x^{f(n)} + b).  The balanced scheme is read as B(n) = ceil(n / 2) on the
degree, which equals floor(#terms / 2) for a dense polynomial with n + 1 terms;
the literal floor(n / 2) (illegal at n = 1) is kept as ``balanced_literal``
with f(1) := 1, for comparison only.
"""


def direct(k: int) -> int:
    """D(k) = k (Section 1.1)."""
    return k


def horner(k: int) -> int:
    """H(k) = 1 (Section 1.1)."""
    return 1


def estrin(k: int) -> int:
    """E(k) = 2^floor(log2 k) (Section 1.1)."""
    e = 1
    while e * 2 <= k:
        e *= 2
    return e


def balanced(k: int) -> int:
    """B(n) = ceil(n / 2) on the degree n (Section 1.2, read on the degree)."""
    return (k + 1) // 2


def balanced_literal(k: int) -> int:
    """floor(k / 2) as printed, with f(1) := 1 to stay legal (comparison only)."""
    return max(1, k // 2)


def threshold(t: int):
    """The combined scheme of the Remark in Section 1.1: E above t, H below."""
    def f(k: int) -> int:
        return estrin(k) if k > t else 1
    return f


def table(values):
    """A user scheme given as a table f(k) = values[k] (Section 1.1 Remark)."""
    vals = list(values)

    def f(k: int) -> int:
        return vals[k]
    return f


BY_NAME = {
    "direct": direct,
    "horner": horner,
    "estrin": estrin,
    "balanced": balanced,
    "balanced_literal": balanced_literal,
}
