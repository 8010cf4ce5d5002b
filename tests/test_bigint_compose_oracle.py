"""Pins of the oracle's composition over the integers (oracle.bigint.compose_int)
against closed forms and against evaluation: p(q(X)) with q = X + 1 and
p = X^n gives the binomial coefficients; q = X gives p back; a constant q
gives the constant p(q); and at any integer x the composed polynomial takes
the value p(q(x)) (evaluation is a ring homomorphism)."""
import math
import random

from oracle import bigint


def terms_of(coeffs):
    return [((e,), c) for e, c in enumerate(coeffs) if c]


def test_binomial_expansion():
    for n in (0, 1, 2, 7, 20, 64):
        got = bigint.compose_int([((n,), 1)], [1, 1])
        assert got == [math.comb(n, k) for k in range(n + 1)]


def test_identity_and_constant_inner_polynomial():
    rng = random.Random(13075655)
    p = [rng.getrandbits(64) for _ in range(17)]
    assert bigint.compose_int(terms_of(p), [0, 1]) == p
    for c in (0, 1, 2, 2 ** 64 - 1):
        assert bigint.compose_int(terms_of(p), [c]) == [bigint.eval_int(terms_of(p), c)]


def test_values_match_evaluation():
    rng = random.Random(7)
    for _ in range(20):
        dp, dq = rng.randint(0, 12), rng.randint(0, 6)
        p = [rng.getrandbits(rng.choice([1, 16, 64])) for _ in range(dp + 1)]
        p[-1] |= 1
        q = [rng.getrandbits(rng.choice([1, 16, 64])) for _ in range(dq + 1)]
        r = bigint.compose_int(terms_of(p), q)
        assert len(r) == dp * dq + 1
        for x in (0, 1, 3, 2 ** 70 + 5):
            qx = sum(c * x ** j for j, c in enumerate(q))
            assert sum(c * x ** k for k, c in enumerate(r)) == bigint.eval_int(terms_of(p), qx)


def test_sparse_outer_polynomial():
    # p = 5 X^3 + 2, q = X^2 + 3: 5 (X^2 + 3)^3 + 2 = 5 X^6 + 45 X^4 + 135 X^2 + 137
    assert bigint.compose_int([((3,), 5), ((0,), 2)], [3, 0, 1]) == [137, 0, 135, 0, 45, 0, 5]
