"""GPU big-integer evaluation (FPE_BIGINT) through the C-ABI, bit-exact
against the oracle's exact integers (p(x) = sum c_m x^m in Python ints), and
composition over the natural numbers at one big point against the oracle's
composition by its definition (sum c_m q^m)."""
import math

import numpy as np
import pytest
import torch

import paper_1307_5655_amd as fpe
from oracle import bigint

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def run(exps, coeffs, scheme, xs, lx, dev):
    t = fpe.Tree(np.asarray(exps, dtype=np.int32).reshape(-1, 1), np.asarray(coeffs, dtype=np.uint64), scheme,
                 fpe.BIGINT).upload(dev)
    xl = np.array([bigint.to_limbs(x, lx) for x in xs], dtype=np.int32)
    out = fpe.eval_bigint(t, torch.from_numpy(xl).to(dev))
    torch.cuda.synchronize()
    return out.cpu().numpy(), t


def check(got, exps, coeffs, xs):
    terms = [((int(e),), int(c)) for e, c in zip(exps, coeffs)]
    for r, x in enumerate(xs):
        want = bigint.eval_int(terms, x)
        assert bigint.from_limbs(got[r].astype(np.int64) & 0xFFFF) == want, r
        assert np.all((got[r] >= 0) & (got[r] < 1 << 16))


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced", "direct"])
def test_bigint_bit_exact(dev, scheme):
    # the direct scheme gives every term its own power: a degree that keeps
    # them all in the table (the big-integer walk computes no power on the fly)
    n = 28 if scheme == "direct" else 60
    say(f"bigint degree {n}, 96-bit points, {scheme}")
    g = np.random.default_rng([13075655, 7, 1])
    coeffs = [int(c) for c in g.integers(0, 2 ** 63, n + 1, dtype=np.uint64)]
    coeffs[-1] |= 1
    for k in g.choice(n, 6, replace=False):
        coeffs[int(k)] = 0
    coeffs[3] = 2 ** 64 - 1
    exps = [e for e in range(n + 1) if coeffs[e]]
    cs = [coeffs[e] for e in exps]
    xs = [int(g.integers(0, 2 ** 62)) << 34 | int(g.integers(0, 2 ** 30)) for _ in range(7)] + [0, 1]
    got, t = run(exps, cs, scheme, xs, 6, dev)
    check(got, exps, cs, xs)


@pytest.mark.parametrize("scheme", ["estrin", "balanced"])
def test_bigint_degree_255_batch(dev, scheme):
    say(f"bigint degree 255, 256-bit points, batch 40, {scheme}")
    g = np.random.default_rng([13075655, 7, 2])
    exps = list(range(256))
    cs = [int(c) | 1 for c in g.integers(0, 2 ** 63, 256, dtype=np.uint64)]
    xs = [int.from_bytes(g.bytes(32), "little") for _ in range(40)]
    got, t = run(exps, cs, scheme, xs, 16, dev)
    check(got, exps, cs, xs)


@pytest.mark.parametrize("scheme", ["horner", "balanced"])
def test_bigint_carry_chains(dev, scheme):
    """All-ones coefficients and points (2^64 - 1, 2^k - 1, 2^k) make the
    product columns' sums carry through long runs of 0xFFFF limbs, across
    the 64-column passes of the carry; values of several hundred limbs."""
    say(f"bigint carry chains, {scheme}")
    n = 40
    exps = list(range(n + 1))
    cs = [2 ** 64 - 1] * (n + 1)
    xs = [2 ** 256 - 1, 2 ** 255, 2 ** 200 - 1, 2 ** 64 - 1, 2 ** 128 + 2 ** 64 - 1, 1, 0, 3]
    got, t = run(exps, cs, scheme, xs, 16, dev)
    check(got, exps, cs, xs)


@pytest.mark.parametrize("scheme", ["horner", "balanced"])
def test_bigint_carry_across_ranges(dev, scheme):
    """Points 2^(16 m) - 1 (m limbs of 0xFFFF) make p(x) = x^2 + x + c0 carry
    from its low limbs through whole runs of propagating columns: results of
    450 to 10,000 limbs, whose carry is split into ranges over the
    workgroup's wavefronts (every column of a middle range propagates), with
    operands too long for LDS and columns in global memory at the top."""
    say(f"bigint carry across wavefront ranges, {scheme}")
    lx = 5000
    xs = [2 ** (16 * m) - 1 for m in (223, 446, 1000, 2047, 5000)] + [2 ** (16 * 5000) - 2, 2 ** (16 * 4999), 0, 1]
    for cs in ([1, 1, 1], [2 ** 64 - 1, 1, 1], [1, 2 ** 64 - 1, 1]):
        got, t = run([0, 1, 2], cs, scheme, xs, lx, dev)
        check(got, [0, 1, 2], cs, xs)
    # more points than compute units (the other workgroup width), rows checked
    # against the oracle and against the small batch
    many = xs * 34
    got_many, _ = run([0, 1, 2], [2 ** 64 - 1, 1, 1], scheme, many, lx, dev)
    check(got_many[::17], [0, 1, 2], [2 ** 64 - 1, 1, 1], many[::17])
    few, _ = run([0, 1, 2], [2 ** 64 - 1, 1, 1], scheme, xs, lx, dev)
    assert np.array_equal(got_many[:len(xs)], few)


def test_bigint_many_points(dev):
    """600 points (a workgroup each) against the oracle, and the first 40
    alone give the same limbs."""
    say("bigint 600 points")
    g = np.random.default_rng([13075655, 7, 3])
    n = 30
    exps = list(range(n + 1))
    cs = [int(c) | 1 for c in g.integers(0, 2 ** 63, n + 1, dtype=np.uint64)]
    xs = [int.from_bytes(g.bytes(12), "little") for _ in range(600)]
    got, t = run(exps, cs, "balanced", xs, 6, dev)
    check(got[::37], exps, cs, xs[::37])
    few, _ = run(exps, cs, "balanced", xs[:40], 6, dev)
    assert np.array_equal(few, got[:40])


def test_bigint_errors(dev):
    say("bigint errors")
    t = fpe.Tree(np.array([[0], [5]], dtype=np.int32), np.array([3, 4], dtype=np.uint64), "horner",
                 fpe.BIGINT).upload(dev)
    x = torch.zeros((2, 3), dtype=torch.int32, device=dev)
    with pytest.raises(fpe.FpeError):
        fpe.eval_bigint(t, x, lout=4)        # too few output limbs
    with pytest.raises(fpe.FpeError):
        fpe.evaluate(t, [torch.zeros(4, dtype=torch.float64, device=dev)])
    got = fpe.eval_bigint(t, x).cpu().numpy()   # p(0) = 3
    assert got[0, 0] == 3 and not got[0, 1:].any()


def run_point(exps, coeffs, scheme, x, lx, dev):
    t = fpe.Tree(np.asarray(exps, dtype=np.int32).reshape(-1, 1), np.asarray(coeffs, dtype=np.uint64), scheme,
                 fpe.BIGINT).upload(dev)
    xl = torch.from_numpy(np.array(bigint.to_limbs(x, lx), dtype=np.int32)).to(dev)
    out = fpe.eval_bigpoint(t, xl)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_point(got, exps, coeffs, x):
    terms = [((int(e),), int(c)) for e, c in zip(exps, coeffs)]
    assert np.all((got >= 0) & (got < 1 << 16))
    assert bigint.from_limbs(got.astype(np.int64) & 0xFFFF) == bigint.eval_int(terms, x)


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced", "balanced_floor"])
def test_bigpoint_one_large_point_exact(dev, scheme):
    """One polynomial at one big point (the Benchmarks section's setting):
    dense and sparse, term counts at and just past powers of two, points of
    1 to 512 limbs (products by transforms above 64 limbs per operand, up to
    2^14 limbs),
    64-bit coefficients including 2^64 - 1; every limb exact."""
    g = np.random.default_rng([13075655, 7, 50])
    for n, lx, sparse in [(1, 1, False), (7, 3, False), (63, 8, True), (64, 40, False), (65, 40, False),
                          (128, 64, False), (129, 64, True), (300, 20, True), (24, 512, False)]:
        say(f"bigpoint {scheme}: degree {n}, {lx} limbs, sparse={sparse}")
        exps = np.arange(n + 1)
        if sparse:
            exps = np.sort(np.concatenate([g.choice(n, n // 3, replace=False), [n]]))
            exps = np.unique(exps)
        coeffs = g.integers(1, 2 ** 63, len(exps), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        coeffs[-1] = np.uint64(2 ** 64 - 1)
        x = int.from_bytes(g.bytes(2 * lx), "little") | (1 << (16 * lx - 1))
        check_point(run_point(exps, coeffs, scheme, x, lx, dev), exps, coeffs, x)


def test_bigpoint_special_points_and_errors(dev):
    say("bigpoint: x = 0, 1, 2^16 - 1; errors")
    exps, coeffs = np.arange(33), np.full(33, 2 ** 64 - 1, dtype=np.uint64)
    for x, lx in [(0, 1), (1, 1), ((1 << 16) - 1, 1), (1 << 100, 8)]:
        check_point(run_point(exps, coeffs, "balanced", x, lx, dev), exps, coeffs, x)
    # p without a constant term: the root carries its own power
    check_point(run_point([5, 9, 30], [3, 1, 7], "estrin", 12345678901234567, 4, dev), [5, 9, 30], [3, 1, 7],
                12345678901234567)
    t = fpe.Tree(np.arange(5, dtype=np.int32).reshape(-1, 1), np.ones(5), "horner", fpe.F64).upload(dev)
    with pytest.raises(fpe.FpeError):
        fpe.eval_bigpoint(t, torch.zeros(4, dtype=torch.int32, device=dev))
    # a product beyond the largest transform is refused before any launch
    t = fpe.Tree(np.arange(41, dtype=np.int32).reshape(-1, 1), np.ones(41, dtype=np.uint64), "horner",
                 fpe.BIGINT).upload(dev)
    with pytest.raises(fpe.FpeError) as e:
        fpe.eval_bigpoint(t, torch.ones(1024, dtype=torch.int32, device=dev))
    assert "2^14" in str(e.value)


def compose_case(dev, p, q, scheme):
    """fpe_compose_bigint of p (dense coefficient list, zeros dropped) with q
    against the oracle's composition over the integers, every limb."""
    exps = [e for e, c in enumerate(p) if c]
    cs = [int(p[e]) for e in exps]
    t = fpe.Tree(np.asarray(exps, dtype=np.int32).reshape(-1, 1), np.asarray(cs, dtype=np.uint64), scheme,
                 fpe.BIGINT).upload(dev)
    got = fpe.compose_bigint(t, q)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    want = bigint.compose_int([((e,), c) for e, c in zip(exps, cs)], q)
    assert g.shape[0] == len(want)
    assert np.all((g >= 0) & (g < 1 << 16))
    for k, w in enumerate(want):
        assert bigint.from_limbs(g[k].astype(np.int64)) == w, k
    return g


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_compose_bigint_exact(dev, scheme):
    """p(q(X)) over the natural numbers (Kronecker substitution into the walk
    at one big point): 64-bit coefficients with zeros in both polynomials,
    every coefficient of the result exact."""
    say(f"compose bigint, {scheme}")
    g = np.random.default_rng([13075655, 9, 1])
    p = [int(c) for c in g.integers(0, 2 ** 63, 21, dtype=np.uint64) * 2 + 1]
    p[4] = p[11] = 0
    p[7] = 2 ** 64 - 1
    q = [2 ** 64 - 1, 0, int(g.integers(1, 2 ** 63)), 12345]
    compose_case(dev, p, q, scheme)
    # term counts at and past a power of two, q of degree 3
    for n in (16, 17, 33):
        p = [int(c) | 1 for c in g.integers(0, 2 ** 63, n, dtype=np.uint64)]
        compose_case(dev, p, [int(c) for c in g.integers(0, 2 ** 63, 4, dtype=np.uint64)], scheme)


def test_compose_bigint_special_cases(dev):
    """Closed forms and degenerate inputs: X^n o (X + 1) gives the binomial
    coefficients; q = X gives p back; a constant q gives the constant p(q);
    a constant p gives itself; a single-term p; q with a zero constant."""
    say("compose bigint special cases")
    for n in (1, 12, 40):
        p = [0] * n + [1]
        r = compose_case(dev, p, [1, 1], "balanced")
        assert [bigint.from_limbs(r[k].astype(np.int64)) for k in range(n + 1)] == [math.comb(n, k) for k in range(n + 1)]
    p = [3, 0, 2 ** 64 - 1, 7, 1]
    compose_case(dev, p, [0, 1], "estrin")
    compose_case(dev, p, [2 ** 40 + 3], "horner")
    compose_case(dev, [5], [1, 2, 3], "horner")
    compose_case(dev, [0, 0, 0, 9], [0, 2 ** 63, 1], "balanced")
    # the zero polynomial inside: only p(0) is left
    compose_case(dev, [7, 3, 0, 2 ** 64 - 1], [0], "estrin")
    compose_case(dev, [7, 3, 0, 2 ** 64 - 1], [0, 0, 0], "balanced")


def test_compose_bigint_limits(dev):
    """q of 65 coefficients and results beyond the big-point walk's 2^14-limb
    products are refused; the largest bench size runs."""
    say("compose bigint limits")
    t = fpe.Tree(np.arange(3, dtype=np.int32).reshape(-1, 1), np.array([1, 2, 3], dtype=np.uint64), "horner",
                 fpe.BIGINT).upload(dev)
    with pytest.raises(fpe.FpeError):
        fpe.compose_bigint(t, [1] * 65)
    big = fpe.Tree(np.arange(200, dtype=np.int32).reshape(-1, 1), np.full(200, 2 ** 63, dtype=np.uint64),
                   "balanced", fpe.BIGINT).upload(dev)
    with pytest.raises(fpe.FpeError):
        fpe.compose_bigint(big, [2 ** 63] * 8)
    g = np.random.default_rng([13075655, 9, 2])
    p = [int(c) | 1 for c in g.integers(0, 2 ** 63, 34, dtype=np.uint64)]
    compose_case(dev, p, [int(c) for c in g.integers(0, 2 ** 63, 4, dtype=np.uint64)], "balanced")
    # every coefficient at its largest: the slot bound is met with the least slack
    compose_case(dev, [2 ** 64 - 1] * 30, [2 ** 64 - 1] * 4, "estrin")
