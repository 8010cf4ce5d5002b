"""GPU: the compensated-FP32 form at the edges of the FP32 range.

The double-float walk's running bound is relative to the values it carries;
its absolute part covers roundings below the normal FP32 range, constants
that do not split into two normal floats and powers that underflow.  Every
point must come back within 1e-12 relative of the oracle (either certified
by the bound or re-evaluated by the fallback), and wherever a point was not
re-evaluated, the bound the walk reported must be at least its true error."""
import math

import numpy as np
import pytest
import torch

import fpe_inputs
import paper_1307_5655_amd as fpe
from oracle import exact, native

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(msg):
    print(msg, flush=True)


def run(coeffs_by_exp, x, scheme, dev):
    """Evaluate the univariate polynomial {exponent: coefficient} at x with
    the compensated form; return values, fallback flags and bounds."""
    ex = np.array(sorted(coeffs_by_exp), dtype=np.int32).reshape(-1, 1)
    co = np.array([coeffs_by_exp[int(e)] for e in ex[:, 0]], dtype=np.float64)
    t = fpe.Tree(ex, co, scheme, fpe.F32C).upload(dev)
    n = len(x)
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    flags = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
    bound = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    y = fpe.evaluate(t, [xd], flags_out=flags, bound_out=bound)
    torch.cuda.synchronize()
    fl = np.unpackbits(flags.cpu().numpy().view(np.uint8), bitorder="little")[:n].astype(bool)
    return y.cpu().numpy(), fl, bound.cpu().numpy(), ex, co


def dense(cbe):
    n = max(cbe)
    c = np.zeros(n + 1)
    for e, v in cbe.items():
        c[e] = v
    return c


def check(y, fl, bound, cbe, x):
    c = dense(cbe)
    ref = native.dd_value(c, x)
    rel = np.abs(y - ref) / np.abs(ref)
    assert np.all(rel <= TOL), f"worst {np.nanmax(rel):.3e} at x={x[~(rel <= TOL)][:3]}"
    # the reported bound covers the true error wherever the point was kept
    # (the oracle's own error, at most about 2n 2^-104 of p~, is the slack)
    keep = ~fl
    slack = native.ptilde(c, x) * 2.0 ** -88
    assert np.all(np.abs(y[keep] - ref[keep]) <= bound[keep] + slack[keep])
    return rel


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_tiny_coefficient_dominates_above_one(dev, scheme):
    # 1e-40 splits into floats below the normal range (the low part is lost)
    # and dominates near x = 2: 1e-40 * 2^100 = 1.27e-10 against 1e-10
    say(f"f32c range: 1e-40 x^100 + 1e-10, {scheme}")
    cbe = {100: 1e-40, 0: 1e-10, 1: 3e-12}
    x = np.linspace(1.9, 2.1, 4001)
    y, fl, bound, *_ = run(cbe, x, scheme, dev)
    check(y, fl, bound, cbe, x)


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_inverse_factorial_coefficients(dev, scheme):
    # the Taylor polynomial of exp of degree 80: 1/k! drops below 2^-100 at
    # k = 30 and below the smallest float at k = 35, yet x^k / k! matters for
    # x up to 20
    say(f"f32c range: 1/k! degree 80, {scheme}")
    cbe = {k: 1.0 / math.factorial(k) for k in range(81)}
    x = np.concatenate([np.linspace(-8, 20, 3001), [0.0, 1e-30, -1e-30, 1.0]])
    y, fl, bound, *_ = run(cbe, x, scheme, dev)
    check(y, fl, bound, cbe, x)


def test_subnormal_coefficient_single_term(dev):
    # a coefficient below the smallest normal float (1.18e-38) times x^30 at
    # x = 2: the value is 1.3e-30 and only the fallback can give it to 1e-12
    say("f32c range: subnormal coefficient")
    cbe = {30: 1.2345678901234e-39}
    x = np.array([2.0, -2.0, 1.5, 3.0, 0.5])
    for scheme in ("horner", "balanced"):
        y, fl, bound, *_ = run(cbe, x, scheme, dev)
        check(y, fl, bound, cbe, x)


def test_tiny_points_and_underflowing_powers(dev):
    # large coefficients times powers that fall below the normal FP32 range
    # (x^2 at x ~ 2^-70 is a subnormal float with a few bits)
    say("f32c range: underflowing powers")
    g = np.random.default_rng([13075655, 910])
    cbe = {2: 1e30, 1: -3.0e-11, 0: 1e-25, 4: 7e38 / 1e10}
    x = np.concatenate([g.uniform(1.0, 1.2, 500) * 2.0 ** -70, -g.uniform(1.0, 1.2, 500) * 2.0 ** -70,
                        g.uniform(-1e-20, 1e-20, 200)])
    for scheme in ("horner", "estrin"):
        y, fl, bound, *_ = run(cbe, x, scheme, dev)
        check(y, fl, bound, cbe, x)


def test_overflow_band_and_large_points(dev):
    # values beyond the FP32 range are flagged and re-evaluated in FP64
    say("f32c range: FP32 overflow band")
    inp = fpe_inputs.sparse_uni(3000, npts=20_000 + 3, lo=-1.2, hi=1.2)
    cbe = {int(e): float(inp.coeffs[e]) for e in np.nonzero(inp.coeffs)[0]}
    for scheme in ("horner", "balanced"):
        y, fl, bound, *_ = run(cbe, inp.points, scheme, dev)
        check(y, fl, bound, cbe, inp.points)
        assert fl[np.abs(inp.points) > 1.04].all()


def test_non_finite_points(dev):
    say("f32c range: NaN and infinite points")
    cbe = {0: 0.5, 1: -1.0, 3: 0.25, 10: 1e-3}
    x = np.array([np.nan, np.inf, -np.inf, 0.5, -0.25, 1.0])
    for scheme in ("horner", "estrin", "balanced"):
        y, fl, bound, *_ = run(cbe, x, scheme, dev)
        assert fl[:3].all()
        assert not np.isfinite(y[:3]).any()
        assert np.isnan(y[0])
        c = dense(cbe)
        ref = native.dd_value(c, x[3:])
        assert np.all(np.abs(y[3:] - ref) <= TOL * np.abs(ref))


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_bound_covers_true_error_on_the_workload(dev, scheme):
    # the benchmark's polynomials (degree 3000, 10 % zeros) at points of the
    # benchmark's range: every kept point's reported bound is at least its
    # true error against the oracle
    say(f"f32c bound vs true error, {scheme}")
    inp = fpe_inputs.sparse_uni(3000, npts=30_000 + 11)
    cbe = {int(e): float(inp.coeffs[e]) for e in np.nonzero(inp.coeffs)[0]}
    y, fl, bound, *_ = run(cbe, inp.points, scheme, dev)
    check(y, fl, bound, cbe, inp.points)
    # the bound is not vacuous: most points near |x| < 0.9 are certified
    inner = np.abs(inp.points) < 0.9
    assert (~fl[inner]).mean() > 0.8
