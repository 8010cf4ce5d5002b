"""The seeded input generators: the pooled served stream draws the same
request mix as the plain one, and every request's points are a window of
the shared pool."""
import math

import numpy as np

import fpe_inputs


def test_pooled_served_stream_windows_and_ranges():
    s = fpe_inputs.served_stream_pooled(300, rate_per_s=50.0, pool_pts=1_200_000)
    assert s.pool.shape == (3, 1_200_000)
    assert np.all(np.abs(s.pool) <= 1.0)
    last = 0.0
    for r, off in zip(s.requests, s.offsets):
        m = r.poly
        v, n = m.points.shape
        T = len(m.coeffs)
        assert 1 <= v <= 3 and 1_000 <= n <= 1_000_000 and 10 <= T <= 10_000
        assert r.scheme in ("horner", "estrin", "balanced")
        assert r.arrival_s > last
        last = r.arrival_s
        # the points are the pool's window, shared, not a copy
        assert np.shares_memory(m.points, s.pool)
        assert np.array_equal(m.points, s.pool[:v, off:off + n])
        # distinct monomials of total degree <= D, D minimal for T terms
        assert len({tuple(e) for e in m.exps}) == T
        D = int(m.exps.sum(axis=1).max())
        assert math.comb(D + v, v) >= T
        assert np.all((m.coeffs >= -1.0) & (m.coeffs <= 1.0) & (m.coeffs != 0.0))
    # log-uniform sizes span the ranges; the schemes and variable counts all occur
    ns = np.array([r.poly.points.shape[1] for r in s.requests])
    assert ns.min() < 3_000 and ns.max() > 300_000
    assert {r.scheme for r in s.requests} == {"horner", "estrin", "balanced"}
    assert {r.poly.points.shape[0] for r in s.requests} == {1, 2, 3}


def test_pooled_served_stream_is_seeded():
    a = fpe_inputs.served_stream_pooled(20, rate_per_s=1.0, pool_pts=1_000_000)
    b = fpe_inputs.served_stream_pooled(20, rate_per_s=1.0, pool_pts=1_000_000)
    assert a.offsets == b.offsets
    for x, y in zip(a.requests, b.requests):
        assert x.arrival_s == y.arrival_s and x.scheme == y.scheme
        assert np.array_equal(x.poly.exps, y.poly.exps) and np.array_equal(x.poly.coeffs, y.poly.coeffs)
