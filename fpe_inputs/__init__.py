"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays them out. It holds none of the
evaluation method's arithmetic (no tree building, no walk, no reduction beyond
canonicalising an integer residue into [0, p)), so that both the CPU oracle and
the GPU path can consume identical inputs without sharing any code.

Workloads (all synthetic; the paper measures on no public dataset):

* ``dense_uni``     one dense FP64 polynomial, degree 1023, coefficients
                    U[-1, 1], 1e5 points U[-1, 1]; Hörner and Estrin schemes.
* ``sparse_uni``    degrees 3000 and 5000, coefficients U[-1, 1] with exactly
                    floor(0.1 (n + 1)) of the exponents 0..n-1 zeroed (the
                    leading coefficient is kept so the degree is exact), 1e7
                    points U[-1.05, 1.05].
* ``trivariate``    all 12,341 monomials of total degree <= 40 in x1 > x2 > x3
                    (lexicographic), int64 coefficients reduced mod 2^61 - 1,
                    1e6 points uniform in (Z/pZ)^3.
* ``compose``       4096 instances of p (degree 255) and q (degree 15), all
                    coefficients uniform in [0, 2^31 - 2].
* ``interval``      boxes around the points of the workloads above: each
                    interval has a width drawn from {0, 2^-20, 2^-8, 0.25} and
                    holds its point at a uniform position (``interval_boxes``).
* ``served``        a Poisson stream of evaluate requests with 1-3 variables,
                    10-10,000 terms (log-uniform), 1e3-1e6 points (log-uniform)
                    in the unit box [-1, 1]^v and a scheme in {H, E, B}.

Seeds: ``numpy.random.default_rng([13075655, k])`` for workload k (1-based, in
the order above).  Draw order: coefficients (ascending exponent, lex order for
the trivariate case), then the zero mask, then the points.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 13075655
P61 = (1 << 61) - 1
P31 = (1 << 31) - 1


def rng_for(k: int, sub: int | None = None) -> np.random.Generator:
    """The generator for workload ``k`` (optionally a sub-stream ``sub``)."""
    if sub is None:
        return np.random.default_rng([SEED_BASE, k])
    return np.random.default_rng([SEED_BASE, k, sub])


# ----------------------------------------------------------------------------
# univariate FP64 workloads
# ----------------------------------------------------------------------------

@dataclass
class UniInput:
    coeffs: np.ndarray   # float64, index = exponent, length n + 1 (zeros kept)
    points: np.ndarray   # float64

    @property
    def degree(self) -> int:
        return len(self.coeffs) - 1

    def terms(self):
        """Nonzero terms as (exponents int32 [T, 1], coeffs float64 [T])."""
        e = np.nonzero(self.coeffs)[0].astype(np.int32)
        return e.reshape(-1, 1), self.coeffs[e].copy()


def dense_uni(npts: int = 100_000, degree: int = 1023, seed_k: int = 1) -> UniInput:
    g = rng_for(seed_k)
    c = g.uniform(-1.0, 1.0, degree + 1)
    x = g.uniform(-1.0, 1.0, npts)
    return UniInput(c, x)


def sparse_uni(degree: int, npts: int = 10_000_000, zero_frac: float = 0.1,
               lo: float = -1.05, hi: float = 1.05, seed_k: int = 2) -> UniInput:
    g = rng_for(seed_k, degree)
    c = g.uniform(-1.0, 1.0, degree + 1)
    nz = int(math.floor(zero_frac * (degree + 1)))
    if nz:
        z = g.choice(degree, nz, replace=False)   # exponents 0..n-1 only
        c[z] = 0.0
    x = g.uniform(lo, hi, npts)
    return UniInput(c, x)


# ----------------------------------------------------------------------------
# trivariate mod 2^61 - 1 workload
# ----------------------------------------------------------------------------

def monomials_total_degree(nvars: int, total: int) -> np.ndarray:
    """All exponent vectors with sum <= total, in decreasing lex order."""
    out = []

    def rec(prefix, left, k):
        if k == nvars - 1:
            for e in range(left, -1, -1):
                out.append(prefix + [e])
            return
        for e in range(left, -1, -1):
            rec(prefix + [e], left - e, k + 1)

    rec([], total, 0)
    return np.array(out, dtype=np.int32)


@dataclass
class ModInput:
    exps: np.ndarray     # int32 [T, v]
    coeffs: np.ndarray   # uint64 residues in [0, p)
    points: np.ndarray   # uint64 [v, N] residues (SoA)
    modulus: int


def canonical_residues(vals: np.ndarray, p: int) -> np.ndarray:
    """Floor-mod canonicalisation of signed integers into [0, p)."""
    return np.array([int(v) % p for v in vals.tolist()], dtype=np.uint64)


def trivariate(npts: int = 1_000_000, total: int = 40, seed_k: int = 3) -> ModInput:
    g = rng_for(seed_k)
    ex = monomials_total_degree(3, total)
    # coefficients in ascending lex order of the monomials, then stored in
    # the (decreasing) order of ``ex``
    raw = g.integers(-(1 << 63), (1 << 63) - 1, size=len(ex), dtype=np.int64, endpoint=True)
    raw = raw[::-1].copy()
    co = canonical_residues(raw, P61)
    pts = g.integers(0, P61, size=(3, npts), dtype=np.uint64)   # [0, p)
    return ModInput(ex, co, pts, P61)


def random_modp_poly(nvars: int, nterms: int, max_total: int, npts: int, p: int = P61,
                     seed=(7,)) -> ModInput:
    """A sparse multivariate polynomial mod p: a uniform subset of monomials."""
    g = np.random.default_rng([SEED_BASE, 90, *seed])
    allm = monomials_total_degree(nvars, max_total)
    nterms = min(nterms, len(allm))
    pick = np.sort(g.choice(len(allm), nterms, replace=False))
    ex = allm[pick]
    co = g.integers(0, p, size=nterms, dtype=np.uint64)
    pts = g.integers(0, p, size=(nvars, npts), dtype=np.uint64)
    return ModInput(ex, co, pts, p)


# ----------------------------------------------------------------------------
# composition workload
# ----------------------------------------------------------------------------

@dataclass
class ComposeInput:
    p: np.ndarray   # uint32 [B, dp + 1], index = exponent
    q: np.ndarray   # uint32 [B, dq + 1]
    modulus: int


def compose_batch(batch: int = 4096, dp: int = 255, dq: int = 15, seed_k: int = 4) -> ComposeInput:
    g = rng_for(seed_k)
    p = g.integers(0, P31 - 1, size=(batch, dp + 1), dtype=np.uint32, endpoint=True)
    q = g.integers(0, P31 - 1, size=(batch, dq + 1), dtype=np.uint32, endpoint=True)
    return ComposeInput(p, q, P31)


# ----------------------------------------------------------------------------
# multivariate FP64 (served) polynomials
# ----------------------------------------------------------------------------

def interval_boxes(points: np.ndarray, g: np.random.Generator,
                   widths=(0.0, 2.0 ** -20, 2.0 ** -8, 0.25)) -> np.ndarray:
    """Intervals (lo, hi) around ``points`` (any shape): a width w drawn
    uniformly from ``widths`` per point and a position u ~ U[0, 1], lo = x - u w,
    hi = x + (1 - u) w.  Returns float64 [..., 2]."""
    x = np.asarray(points, dtype=np.float64)
    w = np.asarray(widths, dtype=np.float64)[g.integers(0, len(widths), size=x.shape)]
    u = g.uniform(0.0, 1.0, size=x.shape)
    lo = x - u * w
    hi = x + (1.0 - u) * w
    return np.ascontiguousarray(np.stack([lo, hi], axis=-1))


@dataclass
class MultiInput:
    exps: np.ndarray     # int32 [T, v]
    coeffs: np.ndarray   # float64 [T]
    points: np.ndarray   # float64 [v, N] (SoA)


def random_multi_f64(nvars: int, nterms: int, npts: int, g: np.random.Generator,
                     lo: float = -1.0, hi: float = 1.0) -> MultiInput:
    """T monomials drawn uniformly from those of total degree <= D, D minimal
    with C(D + v, v) >= T; coefficients U[-1, 1]; points U[lo, hi]^v."""
    D = 0
    while math.comb(D + nvars, nvars) < nterms:
        D += 1
    allm = monomials_total_degree(nvars, D)
    pick = np.sort(g.choice(len(allm), nterms, replace=False))
    ex = allm[pick]
    co = g.uniform(-1.0, 1.0, nterms)
    co[co == 0.0] = 0.5
    pts = g.uniform(lo, hi, size=(nvars, npts))
    return MultiInput(ex, co, pts)


@dataclass
class Request:
    arrival_s: float
    scheme: str          # "horner" | "estrin" | "balanced"
    poly: MultiInput


def served_stream(nreq: int, rate_per_s: float, seed_k: int = 5,
                  max_terms: int = 10_000, max_pts: int = 1_000_000,
                  min_terms: int = 10, min_pts: int = 1_000) -> list[Request]:
    """Poisson arrivals of evaluate requests (log-uniform terms and points)."""
    g = rng_for(seed_k)
    t = 0.0
    out = []
    for _ in range(nreq):
        t += g.exponential(1.0 / rate_per_s)
        v = int(g.integers(1, 4))
        T = int(round(math.exp(g.uniform(math.log(min_terms), math.log(max_terms)))))
        N = int(round(math.exp(g.uniform(math.log(min_pts), math.log(max_pts)))))
        scheme = ["horner", "estrin", "balanced"][int(g.integers(0, 3))]
        out.append(Request(t, scheme, random_multi_f64(v, T, N, g)))
    return out


@dataclass
class PooledStream:
    requests: list[Request]   # poly.points of each is a view of ``pool``
    pool: np.ndarray          # float64 [3, P], U[-1, 1]
    offsets: list[int]        # request k reads pool[:v, offsets[k]:offsets[k] + N]


def served_stream_pooled(nreq: int, rate_per_s: float, pool_pts: int = 4_000_000, seed_k: int = 7,
                         max_terms: int = 10_000, max_pts: int = 1_000_000,
                         min_terms: int = 10, min_pts: int = 1_000) -> PooledStream:
    """The served stream's request mix (as ``served_stream``) for long runs
    (10^4 requests and more): each request's points are a window of one shared
    pool of uniform points at a random offset, so the points of all requests
    fit in a few arrays however many requests there are."""
    assert pool_pts >= max_pts
    g = rng_for(seed_k)
    pool = g.uniform(-1.0, 1.0, size=(3, pool_pts))
    mono = {}
    t = 0.0
    reqs, offs = [], []
    for _ in range(nreq):
        t += g.exponential(1.0 / rate_per_s)
        v = int(g.integers(1, 4))
        T = int(round(math.exp(g.uniform(math.log(min_terms), math.log(max_terms)))))
        N = int(round(math.exp(g.uniform(math.log(min_pts), math.log(max_pts)))))
        scheme = ["horner", "estrin", "balanced"][int(g.integers(0, 3))]
        D = 0
        while math.comb(D + v, v) < T:
            D += 1
        if (v, D) not in mono:
            mono[(v, D)] = monomials_total_degree(v, D)
        allm = mono[(v, D)]
        ex = allm[np.sort(g.choice(len(allm), T, replace=False))]
        co = g.uniform(-1.0, 1.0, T)
        co[co == 0.0] = 0.5
        off = int(g.integers(0, pool_pts - N + 1))
        reqs.append(Request(t, scheme, MultiInput(ex, co, pool[:v, off:off + N])))
        offs.append(off)
    return PooledStream(reqs, pool, offs)
