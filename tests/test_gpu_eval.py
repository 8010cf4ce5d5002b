"""GPU parity: the HIP walk (through the C-ABI) against the CPU oracle.

Floating point: plain FP64 within 1e-13 of the oracle scaled by the condition
sum ptilde(|x|) = sum |c_m| |x|^m (the relative error divided by the
condition number); compensated FP32 (with the FP64 fallback) within 1e-12
relative error at every point.  Mod 2^61 - 1: bit-exact."""
import numpy as np
import pytest
import torch

import fpe_inputs
import paper_1307_5655_amd as fpe
from oracle import exact, native

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-13
TOL_F32C = 1e-12


def say(msg):
    print(msg, flush=True)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def eval_uni(coeffs, x, scheme, domain, dev, **kw):
    e = np.nonzero(coeffs)[0].astype(np.int32).reshape(-1, 1)
    t = fpe.Tree(e, coeffs[e[:, 0]], scheme, domain).upload(dev)
    y = fpe.evaluate(t, [to_dev(x, dev)], **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy(), t


def check_f64(y, coeffs, x):
    ref = native.dd_value(coeffs, x)
    pt = native.ptilde(coeffs, x)
    err = np.abs(y - ref) / pt
    assert np.all(np.isfinite(y))
    assert err.max() <= TOL_F64, f"max scaled error {err.max():.3e}"
    return err


def check_f32c(y, coeffs, x):
    ref = native.dd_value(coeffs, x)
    rel = np.abs(y - ref) / np.abs(ref)
    bad = ~(rel <= TOL_F32C)
    assert not bad.any(), f"{bad.sum()} points above 1e-12, worst {np.nanmax(rel):.3e} at x={x[bad][:4]}"
    return rel


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced", "direct"])
def test_dense_1023_f64(dev, scheme):
    say(f"dense n=1023 f64 {scheme}")
    inp = fpe_inputs.dense_uni(npts=20_000 + 37)       # ragged tail
    y, _ = eval_uni(inp.coeffs, inp.points, scheme, fpe.F64, dev)
    check_f64(y, inp.coeffs, inp.points)


@pytest.mark.parametrize("log2n,depth", [(15, 8), (17, 9)])
def test_deep_estrin_walks(dev, log2n, depth):
    """Walks of depth 8 (the deepest the depth-8 kernels take, every level
    used) and 9 (the deep kernels), in all three domains."""
    n = 1 << log2n
    say(f"estrin n=2^{log2n} walk depth {depth}")
    inp = fpe_inputs.dense_uni(npts=4096 + 37, degree=n - 1, seed_k=1)
    y, t = eval_uni(inp.coeffs, inp.points, "estrin", fpe.F64, dev)
    assert t.info.walk_depth == depth
    check_f64(y, inp.coeffs, inp.points)
    y, t = eval_uni(inp.coeffs, inp.points, "estrin", fpe.F32C, dev)
    check_f32c(y, inp.coeffs, inp.points)
    m = fpe_inputs.random_modp_poly(1, n, n - 1, 1000 + 37, seed=(600 + log2n,))
    t = fpe.Tree(m.exps, m.coeffs, "estrin", fpe.MODP, fpe.P61).upload(dev)
    assert t.info.walk_depth == depth
    got = fpe.evaluate(t, [to_dev(m.points[0].view(np.int64), dev)]).cpu().numpy().view(np.uint64)
    want = native.modp_eval(m.exps, m.coeffs, fpe.P61, m.points)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_points_per_lane_requests_give_the_same_bits(dev, scheme):
    """Whatever width is requested, the launcher runs a kernel at most that
    wide with a grid sized for it: every point is written, with the same bits."""
    say(f"points per lane 1..16 {scheme}")
    inp = fpe_inputs.sparse_uni(3000, npts=10_000 + 77, lo=-0.99, hi=0.99)
    e = np.nonzero(inp.coeffs)[0].astype(np.int32).reshape(-1, 1)
    x = to_dev(inp.points, dev)
    for dom in (fpe.F64, fpe.F32C):
        t = fpe.Tree(e, inp.coeffs[e[:, 0]], scheme, dom).upload(dev)
        ref = fpe.evaluate(t, [x]).cpu().numpy()
        for ppl in (1, 2, 3, 4, 8, 16):
            out = torch.full((len(inp.points),), float("nan"), dtype=torch.float64, device=dev)
            fpe.evaluate(t, [x], out=out, points_per_lane=ppl)
            y = out.cpu().numpy()
            assert np.array_equal(y.view(np.uint64), ref.view(np.uint64)), (dom, ppl)
    m = fpe_inputs.random_modp_poly(2, 400, 30, 5000 + 9, seed=(77,))
    t = fpe.Tree(m.exps, m.coeffs, scheme, fpe.MODP, fpe.P61).upload(dev)
    px = [to_dev(m.points[j].view(np.int64), dev) for j in range(2)]
    ref = fpe.evaluate(t, px).cpu().numpy()
    for ppl in (1, 2, 4, 8):
        out = torch.full((m.points.shape[1],), -1, dtype=torch.int64, device=dev)
        fpe.evaluate(t, px, out=out, points_per_lane=ppl)
        assert np.array_equal(out.cpu().numpy(), ref), ppl


@pytest.mark.parametrize("which", ["threshold", "table"])
def test_threshold_and_table_schemes(dev, which):
    """User schemes (Section 1.2: Estrin above a threshold degree and Hörner
    below; an arbitrary legal table f(n) in [1, n]) on every domain."""
    say(f"scheme {which}")
    inp = fpe_inputs.sparse_uni(1500, npts=6000 + 13, lo=-1.0, hi=1.0)
    e = np.nonzero(inp.coeffs)[0].astype(np.int32).reshape(-1, 1)
    c = inp.coeffs[e[:, 0]]
    if which == "threshold":
        kw = dict(threshold=24)
    else:
        g = np.random.default_rng([13075655, 700])
        kw = dict(table=[0] + [int(g.integers(1, n + 1)) for n in range(1, 1502)])
    x = to_dev(inp.points, dev)
    t = fpe.Tree(e, c, which, fpe.F64, **kw).upload(dev)
    check_f64(fpe.evaluate(t, [x]).cpu().numpy(), inp.coeffs, inp.points)
    t = fpe.Tree(e, c, which, fpe.F32C, **kw).upload(dev)
    check_f32c(fpe.evaluate(t, [x]).cpu().numpy(), inp.coeffs, inp.points)
    m = fpe_inputs.random_modp_poly(1, 1501, 1500, 2000 + 3, seed=(701,))
    t = fpe.Tree(m.exps, m.coeffs, which, fpe.MODP, fpe.P61, **kw).upload(dev)
    got = fpe.evaluate(t, [to_dev(m.points[0].view(np.int64), dev)]).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, native.modp_eval(m.exps, m.coeffs, fpe.P61, m.points))


def test_dense_horner_bit_identical_to_fma_horner(dev):
    say("dense n=1023 horner bit-exact")
    inp = fpe_inputs.dense_uni(npts=5000)
    y, _ = eval_uni(inp.coeffs, inp.points, "horner", fpe.F64, dev)
    want = native.horner_f64(inp.coeffs, inp.points, use_fma=True)
    assert np.array_equal(y, want)


@pytest.mark.parametrize("n", [3000, 5000])
@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_sparse_f64(dev, n, scheme):
    say(f"sparse n={n} f64 {scheme}")
    inp = fpe_inputs.sparse_uni(n, npts=8_000 + 13)
    y, _ = eval_uni(inp.coeffs, inp.points, scheme, fpe.F64, dev)
    check_f64(y, inp.coeffs, inp.points)


@pytest.mark.parametrize("n", [3000, 5000])
@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_sparse_f32c(dev, n, scheme):
    say(f"sparse n={n} f32c {scheme}")
    inp = fpe_inputs.sparse_uni(n, npts=8_000 + 13)
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)
    cond = torch.empty(len(inp.points), dtype=torch.float32, device=dev)
    y, _ = eval_uni(inp.coeffs, inp.points, scheme, fpe.F32C, dev, nfallback_out=nfb, cond_out=cond)
    check_f32c(y, inp.coeffs, inp.points)
    frac = nfb.item() / len(inp.points)
    say(f"  fallback fraction {frac:.4f}")
    # points beyond the FP32 range of x^n must have been re-evaluated
    assert frac >= np.mean(np.abs(inp.points) > 1.04) - 1e-9


def test_f32c_forced_modes(dev):
    say("f32c forced fallback / none")
    inp = fpe_inputs.sparse_uni(3000, npts=3000, lo=-0.99, hi=0.99)
    y_all, _ = eval_uni(inp.coeffs, inp.points, "balanced", fpe.F32C, dev, force=1)
    check_f32c(y_all, inp.coeffs, inp.points)
    y_none, _ = eval_uni(inp.coeffs, inp.points, "balanced", fpe.F32C, dev, force=2)
    ref = native.dd_value(inp.coeffs, inp.points)
    pt = native.ptilde(inp.coeffs, inp.points)
    # without any fallback the double-float walk is still accurate to ~1e-13 ptilde
    assert np.max(np.abs(y_none - ref) / pt) < 1e-12


def test_f32c_cond_and_flags(dev):
    say("f32c cond + flags")
    inp = fpe_inputs.sparse_uni(1000, npts=4096 + 5)
    n = len(inp.points)
    cond = torch.empty(n, dtype=torch.float32, device=dev)
    flags = torch.zeros((n + 31) // 32 + 2, dtype=torch.int32, device=dev)
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)
    y, _ = eval_uni(inp.coeffs, inp.points, "estrin", fpe.F32C, dev, cond_out=cond, flags_out=flags,
                    nfallback_out=nfb)
    ref = native.dd_value(inp.coeffs, inp.points)
    pt = native.ptilde(inp.coeffs, inp.points)
    c = cond.cpu().numpy()
    want = pt / np.abs(ref)
    ok = np.isfinite(c) & (want < 1e6)
    assert np.allclose(c[ok], want[ok], rtol=1e-3)
    bits = np.unpackbits(flags.cpu().numpy().view(np.uint8), bitorder="little")[:n]
    assert bits.sum() == nfb.item()


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_f32c_same_results_with_and_without_cond(dev, scheme):
    """The kernel without condition output drops the condition sums; its
    results and fallback decisions must be the same bits."""
    say(f"f32c with/without cond {scheme}")
    inp = fpe_inputs.sparse_uni(3000, npts=20_000 + 11)
    n = len(inp.points)
    cond = torch.empty(n, dtype=torch.float32, device=dev)
    f1 = torch.zeros((n + 31) // 32 + 2, dtype=torch.int32, device=dev)
    f2 = torch.zeros_like(f1)
    y1, _ = eval_uni(inp.coeffs, inp.points, scheme, fpe.F32C, dev, cond_out=cond, flags_out=f1)
    y2, _ = eval_uni(inp.coeffs, inp.points, scheme, fpe.F32C, dev, flags_out=f2)
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))
    assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy())
    check_f32c(y2, inp.coeffs, inp.points)


def test_edge_cases_f64(dev):
    say("edge cases")
    # single term, constant, zero constant term (root with a power), x = 0, +-1
    x = np.array([0.0, 1.0, -1.0, 0.5, -2.0, 1e-3], dtype=np.float64)
    cases = [
        ({7: 3.0}, None),
        ({0: -2.5}, None),
        ({3: 1.0, 5: -2.0, 9: 0.25}, None),
        ({0: 1.0, 1: 1.0}, None),
    ]
    for d, _ in cases:
        e = np.array(sorted(d), dtype=np.int32).reshape(-1, 1)
        c = np.array([d[k] for k in sorted(d)])
        dense = np.zeros(max(d) + 1)
        for k, v in d.items():
            dense[k] = v
        for scheme in ["horner", "estrin", "balanced", "direct"]:
            for dom in (fpe.F64, fpe.F32C):
                t = fpe.Tree(e, c, scheme, dom).upload(dev)
                y = fpe.evaluate(t, [to_dev(x, dev)]).cpu().numpy()
                ye = np.array([float(exact.exact_value([((k,), v) for k, v in d.items()], [xi])) for xi in x])
                assert np.allclose(y, ye, rtol=1e-14, atol=0), (d, scheme, dom, y, ye)
    # empty input
    t = fpe.Tree(np.array([[1]], dtype=np.int32), [1.0], "horner").upload(dev)
    out = torch.empty(0, dtype=torch.float64, device=dev)
    fpe.evaluate(t, [torch.empty(0, dtype=torch.float64, device=dev)], out=out)
    torch.cuda.synchronize()


def test_multivariate_f64_and_f32c(dev):
    say("multivariate f64 / f32c with junctions")
    g = np.random.default_rng([13075655, 77])
    for v, T in [(2, 300), (3, 1500), (4, 400)]:
        m = fpe_inputs.random_multi_f64(v, T, 3000 + 7, g)
        for scheme in ["horner", "estrin", "balanced"]:
            ref = exact.dd_monomial_sum(m.exps, m.coeffs, m.points)
            pt = exact.monomial_ptilde(m.exps, m.coeffs, m.points)
            for dom in (fpe.F64, fpe.F32C):
                t = fpe.Tree(m.exps, m.coeffs, scheme, dom).upload(dev)
                y = fpe.evaluate(t, [to_dev(m.points[j], dev) for j in range(v)]).cpu().numpy()
                if dom == fpe.F64:
                    err = np.abs(y - ref) / pt
                    assert err.max() <= TOL_F64, (v, scheme, err.max())
                else:
                    rel = np.abs(y - ref) / np.abs(ref)
                    assert rel.max() <= TOL_F32C, (v, scheme, rel.max())


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_trivariate_modp_bit_exact(dev, scheme):
    say(f"trivariate mod p {scheme}")
    inp = fpe_inputs.trivariate(npts=2000 + 3)
    t = fpe.Tree(inp.exps, inp.coeffs, scheme, fpe.MODP, fpe.P61).upload(dev)
    pts = [to_dev(inp.points[j].view(np.int64), dev) for j in range(3)]
    y = fpe.evaluate(t, pts).cpu().numpy().view(np.uint64)
    want = native.modp_eval(inp.exps, inp.coeffs, fpe.P61, inp.points)
    assert np.array_equal(y, want)


def test_sparse_multivariate_modp_bit_exact(dev):
    say("sparse multivariate mod p with junctions")
    for v, T, D in [(2, 200, 30), (3, 800, 25), (4, 300, 12)]:
        m = fpe_inputs.random_modp_poly(v, T, D, 1000 + 1, seed=(v,))
        for scheme in ["horner", "estrin", "balanced", "direct"]:
            t = fpe.Tree(m.exps, m.coeffs, scheme, fpe.MODP, fpe.P61).upload(dev)
            y = fpe.evaluate(t, [to_dev(m.points[j].view(np.int64), dev) for j in range(v)])
            y = y.cpu().numpy().view(np.uint64)
            want = native.modp_eval(m.exps, m.coeffs, fpe.P61, m.points)
            assert np.array_equal(y, want), (v, scheme)


# ----------------------------------------------------------------------------
# full sizes, in the launch configuration the benchmark times, sampled
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n", [3000, 5000])
def test_full_size_sparse_sampled(dev, n):
    say(f"full size sparse n={n}, 1e7 points, sampled")
    inp = fpe_inputs.sparse_uni(n)
    x = to_dev(inp.points, dev)
    rng = np.random.default_rng(n)
    idx = np.sort(rng.choice(len(inp.points), 3000, replace=False))
    idx[-1] = len(inp.points) - 1
    e, c = inp.terms()
    for scheme in ["horner", "estrin", "balanced"]:
        for dom in (fpe.F64, fpe.F32C):
            say(f"  {scheme} {dom}")
            t = fpe.Tree(e, c, scheme, dom).upload(dev)
            y = fpe.evaluate(t, [x])
            torch.cuda.synchronize()
            ys = y.cpu().numpy()[idx]
            if dom == fpe.F64:
                check_f64(ys, inp.coeffs, inp.points[idx])
            else:
                check_f32c(ys, inp.coeffs, inp.points[idx])
            del y


def test_full_size_trivariate_sampled(dev):
    say("full size trivariate mod p, 1e6 points, sampled")
    inp = fpe_inputs.trivariate()
    pts = [to_dev(inp.points[j].view(np.int64), dev) for j in range(3)]
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(inp.points.shape[1], 500, replace=False))
    want = native.modp_eval(inp.exps, inp.coeffs, fpe.P61, np.ascontiguousarray(inp.points[:, idx]))
    for scheme in ["horner", "estrin", "balanced"]:
        t = fpe.Tree(inp.exps, inp.coeffs, scheme, fpe.MODP, fpe.P61).upload(dev)
        y = fpe.evaluate(t, pts).cpu().numpy().view(np.uint64)
        assert np.array_equal(y[idx], want), scheme


# ----------------------------------------------------------------------------
# few points, big trees: the term-parallel path (DPP wavefront sums)
# ----------------------------------------------------------------------------

def test_term_path_few_points_big_trees(dev):
    """One workgroup per point, terms over the lanes, wavefront reductions:
    the trivariate degree-40 tree (12,341 terms) mod 2^61 - 1 bit-exact at 1,
    7, 64 and 301 points (every scheme, the walk the same bits); FP64
    multivariate trees with junctions within 1e-13 of p~ against the oracle;
    univariate degree-5000 and degree-9000 trees (the point's power table in
    LDS, and too large for it); mod 2^61 - 1 at the table's limit (8,000
    entries: degree 7,999 with the table, 8,000 without); four points per
    workgroup from 2,048 points, the same bits as one; the cost model
    picks the terms for few points and the walk for many; path 2 refused for
    the compensated form."""
    say("term path: trivariate mod p, multivariate f64")
    inp = fpe_inputs.trivariate(npts=301)
    for npts in (1, 7, 64, 301):
        pts = [to_dev(inp.points[j, :npts].copy().view(np.int64), dev) for j in range(3)]
        want = native.modp_eval(inp.exps, inp.coeffs, fpe.P61, inp.points[:, :npts].copy())
        for scheme in ("horner", "estrin", "balanced"):
            t = fpe.Tree(inp.exps, inp.coeffs, scheme, fpe.MODP, fpe.P61).upload(dev)
            for path in ("terms", "walk", "auto"):
                y = fpe.evaluate(t, pts, path=path).cpu().numpy().view(np.uint64)
                assert np.array_equal(y, want), (npts, scheme, path)
    g = np.random.default_rng([13075655, 950])
    for v, T, npts in [(3, 4000, 5), (2, 2000, 33), (4, 1500, 2)]:
        m = fpe_inputs.random_multi_f64(v, T, npts, g)
        ref = exact.dd_monomial_sum(m.exps, m.coeffs, m.points)
        pt = exact.monomial_ptilde(m.exps, m.coeffs, m.points)
        for scheme in ("horner", "balanced"):
            t = fpe.Tree(m.exps, m.coeffs, scheme, fpe.F64).upload(dev)
            y = fpe.evaluate(t, [to_dev(m.points[j], dev) for j in range(v)], path="terms").cpu().numpy()
            assert (np.abs(y - ref) / pt).max() <= TOL_F64, (v, scheme)
    for n in (9000, 5000):
        inp = fpe_inputs.sparse_uni(n, npts=3, lo=-1.05, hi=1.05)
        e = np.nonzero(inp.coeffs)[0].astype(np.int32).reshape(-1, 1)
        t = fpe.Tree(e, inp.coeffs[e[:, 0]], "estrin", fpe.F64).upload(dev)
        y = fpe.evaluate(t, [to_dev(inp.points, dev)], path="terms").cpu().numpy()
        check_f64(y, inp.coeffs, inp.points)
    g2 = np.random.default_rng([13075655, 951])
    for dmax in (7999, 8000):
        ex = np.unique(np.concatenate([g2.integers(0, dmax, 400), [dmax]])).astype(np.int32).reshape(-1, 1)
        co = g2.integers(0, int(fpe.P61), len(ex), dtype=np.uint64)
        x = g2.integers(0, int(fpe.P61), (1, 5), dtype=np.uint64)
        want = native.modp_eval(ex, co, fpe.P61, x)
        tm = fpe.Tree(ex, co, "balanced", fpe.MODP, fpe.P61).upload(dev)
        y = fpe.evaluate(tm, [to_dev(x[0].copy().view(np.int64), dev)], path="terms").cpu().numpy().view(np.uint64)
        assert np.array_equal(y, want), dmax
    # from 2,048 points a workgroup takes four (ragged tail of three): mod p
    # bit-exact, FP64 the same bits as one point per workgroup and within
    # tolerance of the oracle
    say("term path: four points per workgroup")
    inp = fpe_inputs.trivariate(npts=2051)
    want = native.modp_eval(inp.exps, inp.coeffs, fpe.P61, inp.points.copy())
    t = fpe.Tree(inp.exps, inp.coeffs, "estrin", fpe.MODP, fpe.P61).upload(dev)
    y = fpe.evaluate(t, [to_dev(inp.points[j].copy().view(np.int64), dev) for j in range(3)],
                     path="terms").cpu().numpy().view(np.uint64)
    assert np.array_equal(y, want)
    m = fpe_inputs.random_multi_f64(3, 3000, 2051, np.random.default_rng([13075655, 952]))
    t = fpe.Tree(m.exps, m.coeffs, "balanced", fpe.F64).upload(dev)
    xs = [to_dev(m.points[j], dev) for j in range(3)]
    y4 = fpe.evaluate(t, xs, path="terms").cpu().numpy()
    y1 = fpe.evaluate(t, [x[:301].contiguous() for x in xs], path="terms").cpu().numpy()
    assert np.array_equal(y4[:301].view(np.uint64), y1.view(np.uint64))
    ref = exact.dd_monomial_sum(m.exps, m.coeffs, m.points)
    pt = exact.monomial_ptilde(m.exps, m.coeffs, m.points)
    assert (np.abs(y4 - ref) / pt).max() <= TOL_F64
    # the library's choice: terms for 16 points, the walk for 1e6
    tri = fpe_inputs.trivariate(npts=1)
    t3 = fpe.Tree(tri.exps, np.ones(len(tri.exps)), "estrin", fpe.F64)
    assert fpe.eval_path(t3, 16) == "terms" and fpe.eval_path(t3, 1_000_000) == "walk"
    tf = fpe.Tree(e, inp.coeffs[e[:, 0]], "estrin", fpe.F32C).upload(dev)
    with pytest.raises(fpe.FpeError):
        fpe.evaluate(tf, [to_dev(inp.points, dev)], path="terms")
