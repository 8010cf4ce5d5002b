"""Serving loop on the GPU: continuous batching of uneven requests.

Each request's result must be bit-identical alone (fpe_evaluate) and in the
mix (fused served launches), and within the stated tolerance of the oracle."""
import numpy as np
import pytest
import torch

import fpe_inputs
import paper_1307_5655_amd as fpe
from oracle import exact

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def make_requests(nreq, seed, max_terms=3000, max_pts=50_000):
    g = np.random.default_rng([13075655, 500, seed])
    reqs = []
    for k in range(nreq):
        v = int(g.integers(1, 4))
        T = int(np.exp(g.uniform(np.log(10), np.log(max_terms))))
        N = int(np.exp(g.uniform(np.log(1000), np.log(max_pts))))
        scheme = ["horner", "estrin", "balanced"][int(g.integers(0, 3))]
        dom = [fpe.F32C, fpe.F64][k % 2]
        reqs.append((scheme, dom, fpe_inputs.random_multi_f64(v, T, N, g)))
    return reqs


def prepare(reqs, dev):
    out = []
    for scheme, dom, m in reqs:
        t = fpe.Tree(m.exps, m.coeffs, scheme, dom).upload(dev)
        pts = [torch.from_numpy(np.ascontiguousarray(m.points[j])).to(dev) for j in range(m.points.shape[0])]
        out.append((t, dom, pts, m))
    torch.cuda.synchronize()
    return out


def test_serve_alone_vs_mix_bit_identical(dev):
    say("serve: 40 uneven requests, alone vs in the mix")
    reqs = prepare(make_requests(40, 1), dev)
    alone = []
    for t, dom, pts, m in reqs:
        y = fpe.evaluate(t, pts)
        alone.append(y.cpu().numpy())
    srv = fpe.Server(hbm_budget=64 << 20, max_inflight=16)
    outs, tickets = [], []
    for t, dom, pts, m in reqs:
        o = torch.full((pts[0].numel(),), np.nan, dtype=torch.float64, device=dev)
        outs.append(o)
        tickets.append(srv.submit(t, pts, o, domain=dom))
    srv.drain()
    for tk in tickets:
        assert srv.poll(tk)
    for k, ((t, dom, pts, m), o) in enumerate(zip(reqs, outs)):
        y = o.cpu().numpy()
        assert np.array_equal(y, alone[k]), k
        # and within tolerance of the oracle on a sample
        idx = np.arange(0, len(y), max(1, len(y) // 200))
        ref = exact.dd_monomial_sum(m.exps, m.coeffs, m.points[:, idx])
        if dom == fpe.F32C:
            assert np.max(np.abs(y[idx] - ref) / np.abs(ref)) <= 1e-12, k
        else:
            pt = exact.monomial_ptilde(m.exps, m.coeffs, m.points[:, idx])
            assert np.max(np.abs(y[idx] - ref) / pt) <= 1e-13, k
    st = srv.stats()
    say(f"  batches {st.batches} p50 {st.p50_ms:.3f} ms p99 {st.p99_ms:.3f} ms fallback {st.fallback_frac:.3f}")
    assert st.completed == st.submitted == 40
    assert st.hbm_in_use == 0
    assert st.p99_ms >= st.p50_ms > 0
    srv.close()


def request_bytes(t, npts, dom, cond=False):
    """The bytes a served evaluate request counts against the budget (as the
    header states: points, output, condition output, fallback list, tree
    image)."""
    scratch = ((4 * npts + 255) // 256) * 256 if dom == fpe.F32C else 0
    return t.device_bytes() + scratch + npts * (8 * t.nvars + 8 + (4 if cond else 0))


def test_serve_tight_budget_admission_and_rejection(dev):
    say("serve: budget admission and rejection")
    reqs = prepare(make_requests(24, 2, max_terms=400, max_pts=20_000), dev)
    biggest = max(request_bytes(t, p[0].numel(), dom) for t, dom, p, _ in reqs)
    # the budget holds about one large request at a time
    srv = fpe.Server(hbm_budget=biggest, max_inflight=8)
    outs, tickets = [], []
    for t, dom, pts, m in reqs:
        o = torch.empty(pts[0].numel(), dtype=torch.float64, device=dev)
        outs.append(o)
        tickets.append(srv.submit(t, pts, o, domain=dom))
    for tk in tickets:
        srv.wait(tk)
    for (t, dom, pts, m), o in zip(reqs, outs):
        assert np.array_equal(o.cpu().numpy(), fpe.evaluate(t, pts).cpu().numpy())
    st = srv.stats()
    assert st.completed == len(reqs) and st.hbm_in_use == 0
    assert st.batches >= 4          # the budget split the stream into several batches
    # a request that can never fit is rejected with FPE_EBUDGET
    g = np.random.default_rng(3)
    n = biggest // 16 + 1
    m = fpe_inputs.random_multi_f64(1, 20, n, g)
    t = fpe.Tree(m.exps, m.coeffs, "horner", fpe.F32C).upload(dev)
    assert request_bytes(t, n, fpe.F32C) > biggest
    pts = [torch.from_numpy(m.points[0]).to(dev)]
    with pytest.raises(fpe.FpeError) as e:
        srv.submit(t, pts, torch.empty(n, dtype=torch.float64, device=dev), domain=fpe.F32C)
    assert e.value.status == -4
    assert srv.stats().rejected == 1
    # tickets: completed ones keep no state and report done; a ticket never
    # issued is an error
    assert all(srv.poll(tk) for tk in tickets)
    with pytest.raises(fpe.FpeError):
        srv.poll(max(tickets) + 1000)
    srv.close()


def test_serve_modp_and_compose_requests_in_the_mix(dev):
    """Exact requests join the batches: mod 2^61 - 1 evaluations and batched
    compositions mod 2^31 - 1, beside compensated and FP64 evaluations; each
    result is the same as the request alone."""
    say("serve: mod-p evaluate and compose requests in the mix")
    from oracle import native
    fl = prepare(make_requests(12, 7, max_terms=800, max_pts=30_000), dev)
    mods = []
    for k in range(4):
        v = 1 + k % 3
        m = fpe_inputs.random_modp_poly(v, 300 + 100 * k, {1: 700, 2: 40, 3: 18}[v], 5000 + 77 * k, seed=(910, k))
        t = fpe.Tree(m.exps, m.coeffs, ["horner", "estrin", "balanced"][k % 3], fpe.MODP, fpe.P61).upload(dev)
        px = [torch.from_numpy(np.ascontiguousarray(m.points[j]).view(np.int64)).to(dev)
              for j in range(m.points.shape[0])]
        mods.append((t, px, m))
    comps = []
    g = np.random.default_rng([13075655, 920])
    for k, (b, dp, dq) in enumerate([(64, 63, 7), (16, 255, 15), (33, 40, 3)]):
        P = g.integers(0, fpe.P31, size=(b, dp + 1)).astype(np.uint64)
        Q = g.integers(0, fpe.P31, size=(b, dq + 1)).astype(np.int32)
        t = fpe.Tree(np.arange(dp + 1, dtype=np.int32).reshape(-1, 1), P, ["balanced", "horner", "estrin"][k],
                     fpe.MODP, fpe.P31).upload(dev)
        comps.append((t, torch.from_numpy(Q).to(dev), P, Q))
    torch.cuda.synchronize()
    srv = fpe.Server(hbm_budget=512 << 20, max_inflight=32)
    outs = []
    for i in range(max(len(fl), len(mods), len(comps))):
        if i < len(fl):
            t, dom, pts, m = fl[i]
            o = torch.full((pts[0].numel(),), np.nan, dtype=torch.float64, device=dev)
            outs.append(("f", i, o, srv.submit(t, pts, o, domain=dom)))
        if i < len(mods):
            t, px, m = mods[i]
            o = torch.full((px[0].numel(),), -1, dtype=torch.int64, device=dev)
            outs.append(("m", i, o, srv.submit(t, px, o, domain=fpe.MODP)))
        if i < len(comps):
            t, q, P, Q = comps[i]
            o = torch.full((P.shape[0], (P.shape[1] - 1) * (Q.shape[1] - 1) + 1), -1, dtype=torch.int32, device=dev)
            outs.append(("c", i, o, srv.submit_compose(t, q, o)))
    srv.drain()
    for kind, i, o, tk in outs:
        assert srv.poll(tk)
        got = o.cpu().numpy()
        if kind == "f":
            t, dom, pts, m = fl[i]
            assert np.array_equal(got, fpe.evaluate(t, pts).cpu().numpy()), i
        elif kind == "m":
            t, px, m = mods[i]
            assert np.array_equal(got, fpe.evaluate(t, px).cpu().numpy()), i
            assert np.array_equal(got.view(np.uint64), native.modp_eval(m.exps, m.coeffs, fpe.P61, m.points)), i
        else:
            t, q, P, Q = comps[i]
            assert np.array_equal(got, fpe.compose(t, q).cpu().numpy()), i
            want = native.compose_modp(P.astype(np.uint32), Q.astype(np.uint32), fpe.P31)
            assert np.array_equal(got.view(np.uint32), want), i
    st = srv.stats()
    assert st.completed == st.submitted == len(outs)
    assert st.compose_instances == sum(P.shape[0] for _, _, P, _ in comps)
    assert st.hbm_in_use == 0
    srv.close()


def test_serve_term_path_requests(dev):
    """Few points on a big tree: FP64 and mod 2^61 - 1 requests on the
    term-parallel path (path "terms", and "auto" where the cost model picks
    it) join the batches beside fused walks; each result is the same bits as
    fpe_evaluate with that path (mod p also the oracle's); a path on a
    compensated request is refused."""
    say("serve: term-path requests in the mix")
    from oracle import native
    tri = fpe_inputs.trivariate(npts=64)
    g = np.random.default_rng([13075655, 930])
    tf = fpe.Tree(tri.exps, g.uniform(-1, 1, len(tri.exps)), "estrin", fpe.F64).upload(dev)
    tm = fpe.Tree(tri.exps, tri.coeffs, "balanced", fpe.MODP, fpe.P61).upload(dev)
    xf = [torch.from_numpy(g.uniform(-1, 1, 64)).to(dev) for _ in range(3)]
    xm = [torch.from_numpy(tri.points[j].copy().view(np.int64)).to(dev) for j in range(3)]
    fl = prepare(make_requests(6, 11, max_terms=800, max_pts=20_000), dev)
    torch.cuda.synchronize()
    srv = fpe.Server(hbm_budget=256 << 20, max_inflight=32)
    outs = []
    for i, (t, dom, pts, m) in enumerate(fl):
        o = torch.full((pts[0].numel(),), np.nan, dtype=torch.float64, device=dev)
        outs.append(("f", t, pts, "walk", o, srv.submit(t, pts, o, domain=dom)))
        n = (1, 16, 64)[i % 3]
        for path in ("terms", "auto"):
            assert fpe.eval_path(tf, n) == "terms" and fpe.eval_path(tm, n) == "terms"
            sub = [x[:n].contiguous() for x in xf]
            o = torch.full((n,), np.nan, dtype=torch.float64, device=dev)
            outs.append(("x", tf, sub, path, o, srv.submit(tf, sub, o, domain=fpe.F64, path=path)))
            subm = [x[:n].contiguous() for x in xm]
            om = torch.full((n,), -1, dtype=torch.int64, device=dev)
            outs.append(("m", tm, subm, path, om, srv.submit(tm, subm, om, domain=fpe.MODP, path=path)))
    srv.drain()
    for kind, t, pts, path, o, tk in outs:
        assert srv.poll(tk)
        got = o.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), fpe.evaluate(t, pts, path=path).cpu().numpy().view(np.uint64)) \
            if kind != "f" else np.array_equal(got, fpe.evaluate(t, pts).cpu().numpy()), (kind, path)
        if kind == "m":
            n = pts[0].numel()
            assert np.array_equal(got.view(np.uint64), native.modp_eval(tri.exps, tri.coeffs, fpe.P61,
                                                                        tri.points[:, :n].copy()))
    st = srv.stats()
    assert st.completed == st.submitted == len(outs) and st.hbm_in_use == 0
    t, dom, pts, m = fl[0]
    tc = fpe.Tree(m.exps, m.coeffs, "estrin", fpe.F32C).upload(dev)
    with pytest.raises(fpe.FpeError):
        srv.submit(tc, pts, torch.empty(pts[0].numel(), dtype=torch.float64, device=dev), domain=fpe.F32C,
                   path="terms")
    srv.close()


def test_serve_requests_arriving_during_a_batch(dev):
    say("serve: requests arriving while others run")
    reqs = prepare(make_requests(60, 4, max_terms=2000, max_pts=100_000), dev)
    srv = fpe.Server(hbm_budget=256 << 20, max_inflight=32)
    outs, tickets = [], []
    for k, (t, dom, pts, m) in enumerate(reqs):
        o = torch.empty(pts[0].numel(), dtype=torch.float64, device=dev)
        outs.append(o)
        tickets.append(srv.submit(t, pts, o, domain=dom))
        if k % 10 == 9:
            srv.wait(tickets[-1])     # some batches complete while others queue
    srv.drain()
    st = srv.stats()
    assert st.completed == 60 and st.batches >= 2
    for (t, dom, pts, m), o in zip(reqs, outs):
        assert np.array_equal(o.cpu().numpy(), fpe.evaluate(t, pts).cpu().numpy())
    srv.close()


def test_serve_tables_by_condition_output_and_table_size(dev):
    """Requests with and without condition numbers, FP64 requests and
    compensated trees whose powers do not fit the multi-point walks (the
    direct scheme: large tables, powers on the fly) are batched into separate
    work tables; every value and condition number matches the request alone."""
    say("serve: condition output, FP64, large tables")
    g = np.random.default_rng([13075655, 500, 9])
    reqs = []
    for k in range(24):
        v = 1 + k % 3
        m = fpe_inputs.random_multi_f64(v, int(g.integers(20, 600)), int(g.integers(1000, 20_000)), g)
        scheme = ["horner", "estrin", "balanced", "direct"][k % 4]
        dom = fpe.F64 if k % 6 == 5 else fpe.F32C
        want_cond = dom == fpe.F32C and k % 2 == 0
        reqs.append((scheme, dom, want_cond, m))
    prepared = []
    for scheme, dom, want_cond, m in reqs:
        t = fpe.Tree(m.exps, m.coeffs, scheme, dom).upload(dev)
        pts = [torch.from_numpy(np.ascontiguousarray(m.points[j])).to(dev) for j in range(m.points.shape[0])]
        prepared.append((t, dom, want_cond, pts, m))
    assert any(t.info.n_table > 32 or t.info.n_offtable > 0 for t, *_ in prepared)
    alone = []
    for t, dom, want_cond, pts, m in prepared:
        c = torch.empty(pts[0].numel(), dtype=torch.float32, device=dev) if want_cond else None
        y = fpe.evaluate(t, pts, cond_out=c)
        alone.append((y.cpu().numpy(), None if c is None else c.cpu().numpy()))
    srv = fpe.Server(hbm_budget=64 << 20, max_inflight=32)
    outs = []
    for t, dom, want_cond, pts, m in prepared:
        o = torch.full((pts[0].numel(),), np.nan, dtype=torch.float64, device=dev)
        c = torch.full((pts[0].numel(),), np.nan, dtype=torch.float32, device=dev) if want_cond else None
        outs.append((o, c))
        srv.submit(t, pts, o, domain=dom, cond_out=c)
    srv.drain()
    for k, ((o, c), (ya, ca)) in enumerate(zip(outs, alone)):
        assert np.array_equal(o.cpu().numpy(), ya), k
        if c is not None:
            assert np.array_equal(c.cpu().numpy(), ca), k
    st = srv.stats()
    assert st.completed == st.submitted == len(prepared)
    srv.close()
