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


def test_serve_tight_budget_admission_and_rejection(dev):
    say("serve: budget admission and rejection")
    reqs = prepare(make_requests(24, 2, max_terms=400, max_pts=20_000), dev)
    biggest = max(p[0].numel() for _, _, p, _ in reqs)
    # the budget holds the fallback list of about one large request at a time
    srv = fpe.Server(hbm_budget=(biggest * 4 + 256) * 1, max_inflight=8)
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
    # a request whose workspace can never fit is rejected with FPE_EBUDGET
    g = np.random.default_rng(3)
    m = fpe_inputs.random_multi_f64(1, 20, biggest * 2, g)
    t = fpe.Tree(m.exps, m.coeffs, "horner", fpe.F32C).upload(dev)
    pts = [torch.from_numpy(m.points[0]).to(dev)]
    with pytest.raises(fpe.FpeError) as e:
        srv.submit(t, pts, torch.empty(biggest * 2, dtype=torch.float64, device=dev), domain=fpe.F32C)
    assert e.value.status == -4
    assert srv.stats().rejected == 1
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
