"""Benchmark of the evaluation-tree hot path on one MI355X.

Timed step: the sparse univariate workload of degrees 3000 and 5000
(coefficients U[-1, 1], 10 % of the exponents below the degree zeroed),
1e7 points U[-1.05, 1.05] resident in HBM, each degree under the balanced,
Estrin and Hörner schemes, each in the served form (compensated FP32 with a
running error bound and FP64 re-evaluation of flagged points) and in plain
FP64: 12 evaluations, 8.1e11 term-evaluations per step.  Trees are compiled
and uploaded once, before the timed region.

After the timed region (not part of ``value``): the accuracy of the last step
against the CPU oracle on a sample; a served stream (Poisson arrivals of
uneven evaluate requests through the continuous-batching server: 10^4
requests, first all at once for the saturation rate, then at 0.5, 0.8 and 0.95
times that rate) for p50/p99 latency; the exact mod 2^61-1 trivariate workload and the batched
composition mod 2^31-1, each timed beside the main line; and the CPU oracle
timed on a bounded sample of the step's workload.

Prints one JSON line; ``roofline`` describes the dominant kernel (the
compensated-FP32 walk), ``roofline_f64`` the plain FP64 walk.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts.  FP32 vector 157.3 TFLOP/s counts
# an FMA as two flops: 256 CU x 128 FP32 lanes x 2.4 GHz = 78.6e12 FP32 VALU
# lane-instructions/s.  FP64 vector 78.6 TFLOP/s = 39.3e12 FP64 FMA/s.
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK = 256 * 128 * 2.4e9
FP64_FMA_PEAK = 256 * 64 * 2.4e9
# FP32 operations of one compensated multiply-add a * X + b (X read as two
# floats): product and its error by fma (2), two cross terms (2), TwoSum (6),
# two low-order adds (2), FastTwoSum (3), then the running error bound:
# e_a |X| + e_b (1 fma, when the product's operand is an accumulator),
# 20 u^2 |p| (1 fma) and 6 u^2 |b| (1 fma when b is an accumulator; a
# coefficient's term is a constant of the op).  Per step kind: LEAF_ADD
# a X + top 17, NODE_OPEN top X + b 17, LEAF_OPEN a X + b 16, NODE_ADD
# top X + below 18; END (once per point) is not counted.  The condition sum (1 more fma) is computed only when per-point
# condition numbers are requested, which the timed step does not do (the
# condition numbers of the workload are reported from the oracle's sample
# instead).
DF32_OPS_BY_KIND = (17, 17, 16, 18, 0)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class HipEvents:
    """Raw hipEvent_t handles (the library records them on the launch stream)."""

    def __init__(self):
        import ctypes
        self.ct = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        e = self.ct.c_void_p()
        if self.hip.hipEventCreate(self.ct.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e

    def elapsed_ms(self, a, b) -> float:
        ms = self.ct.c_float()
        if self.hip.hipEventElapsedTime(self.ct.byref(ms), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)


# The HBM traffic of the compensated walk comes from two profiler passes
# (FETCH_SIZE, WRITE_SIZE) over this benchmark, scaled by what the same
# counters read for a plain copy of known size; the summary records a hash of
# the kernel sources it was taken with, and the figure is reported only while
# the sources are unchanged.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_eval_df32_sparse_uni_1e7_traffic.md")
KERNEL_SOURCES = ("walk_core.h", "eval_df32.hip", "fpe_internal.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1307_5655_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel source hash") != kernel_source_hash():
        return None
    try:
        return float(vals["HBM bytes per launch (scaled)"])
    except (KeyError, ValueError):
        return None


def served_phase(fpe, fpe_inputs, torch, dev, nreq: int, loads=(0.5, 0.8, 0.95)):
    """Poisson arrivals of uneven evaluate requests (compensated FP32 with FP64
    fallback) through the server: first all at once to find the saturation
    request rate, then arrivals at each of ``loads`` times that rate for
    latency.  The points of every request are a window of one resident pool."""
    stream = fpe_inputs.served_stream_pooled(nreq, rate_per_s=1.0)   # unit-rate arrival times, rescaled below
    pool = torch.from_numpy(stream.pool).to(dev)
    prepared = []
    for r, off in zip(stream.requests, stream.offsets):
        m = r.poly
        v, n = m.points.shape
        t = fpe.Tree(m.exps, m.coeffs, r.scheme, fpe.F32C).upload(dev)
        pts = [pool[j, off:off + n] for j in range(v)]
        out = torch.empty(n, dtype=torch.float64, device=dev)
        prepared.append((r.arrival_s, t, pts, out, m))
    torch.cuda.synchronize()
    budget = 8 << 30
    # FP32 operations of the compensated walks of one pass over the stream
    step_ops = float(sum(sum(k * o for k, o in zip(t.info.n_ops_kind, DF32_OPS_BY_KIND)) * m.points.shape[1]
                         for _, t, _, _, m in prepared))
    # each request's ideal time on the roofline: the larger of its compensated
    # walk's FP32 operations at the VALU peak and its point and result bytes
    # (8 v + 8 per point) at the HBM peak
    ideal_s = float(sum(max(sum(k * o for k, o in zip(t.info.n_ops_kind, DF32_OPS_BY_KIND)) * m.points.shape[1]
                            / FP32_VALU_PEAK,
                            (8 * m.points.shape[0] + 8) * m.points.shape[1] / (HBM_PEAK_GBS * 1e9))
                        for _, t, _, _, m in prepared))

    srv = fpe.Server(hbm_budget=budget, max_inflight=64)
    t0 = time.perf_counter()
    for _, t, pts, out, _ in prepared:
        srv.submit(t, pts, out, domain=fpe.F32C)
    srv.drain()
    wall_sat = time.perf_counter() - t0
    st = srv.stats()
    sat = {"requests": nreq, "wall_s": wall_sat, "term_evals": st.term_evals,
           "term_evals_per_s": st.term_evals / wall_sat, "batches": st.batches,
           "fallback_frac": st.fallback_frac, "df32_step_ops": step_ops,
           "fp32_peak_frac_of_wall": step_ops / (wall_sat * FP32_VALU_PEAK),
           "ideal_s": ideal_s, "roofline_frac_of_wall": ideal_s / wall_sat}
    srv.close()
    sat_rps = nreq / wall_sat

    by_load = []
    for load in loads:
        rate = load * sat_rps
        scale = 1.0 / rate
        srv = fpe.Server(hbm_budget=budget, max_inflight=64)
        t0 = time.perf_counter()
        for at, t, pts, out, _ in prepared:
            target = t0 + at * scale
            while True:
                now = time.perf_counter()
                if now >= target:
                    break
                if target - now > 2e-4:
                    time.sleep((target - now) * 0.5)
            srv.submit(t, pts, out, domain=fpe.F32C)
        srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        by_load.append({"load": load, "rate_rps": rate, "requests": nreq, "p50_ms": st.p50_ms,
                        "p99_ms": st.p99_ms, "mean_ms": st.mean_ms, "batches": st.batches,
                        "term_evals_per_s": st.term_evals / wall, "fallback_frac": st.fallback_frac})
        srv.close()
        log(f"served load {load}: p50 {st.p50_ms:.2f} ms, p99 {st.p99_ms:.2f} ms")

    # served results against the oracle on a sample of requests and points
    from oracle import exact
    worst = 0.0
    for _, _, _, out, m in prepared[:: max(1, nreq // 24)]:
        y = out.cpu().numpy()
        idx = np.arange(0, len(y), max(1, len(y) // 64))
        ref = exact.dd_monomial_sum(m.exps, m.coeffs, m.points[:, idx])
        worst = max(worst, float(np.max(np.abs(y[idx] - ref) / np.abs(ref))))
    head = next(d for d in by_load if d["load"] == 0.8) if 0.8 in loads else by_load[-1]
    lat = dict(head)
    lat["max_rel_err_sampled"] = worst
    lat["other_loads"] = [d for d in by_load if d is not head]
    return sat, lat


def modp_phase(fpe, fpe_inputs, torch, dev, hev, reps: int = 3):
    """Exact trivariate evaluation mod 2^61-1 (12,341 terms, 1e6 points)."""
    inp = fpe_inputs.trivariate()
    pts = [torch.from_numpy(np.ascontiguousarray(inp.points[j])).to(dev) for j in range(3)]
    res = {}
    for s in ("balanced", "estrin", "horner"):
        t = fpe.Tree(inp.exps, inp.coeffs, s, fpe.MODP, fpe.P61).upload(dev)
        out = torch.empty(inp.points.shape[1], dtype=torch.int64, device=dev)
        fpe.evaluate(t, pts, out=out)
        ms = []
        for _ in range(reps):
            e0, e1 = hev.create(), hev.create()
            fpe.evaluate(t, pts, out=out, events=(e0, e1))
            torch.cuda.synchronize()
            ms.append(hev.elapsed_ms(e0, e1))
        m = float(np.median(ms))
        res[s] = {"walk_ms": m, "term_evals_per_s": len(inp.coeffs) * inp.points.shape[1] / (m * 1e-3)}
    return res


# FP64 operations of one interval step (bounds rounded outward: one fma or
# product, then two operations per bound to move it out): LEAF_ADD a X + top
# and LEAF_OPEN a X + b take 2 fma + 4; NODE_OPEN top X + b takes 4 end
# products fused with b, 3 min, 3 max and 4; NODE_ADD top X + below 8 fused
# end products, 6 min / max and 4.
IVAL_OPS_BY_KIND = (6, 14, 6, 18, 0)


def interval_phase(fpe, fpe_inputs, torch, dev, hev, npts: int, reps: int = 3):
    """Interval enclosures over boxes around the sparse univariate points
    (degrees 3000 and 5000, widths {0, 2^-20, 2^-8, 0.25})."""
    res = {}
    ops = secs = 0.0
    for n in (3000, 5000):
        inp = fpe_inputs.sparse_uni(n, npts=npts)
        e, c = inp.terms()
        box = torch.from_numpy(fpe_inputs.interval_boxes(inp.points, fpe_inputs.rng_for(6, n))).to(dev)
        out = torch.empty((npts, 2), dtype=torch.float64, device=dev)
        for s in ("balanced", "estrin", "horner"):
            t = fpe.Tree(e, c, s, fpe.IVAL).upload(dev)
            fpe.evaluate(t, [box], out=out)
            ms = []
            for _ in range(reps):
                e0, e1 = hev.create(), hev.create()
                fpe.evaluate(t, [box], out=out, events=(e0, e1))
                torch.cuda.synchronize()
                ms.append(hev.elapsed_ms(e0, e1))
            m = float(np.median(ms))
            k_ops = float(sum(k * o for k, o in zip(t.info.n_ops_kind, IVAL_OPS_BY_KIND))) * npts
            ops += k_ops
            secs += m * 1e-3
            res[f"n{n}_{s}"] = {"walk_ms": m, "term_evals_per_s": float(t.info.n_terms) * npts / (m * 1e-3)}
        del box, out
    res["roofline"] = {"kernel": "k_eval_iv (interval walk)", "bound": "alu",
                       "achieved": ops / secs / 1e12, "peak": FP64_FMA_PEAK / 1e12,
                       "unit": "T FP64 VALU lane-ops/s", "frac": ops / secs / FP64_FMA_PEAK}
    return res


def bigint_phase(fpe, torch, dev, reps: int = 3):
    """Exact evaluation over the natural numbers (the workload of the paper's
    Benchmarks section): 64-bit coefficients, 256 points of 256 bits, dense
    polynomials with term counts around powers of two; time per scheme and
    the ratio to the balanced scheme (the form of the paper's Figure 1)."""
    g = np.random.default_rng([13075655, 8])
    lx, batch = 16, 256
    x = torch.from_numpy(g.integers(0, 1 << 16, size=(batch, lx), dtype=np.int64).astype(np.int32)).to(dev)
    res = {}
    for n in (127, 128, 129, 255, 256, 257):
        ex = np.arange(n + 1, dtype=np.int32).reshape(-1, 1)
        co = g.integers(1, 2 ** 63, n + 1, dtype=np.uint64)
        row = {}
        for s in ("balanced", "estrin", "horner"):
            t = fpe.Tree(ex, co, s, fpe.BIGINT).upload(dev)
            lout = int(fpe.lib.fpe_bigint_out_limbs(t.handle, lx))
            out = torch.empty((batch, lout), dtype=torch.int32, device=dev)
            ws = torch.empty(int(fpe.lib.fpe_bigint_workspace_bytes(t.handle, lout, batch)) + 256, dtype=torch.uint8,
                             device=dev)
            fpe.eval_bigint(t, x, out=out, workspace=ws, lout=lout)
            torch.cuda.synchronize()
            ms = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fpe.eval_bigint(t, x, out=out, workspace=ws, lout=lout, check=False)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            row[s] = float(np.median(ms))
        res[f"terms{n + 1}"] = {"ms": row, "estrin_over_balanced": row["estrin"] / row["balanced"],
                                "horner_over_balanced": row["horner"] / row["balanced"]}
    return res


def compose_phase(fpe, fpe_inputs, torch, dev, reps: int = 3):
    """4096 instances of p(q(x)) mod 2^31-1, deg p = 255, deg q = 15."""
    inp = fpe_inputs.compose_batch()
    b, dp1 = inp.p.shape
    ex = np.arange(dp1, dtype=np.int32).reshape(-1, 1)
    q = torch.from_numpy(np.ascontiguousarray(inp.q.astype(np.int32))).to(dev)
    res = {}
    for s in ("balanced", "estrin", "horner"):
        t = fpe.Tree(ex, inp.p.astype(np.uint64), s, fpe.MODP, fpe.P31).upload(dev)
        out = fpe.compose(t, q)
        ws = torch.empty(int(fpe.lib.fpe_compose_workspace_bytes(t.handle, inp.q.shape[1] - 1)) + 256,
                         dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fpe.compose(t, q, out=out, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        m = float(np.median(ms))
        res[s] = {"ms": m, "instances_per_s": b / (m * 1e-3)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--points", type=int, default=10_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-points", type=int, default=600_000)
    ap.add_argument("--no-extra", action="store_true", help="skip the served, mod-p and composition phases")
    ap.add_argument("--served-requests", type=int, default=10_000)
    ap.add_argument("--served-only", action="store_true",
                    help="run only the served stream (for a profiler run of the fused kernels) and print its results")
    ap.add_argument("--copy-probe", type=float, default=0,
                    help="after the timed steps, copy a device buffer of this many bytes three times "
                         "(calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the evaluation shards by "
                          "point range without communication, so more GPUs are not measured here"}))
        sys.exit(2)

    import torch

    import fpe_inputs
    import paper_1307_5655_amd as fpe

    dev = torch.device("cuda:0")
    if args.served_only:
        served, latency = served_phase(fpe, fpe_inputs, torch, dev, args.served_requests)
        print(json.dumps({"served": {"saturation": served, "poisson": latency}}), flush=True)
        return
    degrees = (3000, 5000)
    schemes = ("balanced", "estrin", "horner")
    forms = (("f32c", fpe.F32C), ("f64", fpe.F64))
    inputs, trees, xs, outs, ws, nfb = {}, {}, {}, {}, {}, {}
    term_evals, df_step_ops = {}, {}
    for n in degrees:
        inp = fpe_inputs.sparse_uni(n, npts=args.points)
        inputs[n] = inp
        e, c = inp.terms()
        xs[n] = torch.from_numpy(inp.points).to(dev)
        for s in schemes:
            for fname, dom in forms:
                t = fpe.Tree(e, c, s, dom).upload(dev)
                trees[(n, s, fname)] = t
                outs[(n, s, fname)] = torch.empty(args.points, dtype=torch.float64, device=dev)
                term_evals[(n, s, fname)] = float(t.info.n_terms) * args.points
                df_step_ops[(n, s, fname)] = float(sum(
                    k * o for k, o in zip(t.info.n_ops_kind, DF32_OPS_BY_KIND))) * args.points
                if dom == fpe.F32C:
                    ws[(n, s)] = torch.empty(fpe.workspace_bytes(t, args.points) + 256, dtype=torch.uint8,
                                             device=dev)
                    nfb[(n, s)] = torch.zeros(1, dtype=torch.int64, device=dev)
    keys = list(trees)
    hev = HipEvents()
    ev = {k: [] for k in keys}

    def step(record):
        for k in keys:
            n, s, fname = k
            kw = {}
            if record:
                e0, e1 = hev.create(), hev.create()
                ev[k].append((e0, e1))
                kw["events"] = (e0, e1)
            if fname == "f32c":
                fpe.evaluate(trees[k], [xs[n]], out=outs[k], workspace=ws[(n, s)],
                             nfallback_out=nfb[(n, s)], **kw)
            else:
                fpe.evaluate(trees[k], [xs[n]], out=outs[k], **kw)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    total_te = sum(term_evals.values())
    value = total_te / ((t1 - t0) / args.steps)

    # per-kernel (walk) durations from the events on the launch stream
    walk_ms = {k: float(np.mean([hev.elapsed_ms(a, b) for a, b in ev[k]])) for k in keys}
    per = {}
    for fname, _ in forms:
        per[fname] = {f"n{k[0]}_{k[1]}": {"walk_ms": round(walk_ms[k], 4),
                                           "term_evals_per_s": term_evals[k] / (walk_ms[k] * 1e-3),
                                           "n_table": int(trees[k].info.n_table),
                                           "walk_depth": int(trees[k].info.walk_depth)}
                      for k in keys if k[2] == fname}

    # dominant kernel: the compensated-FP32 walk (most of the step's time)
    df_keys = [k for k in keys if k[2] == "f32c"]
    df_ops = sum(df_step_ops[k] for k in df_keys)
    df_time = sum(walk_ms[k] for k in df_keys) * 1e-3
    f64_keys = [k for k in keys if k[2] == "f64"]
    f64_fma = sum(term_evals[k] for k in f64_keys)
    f64_time = sum(walk_ms[k] for k in f64_keys) * 1e-3
    traffic = measured_traffic()
    roofline = {
        "kernel": "k_eval_df32 (compensated FP32 walk), 6 launches per step",
        "bound": "alu",
        "achieved": df_ops / df_time / 1e12,
        "peak": FP32_VALU_PEAK / 1e12,
        "unit": "TOP/s (FP32 VALU lane-ops)",
        "frac": (df_ops / df_time) / FP32_VALU_PEAK,
        "traffic": traffic,
        "ops_per_term_eval": df_ops / sum(term_evals[k] for k in df_keys),
        "avg_launch_ms": df_time * 1e3 / len(df_keys),
    }
    roofline_f64 = {
        "kernel": "k_eval_f64 (plain FP64 walk), 6 launches per step",
        "bound": "alu",
        "achieved": f64_fma / f64_time / 1e12,
        "peak": FP64_FMA_PEAK / 1e12,
        "unit": "T FMA/s (FP64)",
        "frac": (f64_fma / f64_time) / FP64_FMA_PEAK,
        "avg_launch_ms": f64_time * 1e3 / len(f64_keys),
    }

    # accuracy of the last step on a sample (outside the timed region)
    from oracle import native
    rng = np.random.default_rng(0)
    acc = {}
    fb = {}
    cond_stats = {}
    for n in degrees:
        idx = np.sort(rng.choice(args.points, 2000, replace=False))
        xs_s = inputs[n].points[idx]
        ref = native.dd_value(inputs[n].coeffs, xs_s)
        pt = native.ptilde(inputs[n].coeffs, xs_s)
        cond = pt / np.abs(ref)
        cond_stats[f"n{n}"] = {"median": float(np.median(cond)), "p99": float(np.quantile(cond, 0.99)),
                               "max": float(cond.max())}
        for s in schemes:
            y32 = outs[(n, s, "f32c")].cpu().numpy()[idx]
            y64 = outs[(n, s, "f64")].cpu().numpy()[idx]
            acc[f"n{n}_{s}"] = {"f32c_max_rel_err": float(np.max(np.abs(y32 - ref) / np.abs(ref))),
                                "f64_max_scaled_err": float(np.max(np.abs(y64 - ref) / pt))}
            fb[f"n{n}_{s}"] = nfb[(n, s)].item() / args.points

    if args.copy_probe > 0:
        nbytes = int(args.copy_probe) // 8 * 8
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # free the main workload before the side phases
    del trees, outs, ws, xs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    served = latency = modp = compose = ival = big = None
    if not args.no_extra:
        log("served stream")
        served, latency = served_phase(fpe, fpe_inputs, torch, dev, args.served_requests)
        log("mod-p trivariate")
        modp = modp_phase(fpe, fpe_inputs, torch, dev, hev)
        log("composition")
        compose = compose_phase(fpe, fpe_inputs, torch, dev)
        log("interval")
        ival = interval_phase(fpe, fpe_inputs, torch, dev, hev, args.points)
        log("big integers")
        big = bigint_phase(fpe, torch, dev)

    cpu = None
    if not args.no_cpu:
        # the CPU oracle as it stands (C, -O2, OpenMP over points): the
        # double-double Hörner that the compensated results are checked
        # against and the plain FP64 Hörner, each over the dense coefficient
        # vector, on the first cpu_points points of both degrees
        log("cpu oracle")
        native.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        cores = native.threads()
        te = 0.0
        c0 = time.perf_counter()
        for n in degrees:
            xs_c = np.ascontiguousarray(inputs[n].points[: args.cpu_points])
            nnz = float(np.count_nonzero(inputs[n].coeffs))
            native.dd_value(inputs[n].coeffs, xs_c)
            native.horner_f64(inputs[n].coeffs, xs_c, use_fma=False)
            te += 2 * nnz * len(xs_c)
        c1 = time.perf_counter()
        cpu = {"value": te / (c1 - c0), "unit": "term-evals/s", "cores": cores, "kind": "oracle",
               "sample": f"double-double and plain FP64 Hörner (C, -O2, OpenMP) on the first "
                         f"{args.cpu_points} points of degrees 3000 and 5000 ({te:.3g} term-evals, "
                         f"{c1 - c0:.2f} s)"}

    out = {
        "metric": "term-evals/sec at stated rel. error vs FP64 oracle; p50/p99 request latency",
        "value": value,
        "unit": "term-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 double-float (f64 fallback) + f64",
        "data": "synthetic",
        "config": {"workload": "sparse univariate, degrees 3000 and 5000, 10% zero coefficients, "
                               "1e7 points U[-1.05,1.05]; schemes balanced/Estrin/Hörner; compensated "
                               "FP32 with FP64 fallback and plain FP64 (12 evaluations per step)",
                   "points": args.points, "term_evals_per_step": total_te},
        "roofline": roofline,
        "roofline_f64": roofline_f64,
        "cpu_baseline": cpu,
        "per_evaluation": per,
        "accuracy_sampled": acc,
        "condition_sampled": cond_stats,
        "fallback_frac": fb,
        "latency_ms": None if latency is None else {"p50": latency["p50_ms"], "p99": latency["p99_ms"]},
        "served": None if served is None else {"saturation": served, "poisson": latency},
        "modp_trivariate": modp,
        "compose_4096": compose,
        "interval_1e7": ival,
        "bigint_256bit_points": big,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
