"""Benchmark of the evaluation-tree hot path on one MI355X.

Timed step: the sparse univariate workload of degrees 3000 and 5000
(coefficients U[-1, 1], 10 % of the exponents below the degree zeroed),
1e7 points U[-1.05, 1.05] resident in HBM, each degree under the balanced,
Estrin and Hörner schemes, each in the served form (compensated FP32 with a
running error bound, each point's condition number written beside its value,
and FP64 re-evaluation of flagged points) and in plain FP64: 12 evaluations,
4.3e11 term-evaluations per step.  Trees are compiled and uploaded once,
before the timed region.

After the timed region (not part of ``value``): the compensated walks without
condition output; the accuracy of a step against the CPU oracle on a sample;
the measured issue rates of the operations the kernels are bound by (rate
probes) and the HBM copy bandwidth; the dense degree-1023 polynomial at 1e5
points; a served stream (Poisson arrivals of uneven evaluate requests through
the continuous-batching server: 10^4 requests, first all at once for the
saturation rate, then at 0.5, 0.8 and 0.95 times that rate) for p50/p99
latency; the exact mod 2^61-1 trivariate workload and the batched composition
mod 2^31-1, each with its roofline; intervals; big integers; and the CPU
oracle timed on bounded samples (plain FP64 Hörner on 1 core and on all
cores, the mod-p definition, schoolbook composition).

Prints one JSON line; ``roofline`` describes the dominant kernel (the
compensated-FP32 walk, priced on 11 FP32 operations per term-evaluation),
``roofline_f64`` the plain FP64 walk.
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
# dense int8 matrix-core operations per second (published; a multiply-add is two)
I8_MFMA_PEAK = 5.0e15
# FP32 operations of one compensated multiply-add a * X + b (X read as two
# floats): product and its error by fma (2), two cross terms (2), TwoSum (6),
# two low-order adds (2), FastTwoSum (3), then the running error bound:
# e_a |X| + e_b (1 fma, when the product's operand is an accumulator),
# 20 u^2 |p| (1 fma) and 6 u^2 |b| (1 fma when b is an accumulator; a
# coefficient's term is a constant of the op).  Per step kind: LEAF_ADD
# a X + top 17, NODE_OPEN top X + b 17, LEAF_OPEN a X + b 16, NODE_ADD
# top X + below 18; END (once per point) is not counted.  The condition sum
# (1 more fma) is computed when per-point condition numbers are requested,
# which the timed step does.
DF32_OPS_BY_KIND = (17, 17, 16, 18, 0)
# The algorithmic FP32 operation count of one compensated step that the
# roofline fraction is quoted on: TwoProd 2, TwoSum 6, first-order error
# propagation 2, running bound 1 (a compensated Hörner step).  The walk's own
# count (above) adds the double-float renormalisation and cross terms that
# keep 48 bits over a chain of 5000 steps; its fraction is reported beside.
DF32_ALG_OPS = 11


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
    ideal_s = float(sum(max(DF32_ALG_OPS * t.info.n_terms * m.points.shape[1] / FP32_VALU_PEAK,
                            (8 * m.points.shape[0] + 8) * m.points.shape[1] / (HBM_PEAK_GBS * 1e9))
                        for _, t, _, _, m in prepared))
    ideal_impl_s = float(sum(max(sum(k * o for k, o in zip(t.info.n_ops_kind, DF32_OPS_BY_KIND)) * m.points.shape[1]
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
           "ideal_s": ideal_s, "roofline_frac_of_wall": ideal_s / wall_sat,
           "ideal_s_walk_ops": ideal_impl_s, "roofline_frac_of_wall_walk_ops": ideal_impl_s / wall_sat}
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


# Published MI355X peaks the probes are compared with (per second).
PUBLISHED = {"fma_f64": FP64_FMA_PEAK, "fma_f32": FP32_VALU_PEAK, "mfma_i8": 5.0e15, "copy": HBM_PEAK_GBS * 1e9,
             "mad_u64": FP64_FMA_PEAK}


def probe_phase(torch, dev):
    """Measured issue rates of the operations the kernels are bound by
    (libfpe_probe.so: independent chains of one operation per thread), and the
    HBM bandwidth of a plain copy."""
    import ctypes
    L = ctypes.CDLL(os.path.join(ROOT, "paper_1307_5655_amd", "libfpe_probe.so"))
    L.fpe_probe_launch.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    L.fpe_probe_launch.restype = ctypes.c_double
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    blocks = 256 * 16
    sink = torch.empty(blocks * 256 * 16, dtype=torch.uint8, device=dev)
    nbytes = 2 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    runs = [("fma_f64", 0, blocks, 10000, "FP64 FMA/s"), ("fma_f32", 1, blocks, 10000, "FP32 FMA/s (not packed)"),
            ("df32_step", 2, blocks, 4000, "compensated steps/s"), ("m61_mac", 3, blocks, 4000, "mod 2^61-1 MAC/s"),
            ("mad_u64", 4, blocks, 10000, "v_mad_u64_u32/s"), ("mfma_i8", 5, 256 * 8, 100, "int8 MFMA ops/s"),
            ("copy", 6, 256 * 32, 0, "bytes/s read + written")]
    res = {}
    for name, kind, b, iters, unit in runs:
        args = (kind, b, iters, ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                ctypes.c_void_p(dst.data_ptr()), nbytes, st)
        if L.fpe_probe_launch(*args) < 0:
            raise RuntimeError(f"probe {name} failed")
        ms = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            ops = L.fpe_probe_launch(*args)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        m = float(np.median(ms))
        rate = ops / (m * 1e-3)
        res[name] = {"rate": rate, "unit": unit, "ms": m}
        if name in PUBLISHED:
            res[name]["published_peak"] = PUBLISHED[name]
            res[name]["frac_of_published"] = rate / PUBLISHED[name]
    res["df32_step"]["fp32_ops_per_s"] = res["df32_step"]["rate"] * DF32_OPS_BY_KIND[3]
    del src, dst, sink
    return res


def dense_phase(fpe, fpe_inputs, torch, dev, reps: int = 50):
    """The plain method at its small size: one dense polynomial of degree 1023
    at 1e5 points, Hörner and Estrin, plain FP64 (and the compensated form
    beside it); each figure the average of back-to-back launches."""
    inp = fpe_inputs.dense_uni()
    e, c = inp.terms()
    x = torch.from_numpy(inp.points).to(dev)
    npts = len(inp.points)
    res = {}
    for s in ("horner", "estrin"):
        for fname, dom in (("f64", fpe.F64), ("f32c", fpe.F32C)):
            t = fpe.Tree(e, c, s, dom).upload(dev)
            out = torch.empty(npts, dtype=torch.float64, device=dev)
            ws = torch.empty(fpe.workspace_bytes(t, npts) + 256, dtype=torch.uint8, device=dev) \
                if dom == fpe.F32C else None
            for _ in range(3):
                fpe.evaluate(t, [x], out=out, workspace=ws)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fpe.evaluate(t, [x], out=out, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            te = float(t.info.n_terms) * npts
            row = {"ms_per_launch": ms, "term_evals_per_s": te / (ms * 1e-3)}
            if dom == fpe.F64:
                row["frac_of_fp64_fma_peak"] = te / (ms * 1e-3) / FP64_FMA_PEAK
            res[f"{s}_{fname}"] = row
    return res


def compose_macs(tree, dq: int) -> float:
    """Modular multiply-adds of one instance's composition walk: every child
    value u(C) times q^{d(C)} (a polynomial product, (deg u(C) + 1) x
    (d(C) dq + 1) multiply-adds), the root's own power, and the powers q^d
    built by halving (q^d = q^{floor(d/2)} q^{ceil(d/2)}), as the compiler
    plans them for composition trees."""
    nd = tree.nodes()
    deg = [0] * len(nd)
    macs = 0.0
    pdegs = set()
    for i, n in enumerate(nd):
        d = int(n["pdeg"])
        if n["parent"] >= 0:
            macs += (deg[i] + 1) * (d * dq + 1)
            par = int(n["parent"])
            deg[par] = max(deg[par], deg[i] + d * dq)
        elif d > 0:
            macs += (deg[i] + 1) * (d * dq + 1)
        if d > 0:
            pdegs.add(d)
    have = {1}

    def ensure(d):
        nonlocal macs
        if d in have:
            return
        a, b = d // 2, d - d // 2
        ensure(a)
        ensure(b)
        macs += (a * dq + 1) * (b * dq + 1)
        have.add(d)

    for d in sorted(pdegs):
        ensure(d)
    return macs


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_phase(native, fpe_inputs, inputs, degrees, npts_all: int, npts_one: int):
    """The oracle as it stands on the host cores: plain FP64 Hörner (C,
    -O2, no fused multiply-add) on 1 core and on all cores, the naive
    mod 2^61-1 definition on the trivariate workload, and schoolbook
    composition."""
    ncores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = cpu_model()
    out = {"model": model}
    for label, threads, npts in (("all_cores", ncores, npts_all), ("one_core", 1, npts_one)):
        native.set_threads(threads)
        te = 0.0
        c0 = time.perf_counter()
        for n in degrees:
            xs_c = np.ascontiguousarray(inputs[n].points[:npts])
            native.horner_f64(inputs[n].coeffs, xs_c, use_fma=False)
            te += float(np.count_nonzero(inputs[n].coeffs)) * len(xs_c)
        c1 = time.perf_counter()
        out[label] = {"value": te / (c1 - c0), "unit": "term-evals/s", "cores": native.threads(), "kind": "oracle",
                      "sample": f"plain FP64 Hörner (C, -O2, no fma) over the dense coefficient vectors of "
                                f"degrees {' and '.join(map(str, degrees))} at their first {npts} points "
                                f"({te:.3g} term-evals, {c1 - c0:.2f} s), {model}"}
    native.set_threads(ncores)
    tri = fpe_inputs.trivariate(npts=20_000)
    c0 = time.perf_counter()
    native.modp_eval(tri.exps, tri.coeffs, (1 << 61) - 1, tri.points)
    c1 = time.perf_counter()
    te = float(len(tri.coeffs)) * tri.points.shape[1]
    out["modp_trivariate"] = {"value": te / (c1 - c0), "unit": "term-evals/s", "cores": native.threads(),
                              "kind": "oracle", "sample": f"naive mod 2^61-1 definition (unsigned __int128), "
                                                          f"12,341 terms at the first 20,000 points ({c1 - c0:.2f} s)"}
    cb = fpe_inputs.compose_batch()
    k = 128
    c0 = time.perf_counter()
    native.compose_modp(cb.p[:k], cb.q[:k], (1 << 31) - 1)
    c1 = time.perf_counter()
    out["compose"] = {"value": k / (c1 - c0), "unit": "instances/s", "cores": native.threads(), "kind": "oracle",
                      "sample": f"schoolbook Hörner composition of the first {k} of the 4096 instances "
                                f"({c1 - c0:.2f} s)"}
    return out


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


def modp_roofline(modp, probes):
    """The modular walk against the measured rate of its own step (one
    multiply-add mod 2^61 - 1, the 64 x 64 -> 128-bit product from four
    32 x 32 -> 64 partial products, then two folds), and against the
    wide-multiply rate: four v_mad_u64_u32 per step at the chip's 39.3e12/s."""
    best = max(v["term_evals_per_s"] for v in modp.values())
    avg = float(np.mean([v["term_evals_per_s"] for v in modp.values()]))
    peak = probes["m61_mac"]["rate"]
    return {"kernel": "k_eval_m61 (nested walk mod 2^61-1), schemes B/E/H", "bound": "alu",
            "achieved": avg, "peak": peak, "unit": "mod-2^61-1 multiply-adds/s",
            "peak_source": "measured: the walk's multiply-add in independent chains (FPE_PROBE_M61_MAC)",
            "frac": avg / peak, "frac_best_scheme": best / peak,
            "frac_of_wide_multiply_peak": 4 * avg / FP64_FMA_PEAK}


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


def bigpoint_phase(fpe, torch, dev, reps: int = 3):
    """The Benchmarks section's setting: one polynomial (64-bit coefficients)
    at ONE point of 512 bits, term counts at and just past 128 and 256; time
    per scheme and the ratio to the balanced scheme (the form of Figure 1)."""
    g = np.random.default_rng([13075655, 9])
    lx = 32
    x = torch.from_numpy(g.integers(0, 1 << 16, size=lx, dtype=np.int64).astype(np.int32)).to(dev)
    res = {}
    for n in (127, 128, 129, 255, 256, 257):
        ex = np.arange(n + 1, dtype=np.int32).reshape(-1, 1)
        co = g.integers(1, 2 ** 63, n + 1, dtype=np.uint64)
        row = {}
        for s in ("balanced", "estrin", "horner"):
            t = fpe.Tree(ex, co, s, fpe.BIGINT).upload(dev)
            out = fpe.eval_bigpoint(t, x)
            ws = torch.empty(int(fpe.lib.fpe_bigpoint_workspace_bytes(t.handle, lx)) + 256, dtype=torch.uint8,
                             device=dev)
            fpe.eval_bigpoint(t, x, out=out, workspace=ws)
            ms = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fpe.eval_bigpoint(t, x, out=out, workspace=ws, check=False)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            row[s] = float(np.median(ms))
        res[f"terms{n + 1}"] = {"ms": row, "estrin_over_balanced": row["estrin"] / row["balanced"],
                                "horner_over_balanced": row["horner"] / row["balanced"]}
    return res


def compose_bigint_phase(fpe, torch, dev, reps: int = 3):
    """Composition over the natural numbers at one big point (fpe_compose_bigint:
    Kronecker substitution into the walk at one big point): p with 64-bit
    coefficients and 16..18 or 32..34 terms, q of degree 3 with 64-bit
    coefficients; time per scheme (single calls) and the ratio to balanced."""
    g = np.random.default_rng([13075655, 10])
    q = [int(c) for c in g.integers(1, 2 ** 63, 4, dtype=np.uint64)]
    res = {}
    for n in (15, 16, 17, 31, 32, 33):
        ex = np.arange(n + 1, dtype=np.int32).reshape(-1, 1)
        co = g.integers(1, 2 ** 63, n + 1, dtype=np.uint64)
        row = {}
        for s in ("balanced", "estrin", "horner"):
            t = fpe.Tree(ex, co, s, fpe.BIGINT).upload(dev)
            out = fpe.compose_bigint(t, q)
            ws = torch.empty(fpe.compose_bigint_workspace_bytes(t, q) + 256, dtype=torch.uint8, device=dev)
            fpe.compose_bigint(t, q, out=out, workspace=ws)
            ms = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fpe.compose_bigint(t, q, out=out, workspace=ws, check=False)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            row[s] = float(np.median(ms))
        res[f"terms{n + 1}"] = {"ms": row, "estrin_over_balanced": row["estrin"] / row["balanced"],
                                "horner_over_balanced": row["horner"] / row["balanced"],
                                "coef_limbs": int(out.shape[1]), "coefs": int(out.shape[0])}
    return res


def warm_events(torch):
    """Record and wait on one pair of torch timing events: their first use
    sets up state on the host (tens of milliseconds), which would otherwise
    land inside the first timed region of a phase run on its own."""
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    b.record()
    torch.cuda.synchronize()
    a.elapsed_time(b)


def term_path_ops(exps) -> float:
    """Operations the term-parallel kernel issues per point: each term one
    multiplication per variable (by its entry of the point's power table,
    x^0 = 1 included) and one addition; the table, x_j^k for k up to the
    largest exponent of x_j, by fast exponentiation: bit_length(k) squarings
    and popcount(k) multiplications an entry."""
    e = np.asarray(exps, dtype=np.int64)
    ops = float(e.shape[0] * (e.shape[1] + 1))
    for j in range(e.shape[1]):
        ks = np.arange(int(e[:, j].max()) + 1)
        ops += float(sum(int(k).bit_length() + bin(int(k)).count("1") for k in ks))
    return ops


def few_points_phase(fpe, fpe_inputs, torch, dev, reps: int = 20, probes=None):
    """Few points, big tree: the trivariate degree-40 polynomial (12,341
    terms; FP64 coefficients U[-1, 1] at points U[-1, 1]^3, and mod 2^61 - 1)
    at 1 to 4096 points, by the tree walk (one lane per point) and by the
    term-parallel path (one workgroup per point, DPP wavefront sums), with the
    library's choice.  The term path's roofline: its issued operations per
    point over the launch time, against the FP64 multiply/add rate, and mod
    2^61 - 1 against the measured rate of the modular multiply-add (each
    modular multiplication counted as one); few points cannot fill the chip,
    so the fraction rises with the point count."""
    warm_events(torch)
    tri = fpe_inputs.trivariate(npts=4096)
    g = np.random.default_rng([13075655, 960])
    ops_pt = term_path_ops(tri.exps)
    peaks = {"f64": (FP64_FMA_PEAK, "FP64 multiplies and adds/s", "published: 39.3e12 FP64 lane-operations/s"),
             "modp": ((probes or {}).get("m61_mac", {}).get("rate"), "mod-2^61-1 multiplications/s",
                      "measured: the modular multiply-add in independent chains (FPE_PROBE_M61_MAC)")}
    res = {"term_path_ops_per_point": ops_pt}
    for name, dom in (("f64", fpe.F64), ("modp", fpe.MODP)):
        if dom == fpe.F64:
            t = fpe.Tree(tri.exps, g.uniform(-1, 1, len(tri.exps)), "estrin", dom).upload(dev)
            pts = [torch.from_numpy(g.uniform(-1, 1, 4096)).to(dev) for _ in range(3)]
        else:
            t = fpe.Tree(tri.exps, tri.coeffs, "estrin", dom, fpe.P61).upload(dev)
            pts = [torch.from_numpy(tri.points[j].view(np.int64).copy()).to(dev) for j in range(3)]
        for n in (1, 16, 256, 4096):
            sub = [p[:n].contiguous() for p in pts]
            row = {}
            for path in ("walk", "terms"):
                fpe.evaluate(t, sub, path=path)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    fpe.evaluate(t, sub, path=path)
                e1.record()
                torch.cuda.synchronize()
                row[f"{path}_ms"] = e0.elapsed_time(e1) / reps
            row["speedup"] = row["walk_ms"] / row["terms_ms"]
            row["library_choice"] = fpe.eval_path(t, n)
            peak = peaks[name][0]
            row["terms_ops_per_s"] = n * ops_pt / (row["terms_ms"] * 1e-3)
            row["terms_frac"] = row["terms_ops_per_s"] / peak if peak else None
            res[f"{name}_{n}"] = row
        peak, unit, src = peaks[name]
        big = res[f"{name}_4096"]
        res[f"roofline_{name}"] = {"kernel": f"k_eval_terms<{0 if name == 'f64' else 1}> at 4096 points",
                                   "bound": "alu", "achieved": big["terms_ops_per_s"], "peak": peak, "unit": unit,
                                   "peak_source": src, "frac": big["terms_frac"]}
    return res


def compose_phase(fpe, fpe_inputs, torch, dev, reps: int = 10):
    """4096 instances of p(q(x)) mod 2^31-1, deg p = 255, deg q = 15: the time
    per call over `reps` back-to-back calls (the throughput of a stream of
    batches), and the median time of single calls with the device idle
    before each (latency, including the schedule's upload and the launches)."""
    warm_events(torch)
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
        for _ in range(2):   # warm: the schedule is built and uploaded on the first calls
            fpe.compose(t, q, out=out, workspace=ws)
        torch.cuda.synchronize()
        # one untimed pass of the back-to-back loop: run on its own, the phase's
        # first back-to-back window took a one-time host stall of tens of
        # milliseconds (a gap before its first call in the kernel trace), even
        # after a warm-up pair of timing events
        for _ in range(reps):
            fpe.compose(t, q, out=out, workspace=ws)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fpe.compose(t, q, out=out, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        m = e0.elapsed_time(e1) / reps
        single = []
        for _ in range(3):
            e0.record()
            fpe.compose(t, q, out=out, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            single.append(e0.elapsed_time(e1))
        macs = compose_macs(t, inp.q.shape[1] - 1) * b
        res[s] = {"ms": m, "single_call_ms": float(np.median(single)), "instances_per_s": b / (m * 1e-3),
                  "mod_macs": macs, "mod_macs_per_s": macs / (m * 1e-3),
                  # the product method fpe_compose picks: the level walk on the matrix
                  # cores for the divide-and-conquer trees, the fused VALU walk for
                  # Hörner's 255 levels
                  "product": "fused" if s == "horner" else "mfma"}
        if s == "horner":
            res[s]["frac_of_mad_u64_peak"] = macs / (m * 1e-3) / FP64_FMA_PEAK
        else:
            # one modular multiply-add = 16 products of balanced 8-bit digits
            # (2 ops each) on the int8 matrix cores
            res[s]["i8_ops"] = 32.0 * macs
            res[s]["frac_of_i8_mfma_peak"] = 32.0 * macs / (m * 1e-3) / I8_MFMA_PEAK
    return res


def compose_methods_phase(fpe, fpe_inputs, torch, dev, reps: int = 3):
    """Composition by product method: the 4096 x (255 o 15) workload with the
    fused walk, with the op-by-op walk using schoolbook or transform
    (subquadratic) products, and with the level walk on the matrix cores;
    then larger compositions (64 instances of
    degree 511, 512 and 1023 in p, degree 15 in q), where the transform
    products make the divide-and-conquer schemes pay off against Hörner and
    the term count just past a power of two shows Estrin's staircase."""
    res = {}

    def timed(t, q, product):
        out = fpe.compose(t, q, product=product)
        ws = torch.empty(fpe.compose_workspace_bytes(t, q.shape[1] - 1, product) + 256, dtype=torch.uint8,
                         device=dev)
        fpe.compose(t, q, out=out, workspace=ws, product=product)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fpe.compose(t, q, out=out, workspace=ws, product=product)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    inp = fpe_inputs.compose_batch()
    q = torch.from_numpy(np.ascontiguousarray(inp.q.astype(np.int32))).to(dev)
    ex = np.arange(inp.p.shape[1], dtype=np.int32).reshape(-1, 1)
    c4 = {}
    for s in ("balanced", "estrin", "horner"):
        t = fpe.Tree(ex, inp.p.astype(np.uint64), s, fpe.MODP, fpe.P31).upload(dev)
        c4[s] = {m: timed(t, q, m) for m in ("fused", "schoolbook", "ntt", "mfma")}
    res["4096x255o15_ms"] = c4
    g = np.random.default_rng([13075655, 940])
    for dp in (511, 512, 1023):
        P = g.integers(0, fpe.P31, size=(64, dp + 1), dtype=np.uint32).astype(np.uint64)
        Q = torch.from_numpy(g.integers(0, fpe.P31, size=(64, 16), dtype=np.uint32).astype(np.int32)).to(dev)
        exd = np.arange(dp + 1, dtype=np.int32).reshape(-1, 1)
        row = {}
        for s in ("balanced", "estrin", "horner"):
            t = fpe.Tree(exd, P, s, fpe.MODP, fpe.P31).upload(dev)
            row[s] = {m: timed(t, Q, m) for m in ("schoolbook", "ntt")}
        row["estrin_over_balanced_ntt"] = row["estrin"]["ntt"] / row["balanced"]["ntt"]
        row["horner_over_balanced_ntt"] = row["horner"]["ntt"] / row["balanced"]["ntt"]
        res[f"64x{dp}o15_ms"] = row
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--points", type=int, default=10_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--cpu-points", type=int, default=1_600_000,
                    help="points of the all-cores CPU baseline sample (the 1-core sample takes a tenth)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the phases after the timed step (probes, dense, served, mod-p, composition, ...)")
    ap.add_argument("--served-requests", type=int, default=10_000)
    ap.add_argument("--served-only", action="store_true",
                    help="run only the served stream (for a profiler run of the fused kernels) and print its results")
    ap.add_argument("--probes-only", action="store_true",
                    help="run only the rate probes (for a profiler run of the probe kernels) and print them")
    ap.add_argument("--compose-only", action="store_true",
                    help="run only the 4096 x (255 o 15) composition (for a profiler run of its kernels) and print it")
    ap.add_argument("--interval-only", action="store_true",
                    help="run only the interval walk over 1e7 boxes (for a profiler run of its kernel) and print it")
    ap.add_argument("--bigint-only", action="store_true",
                    help="run only the big-integer phases, many points and one big point (for a profiler run of "
                         "their kernels) and print them")
    ap.add_argument("--few-points-only", action="store_true",
                    help="run only the few-point trivariate comparison (for a profiler run of the term-parallel "
                         "and walk kernels) and print it")
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
    if args.probes_only:
        print(json.dumps({"probes": probe_phase(torch, dev)}), flush=True)
        return
    if args.compose_only:
        print(json.dumps({"compose_4096": compose_phase(fpe, fpe_inputs, torch, dev)}), flush=True)
        return
    if args.few_points_only:
        print(json.dumps({"few_points_trivariate": few_points_phase(fpe, fpe_inputs, torch, dev)}), flush=True)
        return
    if args.interval_only:
        print(json.dumps({"interval_1e7": interval_phase(fpe, fpe_inputs, torch, dev, HipEvents(), args.points)}),
              flush=True)
        return
    if args.bigint_only:
        warm_events(torch)
        print(json.dumps({"bigint_256bit_points": bigint_phase(fpe, torch, dev),
                          "bigint_one_512bit_point": bigpoint_phase(fpe, torch, dev),
                          "compose_bigint_one_point": compose_bigint_phase(fpe, torch, dev)}), flush=True)
        return
    degrees = (3000, 5000)
    schemes = ("balanced", "estrin", "horner")
    forms = (("f32c", fpe.F32C), ("f64", fpe.F64))
    inputs, trees, xs, outs, ws, nfb, conds = {}, {}, {}, {}, {}, {}, {}
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
                    conds[(n, s)] = torch.empty(args.points, dtype=torch.float32, device=dev)
    keys = list(trees)
    hev = HipEvents()
    ev = {k: [] for k in keys}

    # One step: every evaluation of the workload; the compensated ones write
    # each point's condition number p~(|x|) / |y| beside its value.
    def step(record, cond=True, evd=ev):
        for k in keys:
            n, s, fname = k
            kw = {}
            if record:
                e0, e1 = hev.create(), hev.create()
                evd[k].append((e0, e1))
                kw["events"] = (e0, e1)
            if fname == "f32c":
                fpe.evaluate(trees[k], [xs[n]], out=outs[k], workspace=ws[(n, s)], nfallback_out=nfb[(n, s)],
                             cond_out=conds[(n, s)] if cond else None, **kw)
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

    # dominant kernel: the compensated-FP32 walk (most of the step's time),
    # priced on the algorithmic 11 FP32 operations per term-evaluation
    df_keys = [k for k in keys if k[2] == "f32c"]
    df_te = sum(term_evals[k] for k in df_keys)
    df_ops = sum(df_step_ops[k] for k in df_keys)
    df_time = sum(walk_ms[k] for k in df_keys) * 1e-3
    f64_keys = [k for k in keys if k[2] == "f64"]
    f64_fma = sum(term_evals[k] for k in f64_keys)
    f64_time = sum(walk_ms[k] for k in f64_keys) * 1e-3
    traffic = measured_traffic()
    roofline = {
        "kernel": "k_eval_df32 (compensated FP32 walk with condition output), 6 launches per step",
        "bound": "alu",
        "achieved": DF32_ALG_OPS * df_te / df_time / 1e12,
        "peak": FP32_VALU_PEAK / 1e12,
        "unit": "TFLOP/s (FP32 VALU lane-ops, 11 per term-eval)",
        "frac": DF32_ALG_OPS * df_te / df_time / FP32_VALU_PEAK,
        "traffic": traffic,
        "ops_per_term_eval": DF32_ALG_OPS,
        "avg_launch_ms": df_time * 1e3 / len(df_keys),
        "walk_ops_per_term_eval": df_ops / df_te,
        "frac_walk_ops": df_ops / df_time / FP32_VALU_PEAK,
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

    # the compensated walks again without condition output (outside the
    # timed region), for comparison
    ev_nc = {k: [] for k in keys}
    step(True, cond=False, evd=ev_nc)
    step(True, cond=False, evd=ev_nc)
    torch.cuda.synchronize()
    nc_time = sum(float(np.mean([hev.elapsed_ms(a, b) for a, b in ev_nc[k]])) for k in df_keys) * 1e-3
    no_cond = {"walk_ms_total": nc_time * 1e3, "frac": DF32_ALG_OPS * df_te / nc_time / FP32_VALU_PEAK,
               "frac_walk_ops": df_ops / nc_time / FP32_VALU_PEAK}

    # accuracy of the last step on a sample (outside the timed region): the
    # last step wrote values without condition numbers, so one more step with
    # them, whose values the sample checks, and whose condition numbers are
    # compared with the oracle's
    step(False)
    torch.cuda.synchronize()
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
            cg = conds[(n, s)].cpu().numpy()[idx].astype(np.float64)
            # the walk's condition numbers against the oracle's, where the
            # walk stayed in the FP32 range (elsewhere it reports inf / NaN)
            okc = np.isfinite(cg) & np.isfinite(cond)
            acc[f"n{n}_{s}"] = {"f32c_max_rel_err": float(np.max(np.abs(y32 - ref) / np.abs(ref))),
                                "f64_max_scaled_err": float(np.max(np.abs(y64 - ref) / pt)),
                                "f32c_cond_max_rel_dev": float(np.max(np.abs(cg[okc] - cond[okc]) / cond[okc])),
                                "f32c_cond_finite_frac": float(okc.mean())}
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

    # free the main workload's device buffers before the side phases
    del trees, outs, ws, xs, conds
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    probes = dense = served = latency = modp = compose = ival = big = modp_roof = compose_methods = bigpoint = compose_big = None
    few = None
    if not args.no_extra:
        log("rate probes")
        probes = probe_phase(torch, dev)
        log("dense degree 1023")
        dense = dense_phase(fpe, fpe_inputs, torch, dev)
        log("served stream")
        served, latency = served_phase(fpe, fpe_inputs, torch, dev, args.served_requests)
        log("mod-p trivariate")
        modp = modp_phase(fpe, fpe_inputs, torch, dev, hev)
        modp_roof = modp_roofline(modp, probes)
        log("few points, big tree")
        few = few_points_phase(fpe, fpe_inputs, torch, dev, probes=probes)
        log("composition")
        compose = compose_phase(fpe, fpe_inputs, torch, dev)
        log("composition by product method")
        compose_methods = compose_methods_phase(fpe, fpe_inputs, torch, dev)
        log("interval")
        ival = interval_phase(fpe, fpe_inputs, torch, dev, hev, args.points)
        log("big integers")
        big = bigint_phase(fpe, torch, dev)
        log("one big point")
        bigpoint = bigpoint_phase(fpe, torch, dev)
        log("composition over the integers at one big point")
        compose_big = compose_bigint_phase(fpe, torch, dev)

    cpu = None
    if not args.no_cpu:
        log("cpu oracle")
        cpu = cpu_phase(native, fpe_inputs, inputs, degrees, args.cpu_points, args.cpu_points // 10)

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
                               "FP32 with FP64 fallback and condition numbers, and plain FP64 (12 evaluations "
                               "per step)",
                   "points": args.points, "term_evals_per_step": total_te},
        "roofline": roofline,
        "roofline_f64": roofline_f64,
        "cpu_baseline": None if cpu is None else cpu["all_cores"],
        "cpu_baselines": cpu,
        "per_evaluation": per,
        "f32c_without_condition_output": no_cond,
        "accuracy_sampled": acc,
        "condition_sampled": cond_stats,
        "fallback_frac": fb,
        "latency_ms": None if latency is None else {"p50": latency["p50_ms"], "p99": latency["p99_ms"]},
        "peaks_measured": probes,
        "dense_1023_1e5": dense,
        "served": None if served is None else {"saturation": served, "poisson": latency},
        "modp_trivariate": modp,
        "modp_roofline": modp_roof,
        "few_points_trivariate": few,
        "compose_4096": compose,
        "compose_by_product_method": compose_methods,
        "interval_1e7": ival,
        "bigint_256bit_points": big,
        "bigint_one_512bit_point": bigpoint,
        "compose_bigint_one_point": compose_big,
    }
    # no child process is ever started; the device buffers of the phases are
    # released before the line is printed, so the process ends right after it
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
