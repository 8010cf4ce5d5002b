"""Benchmark of the evaluation-tree hot path on one MI355X.

Workload (timed step): the sparse univariate workload of degrees 3000 and
5000 (coefficients U[-1, 1], 10 % of the exponents below the degree zeroed),
1e7 points U[-1.05, 1.05] resident in HBM, each degree under the balanced,
Estrin and Hörner schemes, each in the served form (compensated FP32 with a
running error bound and FP64 re-evaluation of flagged points) and in plain
FP64: 12 evaluations, 4.32e11 term-evaluations per step.  Trees are compiled
and uploaded once, before the timed region.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects): the
value is whole-step term-evaluations per second; the accuracy of the last
step against the CPU oracle is checked on a sample after the timed region.
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

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
N_CU, CLOCK_GHZ, LANES_PER_CU = 256, 2.4, 64
VALU_LANE_OPS = N_CU * LANES_PER_CU * CLOCK_GHZ * 1e9      # 3.93e13 lane-instructions/s
FP64_FMA_PEAK = 78.6e12 / 2                                # FMA/s
DF32_OPS_PER_TERM = 16      # FP32 VALU ops of one double-float multiply-add (TwoProd,
                            # 3 cross-term fmas, TwoSum, 2 adds, FastTwoSum)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--points", type=int, default=10_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-points", type=int, default=400_000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the evaluate path "
                          "shards by point range without communication (see DESIGN.md)"}))
        sys.exit(2)

    import torch

    import fpe_inputs
    import paper_1307_5655_amd as fpe

    dev = torch.device("cuda:0")
    degrees = (3000, 5000)
    schemes = ("balanced", "estrin", "horner")
    forms = (("f32c", fpe.F32C), ("f64", fpe.F64))
    inputs, trees, xs, outs, ws, nfb = {}, {}, {}, {}, {}, {}
    term_evals = {}
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
        ks = [k for k in keys if k[2] == fname]
        per[fname] = {f"n{k[0]}_{k[1]}": {"walk_ms": round(walk_ms[k], 4),
                                           "term_evals_per_s": term_evals[k] / (walk_ms[k] * 1e-3)}
                      for k in ks}

    # dominant kernel: the double-float walk (most of the step's time)
    df_keys = [k for k in keys if k[2] == "f32c"]
    df_ops = sum(term_evals[k] * DF32_OPS_PER_TERM for k in df_keys)
    df_time = sum(walk_ms[k] for k in df_keys) * 1e-3
    f64_keys = [k for k in keys if k[2] == "f64"]
    f64_fma = sum(term_evals[k] for k in f64_keys)
    f64_time = sum(walk_ms[k] for k in f64_keys) * 1e-3
    roofline = {
        "kernel": "k_eval_df32 (compensated FP32 walk)",
        "bound": "alu",
        "achieved": df_ops / df_time / 1e12,
        "peak": VALU_LANE_OPS / 1e12,
        "unit": "TOP/s (FP32 VALU lane-ops)",
        "frac": (df_ops / df_time) / VALU_LANE_OPS,
        "traffic": None,
        "ops_per_term_eval": DF32_OPS_PER_TERM,
    }
    roofline_f64 = {
        "kernel": "k_eval_f64 (plain FP64 walk)",
        "bound": "alu",
        "achieved": f64_fma / f64_time / 1e12,
        "peak": FP64_FMA_PEAK / 1e12,
        "unit": "T FMA/s (FP64)",
        "frac": (f64_fma / f64_time) / FP64_FMA_PEAK,
    }

    # accuracy of the last step on a sample (outside the timed region)
    from oracle import native
    rng = np.random.default_rng(0)
    acc = {}
    fb = {}
    for n in degrees:
        idx = np.sort(rng.choice(args.points, 2000, replace=False))
        xs_s = inputs[n].points[idx]
        ref = native.dd_value(inputs[n].coeffs, xs_s)
        pt = native.ptilde(inputs[n].coeffs, xs_s)
        for s in schemes:
            y32 = outs[(n, s, "f32c")].cpu().numpy()[idx]
            y64 = outs[(n, s, "f64")].cpu().numpy()[idx]
            acc[f"n{n}_{s}"] = {"f32c_max_rel_err": float(np.max(np.abs(y32 - ref) / np.abs(ref))),
                                "f64_max_scaled_err": float(np.max(np.abs(y64 - ref) / pt))}
            fb[f"n{n}_{s}"] = nfb[(n, s)].item() / args.points

    cpu = None
    if not args.no_cpu:
        # the CPU oracle as it stands: plain FP64 Hörner over the dense
        # coefficient vector, OpenMP over points, on the host's cores
        native.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        cores = native.threads()
        te = 0.0
        c0 = time.perf_counter()
        for n in degrees:
            xs_c = inputs[n].points[: args.cpu_points]
            native.horner_f64(inputs[n].coeffs, xs_c, use_fma=False)
            te += float(np.count_nonzero(inputs[n].coeffs)) * len(xs_c)
        c1 = time.perf_counter()
        cpu = {"value": te / (c1 - c0), "unit": "term-evals/s", "cores": cores, "kind": "oracle",
               "sample": f"plain FP64 Hörner (C, -O2, OpenMP) on the first {args.cpu_points} points of "
                         f"degrees 3000 and 5000 ({te:.3g} term-evals, {c1 - c0:.2f} s)"}

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
        "dtype": "f32 (double-float) + f64",
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
        "fallback_frac": fb,
        "latency_ms": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
