"""Builds libfpe.so (HIP kernels for gfx950 + host compiler + C-ABI) and the
rate-probe library libfpe_probe.so, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfpe.so")
PROBE_LIB = os.path.join(HERE, "libfpe_probe.so")
PROBE_SOURCES = ["probes.hip"]
SOURCES = ["compile.cpp", "api.cpp", "walk.hip", "eval_f64.hip", "eval_terms.hip", "eval_m61.hip", "eval_df32.hip", "eval_iv.hip", "bigint.hip",
           "serve_kernels.hip", "compose.hip", "ntt.hip", "compose_mfma.hip", "bigpoint.hip", "compose_bigint.hip",
           "server.cpp"]
EXTRA_SOURCES = []

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # error-free transforms (TwoSum, TwoProd) must not be contracted: every
    # intended fused multiply-add is written as an explicit builtin
    "-ffp-contract=off",
    # the walk's branches are wave-uniform: leave them unstructurised so the
    # accumulators are not copied through flow blocks on every op
    "-mllvm", "-structurizecfg-skip-uniform-regions=true",
    # packed FP32 VALU instructions are disabled on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include"),
]


def sources():
    out = []
    for s in SOURCES + EXTRA_SOURCES:
        p = os.path.join(CSRC, s)
        if os.path.exists(p):
            out.append(p)
    return out


def build(verbose: bool = False) -> str:
    objs = []
    procs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    probe_objs = [os.path.join(HERE, "_build", s + ".o") for s in PROBE_SOURCES]
    for src in sources() + [os.path.join(CSRC, s) for s in PROBE_SOURCES]:
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-c"] + lang + [src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if obj not in probe_objs:
            objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the packed-fp32 target feature: harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l]
        if p.returncode != 0 or (verbose and lines):
            print("\n".join(lines), file=sys.stderr)
        if p.returncode != 0:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    for lib, o in ((LIB, objs), (PROBE_LIB, probe_objs)):
        tmp = lib + ".tmp"
        cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + o
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
