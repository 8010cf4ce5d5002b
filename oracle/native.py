"""ctypes loader for the plain C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build() -> str:
    subprocess.run(["sh", os.path.join(_HERE, "build_native.sh")], check=True)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_horner_f64.argtypes = [P, i64, P, i64, P, ctypes.c_int]
        L.orc_dd_horner.argtypes = [P, i64, P, i64, P, P]
        L.orc_ptilde.argtypes = [P, i64, P, i64, P]
        L.orc_modp_eval.argtypes = [ctypes.c_int32, i64, P, P, ctypes.c_uint64, P, i64, P]
        L.orc_compose_modp.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, i64, ctypes.c_uint64, P]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def horner_f64(coeffs, xs, use_fma: bool) -> np.ndarray:
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    x = np.ascontiguousarray(xs, dtype=np.float64)
    y = np.empty_like(x)
    lib().orc_horner_f64(_p(c), len(c) - 1, _p(x), len(x), _p(y), int(use_fma))
    return y


def dd_horner(coeffs, xs):
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    x = np.ascontiguousarray(xs, dtype=np.float64)
    hi = np.empty_like(x)
    lo = np.empty_like(x)
    lib().orc_dd_horner(_p(c), len(c) - 1, _p(x), len(x), _p(hi), _p(lo))
    return hi, lo


def dd_value(coeffs, xs) -> np.ndarray:
    hi, lo = dd_horner(coeffs, xs)
    return hi + lo


def ptilde(coeffs, xs) -> np.ndarray:
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    x = np.ascontiguousarray(xs, dtype=np.float64)
    y = np.empty_like(x)
    lib().orc_ptilde(_p(c), len(c) - 1, _p(x), len(x), _p(y))
    return y


def modp_eval(exps, coeffs, p: int, pts) -> np.ndarray:
    e = np.ascontiguousarray(exps, dtype=np.int32)
    c = np.ascontiguousarray(coeffs, dtype=np.uint64)
    x = np.ascontiguousarray(pts, dtype=np.uint64)
    nv, npts = x.shape
    out = np.empty(npts, dtype=np.uint64)
    lib().orc_modp_eval(nv, len(c), _p(e), _p(c), p, _p(x), npts, _p(out))
    return out


def compose_modp(pc, qc, p: int) -> np.ndarray:
    P = np.ascontiguousarray(pc, dtype=np.uint32)
    Q = np.ascontiguousarray(qc, dtype=np.uint32)
    b, dp1 = P.shape
    dq1 = Q.shape[1]
    out = np.empty((b, (dp1 - 1) * (dq1 - 1) + 1), dtype=np.uint32)
    lib().orc_compose_modp(_p(P), dp1 - 1, _p(Q), dq1 - 1, b, p, _p(out))
    return out
