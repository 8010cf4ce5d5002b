"""fpe: fast polynomial evaluation through evaluation trees on MI355X (gfx950).

Thin ctypes binding over libfpe.so (include/fpe.h).  Argument marshalling
only: every step of compile, evaluate and compose runs in the native library
(host C++ for the tree compiler, HIP kernels for everything per point).
PyTorch provides device memory and streams.  Importing this package fails
loudly when libfpe.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfpe.so")

F64, F32C, MODP, IVAL, BIGINT = 0, 1, 2, 3, 4
DIRECT, HORNER, ESTRIN, BALANCED, BALANCED_FLOOR, THRESHOLD, TABLE = range(7)
SCHEMES = {"direct": DIRECT, "horner": HORNER, "estrin": ESTRIN, "balanced": BALANCED,
           "balanced_floor": BALANCED_FLOOR, "threshold": THRESHOLD, "table": TABLE}
P61 = (1 << 61) - 1
P31 = (1 << 31) - 1

NODE_LEAF, NODE_FIRST_CHILD, NODE_JUNCTION, NODE_ROOT = 1, 2, 4, 8


class FpeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fpe status {status}: {msg}")
        self.status = status


class _Scheme(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("threshold", ctypes.c_int32),
                ("table", ctypes.POINTER(ctypes.c_int32)), ("table_len", ctypes.c_int32)]


class Node(ctypes.Structure):
    _fields_ = [("coef", ctypes.c_uint64), ("pdeg", ctypes.c_int32), ("var", ctypes.c_uint8),
                ("slot", ctypes.c_uint8), ("lazy_height", ctypes.c_uint8), ("flags", ctypes.c_uint8),
                ("parent", ctypes.c_int32), ("sub_begin", ctypes.c_int32)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_terms", ctypes.c_int64), ("nvars", ctypes.c_int32),
                ("max_slot", ctypes.c_int32), ("max_lazy_height", ctypes.c_int32),
                ("walk_depth", ctypes.c_int32), ("n_powers", ctypes.c_int32),
                ("n_table", ctypes.c_int32), ("n_chain", ctypes.c_int32),
                ("n_offtable", ctypes.c_int32), ("n_pair_ops", ctypes.c_int32),
                ("n_ops_kind", ctypes.c_int32 * 5), ("domain", ctypes.c_int32),
                ("modulus", ctypes.c_uint64), ("batch", ctypes.c_int64)]


class EvalOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("force", ctypes.c_int32),
                ("points_per_lane", ctypes.c_int32), ("cond_out", ctypes.c_void_p),
                ("flags_out", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("nfallback_out", ctypes.c_void_p),
                ("ev_walk_begin", ctypes.c_void_p), ("ev_walk_end", ctypes.c_void_p),
                ("bound_out", ctypes.c_void_p), ("path", ctypes.c_int32)]


# fpe_eval_opts.path: the tree walk, the library's choice, the term-parallel few-point path
PATHS = {"walk": 0, "auto": 1, "terms": 2}


REQ_EVALUATE, REQ_COMPOSE = 0, 1


class Request(ctypes.Structure):
    _fields_ = [("tree", ctypes.c_void_p), ("pts", ctypes.c_void_p * 8), ("npts", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("cond_out", ctypes.c_void_p), ("tol", ctypes.c_double),
                ("domain", ctypes.c_int32), ("kind", ctypes.c_int32), ("q", ctypes.c_void_p),
                ("dq", ctypes.c_int32),
                ("path", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("term_evals", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("fallback_frac", ctypes.c_double), ("hbm_in_use", ctypes.c_int64),
                ("compose_instances", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_1307_5655_amd/build.py")
    # Device buffers and stream handles come from PyTorch, so the library must
    # bind to the HIP runtime PyTorch loaded: import it first, so that the
    # dynamic loader resolves libfpe's libamdhip64 to that copy instead of
    # loading a second runtime (which then finds no device of its own).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "fpe_last_error": ([], ctypes.c_char_p),
        "fpe_version": ([], ctypes.c_char_p),
        "fpe_compile": ([i32, i64, P, P, i64, i32, u64, ctypes.POINTER(_Scheme), ctypes.POINTER(P)], i32),
        "fpe_tree_free": ([P], None),
        "fpe_tree_nodes": ([P, ctypes.POINTER(ctypes.POINTER(Node)), ctypes.POINTER(i64),
                            ctypes.POINTER(i32)], i32),
        "fpe_tree_get_info": ([P, ctypes.POINTER(TreeInfo)], i32),
        "fpe_tree_node_exps": ([P, i64, P], i32),
        "fpe_tree_device_bytes": ([P], sz),
        "fpe_tree_upload": ([P, P, sz, P], i32),
        "fpe_tree_serialize": ([P, P, ctypes.POINTER(sz)], i32),
        "fpe_tree_deserialize": ([P, sz, ctypes.POINTER(P)], i32),
        "fpe_workspace_bytes": ([P, i64], sz),
        "fpe_evaluate": ([P, P, i64, P, ctypes.POINTER(EvalOpts), P], i32),
        "fpe_evaluate_noalloc": ([P, P, i64, P, ctypes.POINTER(EvalOpts), P], i32),
        "fpe_compose_workspace_bytes": ([P, i32], sz),
        "fpe_compose": ([P, P, i32, P, P, sz, P], i32),
        "fpe_compose_ex_workspace_bytes": ([P, i32, i32], sz),
        "fpe_eval_path": ([P, i64], i32),
        "fpe_compose_ex": ([P, P, i32, P, i32, P, sz, P], i32),
        "fpe_server_workspace_bytes": ([sz], sz),
        "fpe_server_create": ([P, sz, sz, i32, P, ctypes.POINTER(P)], i32),
        "fpe_server_submit": ([P, ctypes.POINTER(Request), ctypes.POINTER(u64)], i32),
        "fpe_server_poll": ([P, u64, ctypes.POINTER(i32)], i32),
        "fpe_server_wait": ([P, u64], i32),
        "fpe_server_drain": ([P], i32),
        "fpe_server_stats": ([P, ctypes.POINTER(Stats)], i32),
        "fpe_server_destroy": ([P], None),
        "fpe_bigint_out_limbs": ([P, i32], i32),
        "fpe_bigint_workspace_bytes": ([P, i32, i64], sz),
        "fpe_eval_bigint": ([P, P, i32, i64, P, i32, P, sz, P], i32),
        "fpe_bigint_status": ([P, P], i32),
        "fpe_bigpoint_out_limbs": ([P, i32], i64),
        "fpe_bigpoint_workspace_bytes": ([P, i32], sz),
        "fpe_eval_bigpoint": ([P, P, i32, P, i64, P, sz, P], i32),
        "fpe_compose_bigint_coef_limbs": ([P, P, i32], i32),
        "fpe_compose_bigint_out_limbs": ([P, P, i32], i64),
        "fpe_compose_bigint_workspace_bytes": ([P, P, i32], sz),
        "fpe_compose_bigint": ([P, P, i32, P, i64, P, sz, P], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()

EXPORTED = ["fpe_last_error", "fpe_version", "fpe_compile", "fpe_tree_free", "fpe_tree_nodes",
            "fpe_tree_get_info", "fpe_tree_node_exps", "fpe_tree_device_bytes", "fpe_tree_upload",
            "fpe_tree_serialize", "fpe_tree_deserialize", "fpe_workspace_bytes", "fpe_evaluate",
            "fpe_evaluate_noalloc", "fpe_eval_path",
            "fpe_compose_workspace_bytes", "fpe_compose", "fpe_compose_ex_workspace_bytes", "fpe_compose_ex",
            "fpe_server_workspace_bytes", "fpe_server_create",
            "fpe_server_submit",
            "fpe_server_poll", "fpe_server_wait", "fpe_server_drain", "fpe_server_stats",
            "fpe_server_destroy", "fpe_bigint_out_limbs", "fpe_bigint_workspace_bytes", "fpe_eval_bigint",
            "fpe_bigint_status", "fpe_bigpoint_out_limbs", "fpe_bigpoint_workspace_bytes", "fpe_eval_bigpoint"]


def _check(st: int):
    if st != 0:
        raise FpeError(st, (lib.fpe_last_error() or b"").decode())


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _scheme(scheme, threshold: int = 10, table=None):
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    s = _Scheme(scheme, threshold, None, 0)
    keep = None
    if scheme == TABLE:
        keep = np.ascontiguousarray(table, dtype=np.int32)
        s.table = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        s.table_len = len(keep)
    return s, keep


class Tree:
    """A compiled evaluation tree (fpe_compile) and its device image."""

    def __init__(self, exps, coeffs, scheme="balanced", domain=F64, modulus=0, threshold=10,
                 table=None):
        exps = np.ascontiguousarray(np.asarray(exps, dtype=np.int32))
        if exps.ndim == 1:
            exps = exps.reshape(-1, 1)
        nterms, nvars = exps.shape
        if domain in (MODP, BIGINT):
            c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint64))
            batch = 1 if c.ndim == 1 else c.shape[0]
            c = c.reshape(batch, nterms)
        else:
            c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
            batch = 1
        sch, keep = _scheme(scheme, threshold, table)
        h = ctypes.c_void_p()
        _check(lib.fpe_compile(nvars, nterms, exps.ctypes.data_as(ctypes.c_void_p),
                               c.ctypes.data_as(ctypes.c_void_p), batch, domain, modulus,
                               ctypes.byref(sch), ctypes.byref(h)))
        self._h = h
        self.nvars, self.domain, self.modulus, self.batch = nvars, domain, modulus, batch
        self._dev = None
        info = TreeInfo()
        _check(lib.fpe_tree_get_info(self._h, ctypes.byref(info)))
        self.info = info

    @classmethod
    def _from_handle(cls, h):
        self = cls.__new__(cls)
        self._h = h
        info = TreeInfo()
        _check(lib.fpe_tree_get_info(h, ctypes.byref(info)))
        self.info = info
        self.nvars, self.domain, self.modulus, self.batch = info.nvars, info.domain, info.modulus, info.batch
        self._dev = None
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and lib is not None:   # lib is None while the interpreter shuts down
            lib.fpe_tree_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def nodes(self):
        """The node array as a structured numpy array (copy)."""
        p = ctypes.POINTER(Node)()
        n = ctypes.c_int64()
        ms = ctypes.c_int32()
        _check(lib.fpe_tree_nodes(self._h, ctypes.byref(p), ctypes.byref(n), ctypes.byref(ms)))
        dt = np.dtype([("coef", "<u8"), ("pdeg", "<i4"), ("var", "u1"), ("slot", "u1"),
                       ("lazy_height", "u1"), ("flags", "u1"), ("parent", "<i4"), ("sub_begin", "<i4")])
        buf = ctypes.string_at(p, n.value * ctypes.sizeof(Node))
        return np.frombuffer(buf, dtype=dt).copy()

    def node_exps(self):
        n = self.info.n_nodes
        out = np.empty((n, self.nvars), dtype=np.int32)
        row = np.empty(self.nvars, dtype=np.int32)
        for i in range(n):
            _check(lib.fpe_tree_node_exps(self._h, i, row.ctypes.data_as(ctypes.c_void_p)))
            out[i] = row
        return out

    def device_bytes(self) -> int:
        return int(lib.fpe_tree_device_bytes(self._h))

    def upload(self, device="cuda", stream=None):
        import torch
        nb = self.device_bytes()
        buf = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + nb]
        _check(lib.fpe_tree_upload(self._h, ctypes.c_void_p(view.data_ptr()), nb, _stream_ptr(stream)))
        self._dev = buf          # keeps the device image alive
        return self

    def serialize(self) -> bytes:
        n = ctypes.c_size_t(0)
        _check(lib.fpe_tree_serialize(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib.fpe_tree_serialize(self._h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    @classmethod
    def deserialize(cls, data: bytes):
        """A tree from ``serialize()``; its domain, modulus and batch come from the data."""
        h = ctypes.c_void_p()
        _check(lib.fpe_tree_deserialize(data, len(data), ctypes.byref(h)))
        return cls._from_handle(h)


def eval_path(tree: Tree, npts: int) -> str:
    """The path fpe_evaluate takes with path="auto" (fpe_eval_path): "walk" or "terms"."""
    return {1: "walk", 2: "terms"}[int(lib.fpe_eval_path(tree.handle, npts))]


def workspace_bytes(tree: Tree, npts: int) -> int:
    return int(lib.fpe_workspace_bytes(tree.handle, npts))


def evaluate(tree: Tree, pts, out=None, tol: float = 1e-12, force: int = 0, cond_out=None,
             flags_out=None, workspace=None, nfallback_out=None, stream=None, events=None,
             points_per_lane: int = 0, bound_out=None, path="walk"):
    """Evaluate ``tree`` at device points ``pts`` (list of tensors, one per
    variable: 1-D float64, or uint64 residues stored as int64 for FPE_MODP;
    for FPE_IVAL [npts, 2] float64 intervals (lo, hi), and the result is
    [npts, 2] enclosures).  ``path`` (FPE_F64 / FPE_MODP): "walk" (default),
    "auto" (the library's cost model) or "terms" (fpe_eval_opts.path)."""
    import torch
    if tree._dev is None:
        raise FpeError(-1, "tree is not uploaded")
    pts = list(pts) if isinstance(pts, (list, tuple)) else [pts]
    if len(pts) != tree.nvars:
        raise FpeError(-1, f"{tree.nvars} point arrays expected, {len(pts)} given")
    npts = pts[0].shape[0] if tree.domain == IVAL else pts[0].numel()
    # the library takes raw pointers: check the sizes it will read and write
    shape = (npts, 2) if tree.domain == IVAL else (npts,)
    for p in pts:
        if tuple(p.shape) != shape or not p.is_contiguous() or p.element_size() != 8:
            raise FpeError(-1, f"point arrays must be contiguous 8-byte tensors of shape {shape}")
    if out is None:
        dt = torch.int64 if tree.domain == MODP else torch.float64
        out = torch.empty(shape, dtype=dt, device=pts[0].device)
    elif out.numel() < (2 * npts if tree.domain == IVAL else npts) or not out.is_contiguous() \
            or out.element_size() != 8:
        raise FpeError(-1, "output must be a contiguous 8-byte tensor with a value (or interval) per point")
    arr = (ctypes.c_void_p * 8)(*[p.data_ptr() for p in pts])
    opts = EvalOpts(tol, force, points_per_lane, cond_out.data_ptr() if cond_out is not None else None,
                    flags_out.data_ptr() if flags_out is not None else None, None, 0,
                    nfallback_out.data_ptr() if nfallback_out is not None else None)
    if bound_out is not None:
        if bound_out.numel() < npts or not bound_out.is_contiguous() or bound_out.element_size() != 8:
            raise FpeError(-1, "bound_out must be a contiguous float64 tensor with a value per point")
        opts.bound_out = bound_out.data_ptr()
    opts.path = PATHS.get(path, path)
    if events is not None:
        # raw hipEvent_t handles (ctypes.c_void_p or int)
        opts.ev_walk_begin = getattr(events[0], "value", events[0])
        opts.ev_walk_end = getattr(events[1], "value", events[1])
    if tree.domain == F32C:
        need = workspace_bytes(tree, npts)
        if workspace is None:
            workspace = torch.empty(need + 256, dtype=torch.uint8, device=pts[0].device)
        off = (-workspace.data_ptr()) % 256
        opts.workspace = workspace.data_ptr() + off
        opts.workspace_bytes = workspace.numel() - off
    _check(lib.fpe_evaluate(tree.handle, arr, npts, ctypes.c_void_p(out.data_ptr()),
                            ctypes.byref(opts), _stream_ptr(stream)))
    return out


NOALLOC_MAX_POINTS = 1 << 22


def evaluate_noalloc(tree: Tree, pts, out, tol: float = 1e-12, force: int = 0, cond_out=None,
                     flags_out=None, nfallback_out=None, stream=None):
    """fpe_evaluate_noalloc: like ``evaluate`` with a caller-given ``out``, but
    the compensated form's scratch is the library's static device array
    (nothing is allocated by this call, here or in the library)."""
    if tree._dev is None:
        raise FpeError(-1, "tree is not uploaded")
    pts = list(pts) if isinstance(pts, (list, tuple)) else [pts]
    if len(pts) != tree.nvars:
        raise FpeError(-1, f"{tree.nvars} point arrays expected, {len(pts)} given")
    npts = pts[0].shape[0] if tree.domain == IVAL else pts[0].numel()
    shape = (npts, 2) if tree.domain == IVAL else (npts,)
    for p in pts:
        if tuple(p.shape) != shape or not p.is_contiguous() or p.element_size() != 8:
            raise FpeError(-1, f"point arrays must be contiguous 8-byte tensors of shape {shape}")
    if out.numel() < (2 * npts if tree.domain == IVAL else npts) or not out.is_contiguous() \
            or out.element_size() != 8:
        raise FpeError(-1, "output must be a contiguous 8-byte tensor with a value (or interval) per point")
    arr = (ctypes.c_void_p * 8)(*[p.data_ptr() for p in pts])
    opts = EvalOpts(tol, force, 0, cond_out.data_ptr() if cond_out is not None else None,
                    flags_out.data_ptr() if flags_out is not None else None, None, 0,
                    nfallback_out.data_ptr() if nfallback_out is not None else None)
    _check(lib.fpe_evaluate_noalloc(tree.handle, arr, npts, ctypes.c_void_p(out.data_ptr()),
                                    ctypes.byref(opts), _stream_ptr(stream)))
    return out


def eval_bigint(tree: Tree, x, lout=None, out=None, workspace=None, stream=None, check=True):
    """p(x_r) over the natural numbers for every point r: ``x`` is a device
    int32 tensor [batch, lx] of 16-bit limbs (least significant first); the
    result is [batch, lout] int32 limbs (values < 2^16).  With ``check`` the
    device overflow flag is read back (fpe_bigint_status, which waits for the
    stream) and a truncated result raises."""
    import torch
    if tree._dev is None:
        raise FpeError(-1, "tree is not uploaded")
    if x.dim() != 2 or not x.is_contiguous() or x.element_size() != 4:
        raise FpeError(-1, "x must be a contiguous 32-bit tensor [batch, lx]")
    batch, lx = x.shape
    if lout is None:
        lout = int(lib.fpe_bigint_out_limbs(tree.handle, lx))
    if out is None:
        out = torch.empty((batch, lout), dtype=torch.int32, device=x.device)
    elif tuple(out.shape) != (batch, lout) or not out.is_contiguous() or out.element_size() != 4:
        raise FpeError(-1, "out must be a contiguous 32-bit tensor [batch, lout]")
    need = int(lib.fpe_bigint_workspace_bytes(tree.handle, lout, batch))
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=x.device)
    off = (-workspace.data_ptr()) % 256
    _check(lib.fpe_eval_bigint(tree.handle, ctypes.c_void_p(x.data_ptr()), lx, batch,
                               ctypes.c_void_p(out.data_ptr()), lout, ctypes.c_void_p(workspace.data_ptr() + off),
                               workspace.numel() - off, _stream_ptr(stream)))
    if check:
        _check(lib.fpe_bigint_status(ctypes.c_void_p(workspace.data_ptr() + off), _stream_ptr(stream)))
    return out


PRODUCT_AUTO, PRODUCT_FUSED, PRODUCT_SCHOOLBOOK, PRODUCT_NTT, PRODUCT_MFMA = 0, 1, 2, 3, 4
PRODUCTS = {"auto": PRODUCT_AUTO, "fused": PRODUCT_FUSED, "schoolbook": PRODUCT_SCHOOLBOOK, "ntt": PRODUCT_NTT,
            "mfma": PRODUCT_MFMA}


def eval_bigpoint(tree: Tree, x, out=None, workspace=None, stream=None, check=True):
    """p(x) over the natural numbers at ONE big point: ``x`` is a device int32
    tensor [lx] of 16-bit limbs (least significant first); the result is a
    tensor [fpe_bigpoint_out_limbs] of int32 limbs (values < 2^16).  With
    ``check`` the overflow flag is read back (fpe_bigint_status, which waits
    for the stream)."""
    import torch
    if tree._dev is None:
        raise FpeError(-1, "tree is not uploaded")
    if x.dim() != 1 or not x.is_contiguous() or x.element_size() != 4:
        raise FpeError(-1, "x must be a contiguous 32-bit tensor [lx]")
    lx = x.numel()
    lout = int(lib.fpe_bigpoint_out_limbs(tree.handle, lx))
    if lout <= 0:
        raise FpeError(-5, (lib.fpe_last_error() or b"").decode() or "unsupported size")
    if out is None:
        out = torch.empty(lout, dtype=torch.int32, device=x.device)
    elif out.numel() < lout or not out.is_contiguous() or out.element_size() != 4:
        raise FpeError(-1, f"out must be a contiguous 32-bit tensor of at least {lout} limbs")
    need = int(lib.fpe_bigpoint_workspace_bytes(tree.handle, lx))
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=x.device)
    off = (-workspace.data_ptr()) % 256
    _check(lib.fpe_eval_bigpoint(tree.handle, ctypes.c_void_p(x.data_ptr()), lx, ctypes.c_void_p(out.data_ptr()),
                                 out.numel(), ctypes.c_void_p(workspace.data_ptr() + off), workspace.numel() - off,
                                 _stream_ptr(stream)))
    if check:
        _check(lib.fpe_bigint_status(ctypes.c_void_p(workspace.data_ptr() + off), _stream_ptr(stream)))
    return out


def _q_u64(q):
    import numpy as np
    return np.ascontiguousarray(np.asarray([int(c) for c in q], dtype=np.uint64))


def compose_bigint_workspace_bytes(tree: Tree, q) -> int:
    qa = _q_u64(q)
    return int(lib.fpe_compose_bigint_workspace_bytes(tree.handle, ctypes.c_void_p(qa.ctypes.data), len(qa) - 1))


def compose_bigint(tree: Tree, q, out=None, workspace=None, stream=None, check=True):
    """p(q(X)) over the natural numbers (fpe_compose_bigint): ``tree`` is an
    uploaded FPE_BIGINT tree, ``q`` the inner polynomial's coefficients
    (sequence of ints in [0, 2^64), q[0] first, at most 64).  Returns a device
    int32 tensor [deg p * dq + 1, lc]: row k holds the coefficient of X^k as
    16-bit limbs, least significant first.  With ``check`` the overflow flag
    is read back (fpe_bigint_status, which waits for the stream)."""
    import torch
    if tree._dev is None:
        raise FpeError(-1, "tree is not uploaded")
    qa = _q_u64(q)
    dq = len(qa) - 1
    qp = ctypes.c_void_p(qa.ctypes.data)
    lc = int(lib.fpe_compose_bigint_coef_limbs(tree.handle, qp, dq))
    if lc <= 0:
        raise FpeError(-5, "composition at one big point: unsupported size")
    nout = int(lib.fpe_compose_bigint_out_limbs(tree.handle, qp, dq))
    dev = tree._dev.device
    if out is None:
        out = torch.empty(nout, dtype=torch.int32, device=dev)
    elif out.numel() < nout or not out.is_contiguous() or out.element_size() != 4:
        raise FpeError(-1, f"out must be a contiguous 32-bit tensor of at least {nout} limbs")
    out = out.view(-1)
    need = int(lib.fpe_compose_bigint_workspace_bytes(tree.handle, qp, dq))
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-workspace.data_ptr()) % 256
    _check(lib.fpe_compose_bigint(tree.handle, qp, dq, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                  ctypes.c_void_p(workspace.data_ptr() + off), workspace.numel() - off,
                                  _stream_ptr(stream)))
    if check:
        _check(lib.fpe_bigint_status(ctypes.c_void_p(workspace.data_ptr() + off), _stream_ptr(stream)))
    return out[:nout].view(nout // lc, lc)


def compose_workspace_bytes(tree: Tree, dq: int, product=PRODUCT_AUTO) -> int:
    product = PRODUCTS.get(product, product)
    return int(lib.fpe_compose_ex_workspace_bytes(tree.handle, dq, product))


def compose(tree: Tree, q, out=None, workspace=None, stream=None, product=PRODUCT_AUTO):
    """p_r(q_r(x)) mod 2^31-1 for every instance r compiled into ``tree``;
    ``q`` is a device int32/uint32 tensor [batch, dq + 1]; ``product`` picks
    how the polynomial products are computed (fpe_compose_ex)."""
    import torch
    if tree._dev is None:
        raise FpeError(-1, "tree is not uploaded")
    product = PRODUCTS.get(product, product)
    batch, dq1 = q.shape
    dq = dq1 - 1
    dp = int(tree.node_exps().max())
    if batch != tree.batch or not q.is_contiguous() or q.element_size() != 4:
        raise FpeError(-1, "q must be a contiguous 32-bit tensor [batch, dq + 1]")
    if out is None:
        out = torch.empty((batch, dp * dq + 1), dtype=torch.int32, device=q.device)
    elif out.numel() < batch * (dp * dq + 1) or not out.is_contiguous() or out.element_size() != 4:
        raise FpeError(-1, "out must be a contiguous 32-bit tensor [batch, deg_p * dq + 1]")
    need = compose_workspace_bytes(tree, dq, product)
    if workspace is None:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=q.device)
    off = (-workspace.data_ptr()) % 256
    _check(lib.fpe_compose_ex(tree.handle, ctypes.c_void_p(q.data_ptr()), dq, ctypes.c_void_p(out.data_ptr()),
                              product, ctypes.c_void_p(workspace.data_ptr() + off), workspace.numel() - off,
                              _stream_ptr(stream)))
    return out


class Server:
    """Continuous-batching request loop (fpe_server_*).  Its device workspace
    (work tables and per-request scratch) is a torch tensor owned here."""

    def __init__(self, hbm_budget: int, max_inflight: int = 64, stream=None, device="cuda"):
        import torch
        nb = int(lib.fpe_server_workspace_bytes(hbm_budget))
        self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        off = (-self._ws.data_ptr()) % 256
        h = ctypes.c_void_p()
        _check(lib.fpe_server_create(ctypes.c_void_p(self._ws.data_ptr() + off), nb, hbm_budget, max_inflight,
                                     _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def submit(self, tree: Tree, pts, out, domain=F32C, tol=1e-12, cond_out=None, path="walk") -> int:
        """An evaluate request: FPE_F64 / FPE_F32C (float64 points and output)
        or FPE_MODP (residues as int64 tensors); ``path`` as in evaluate()
        (FPE_F64 / FPE_MODP)."""
        n = pts[0].numel()
        if len(pts) != tree.nvars or any(p.numel() != n or not p.is_contiguous() or p.element_size() != 8
                                         for p in pts) \
                or out.numel() < n or not out.is_contiguous() or out.element_size() != 8 \
                or (cond_out is not None and (cond_out.numel() < n or cond_out.element_size() != 4)):
            raise FpeError(-1, "one contiguous 8-byte point array per variable, all of one length, and outputs that long")
        r = Request()
        r.tree = tree.handle
        for j, p in enumerate(pts):
            r.pts[j] = p.data_ptr()
        r.npts = n
        r.out = out.data_ptr()
        r.cond_out = cond_out.data_ptr() if cond_out is not None else None
        r.tol = tol
        r.domain = domain
        r.kind = REQ_EVALUATE
        r.path = PATHS.get(path, path)
        t = ctypes.c_uint64()
        _check(lib.fpe_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def submit_compose(self, tree: Tree, q, out) -> int:
        """A compose request: p_r(q_r(x)) mod 2^31 - 1 for every instance of
        ``tree``; ``q`` is int32 [batch, dq + 1], ``out`` int32
        [batch, deg_p * dq + 1]."""
        batch, dq1 = q.shape
        dp = int(tree.node_exps().max())
        if batch != tree.batch or not q.is_contiguous() or q.element_size() != 4 or not out.is_contiguous() \
                or out.element_size() != 4 or out.numel() < batch * (dp * (dq1 - 1) + 1):
            raise FpeError(-1, "q must be [batch, dq + 1] and out [batch, deg_p * dq + 1], contiguous 32-bit")
        r = Request()
        r.tree = tree.handle
        r.out = out.data_ptr()
        r.domain = tree.domain
        r.kind = REQ_COMPOSE
        r.q = q.data_ptr()
        r.dq = dq1 - 1
        t = ctypes.c_uint64()
        _check(lib.fpe_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        _check(lib.fpe_server_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        _check(lib.fpe_server_wait(self._h, ticket))

    def drain(self):
        _check(lib.fpe_server_drain(self._h))

    def stats(self) -> Stats:
        s = Stats()
        _check(lib.fpe_server_stats(self._h, ctypes.byref(s)))
        return s

    def close(self):
        if getattr(self, "_h", None) and lib is not None:
            lib.fpe_server_destroy(self._h)
            self._h = None
        self._ws = None      # the workspace outlives the server

    def __del__(self):
        self.close()
