"""Host compiler (fpe_compile through the C-ABI) against the oracle's own,
independent tree builder, and the boundary's error behaviour.  No GPU."""
import json
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import fpe_inputs
import paper_1307_5655_amd as fpe
from oracle import schemes, tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SCHEMES = {"direct": schemes.direct, "horner": schemes.horner, "estrin": schemes.estrin,
                  "balanced": schemes.balanced, "balanced_floor": schemes.balanced_literal}


def lib_tree(terms, scheme, domain=fpe.F64):
    ex = np.array([m for m, _ in terms], dtype=np.int32)
    co = np.array([c for _, c in terms], dtype=np.float64)
    return fpe.Tree(ex, co, scheme, domain)


def compare(terms, scheme):
    t = lib_tree(terms, scheme)
    nodes = t.nodes()
    exps = t.node_exps()
    o = tree.build_tree(terms, ORACLE_SCHEMES[scheme])
    assert len(o) == len(nodes)
    lh = tree.lazy_heights(o)
    ss = tree.safe_slots(o)
    for i, on in enumerate(o):
        assert tuple(exps[i]) == on.exps
        p = nodes["parent"][i]
        if on.parent is None:
            assert p == -1 and nodes["flags"][i] & fpe.NODE_ROOT
        else:
            assert p == on.parent.index
            first = on.parent.children[0] is on
            assert bool(nodes["flags"][i] & fpe.NODE_FIRST_CHILD) == first
        assert bool(nodes["flags"][i] & fpe.NODE_LEAF) == (not on.children)
        assert bool(nodes["flags"][i] & fpe.NODE_JUNCTION) == on.junction
        nz = [(j, e) for j, e in enumerate(on.pdeg) if e]
        if nz:
            assert (nodes["var"][i], nodes["pdeg"][i]) == nz[0]
        else:
            assert nodes["pdeg"][i] == 0
        assert nodes["slot"][i] == ss[i]
        assert nodes["lazy_height"][i] == lh[i]
        # subtree = [sub_begin, i]
        lo = i
        stack = [on]
        while stack:
            n = stack.pop()
            lo = min(lo, n.index)
            stack.extend(n.children)
        assert nodes["sub_begin"][i] == lo
    return t


@pytest.mark.parametrize("scheme", ["direct", "horner", "estrin", "balanced", "balanced_floor"])
def test_worked_example_matches_golden(scheme):
    with open(os.path.join(ROOT, "tests", "golden", "worked_example.json")) as f:
        g = json.load(f)
    c = g["coeffs_by_exponent"]
    terms = [((e,), float(v)) for e, v in enumerate(c) if v]
    t = compare(terms, scheme)
    if scheme in g["children_by_exponent"]:
        nodes = t.nodes()
        exps = t.node_exps()[:, 0]
        ch = {}
        for i, p in enumerate(nodes["parent"]):
            if p >= 0:
                ch.setdefault(str(exps[p]), []).append(int(exps[i]))
        assert ch == g["children_by_exponent"][scheme]


poly_uni = st.dictionaries(st.integers(0, 300), st.integers(-9, 9).filter(lambda v: v != 0),
                           min_size=1, max_size=80)


@settings(max_examples=80, deadline=None)
@given(poly_uni, st.sampled_from(["direct", "horner", "estrin", "balanced", "balanced_floor"]))
def test_univariate_trees_match_oracle(d, scheme):
    compare([((e,), float(c)) for e, c in d.items()], scheme)


poly_multi = st.integers(1, 4).flatmap(lambda v: st.dictionaries(
    st.tuples(*[st.integers(0, 7)] * v), st.integers(-5, 5).filter(lambda c: c != 0),
    min_size=1, max_size=60))


@settings(max_examples=80, deadline=None)
@given(poly_multi, st.sampled_from(["horner", "estrin", "balanced", "direct"]))
def test_multivariate_trees_match_oracle(d, scheme):
    compare([(m, float(c)) for m, c in d.items()], scheme)


@pytest.mark.parametrize("n", [1023, 3000, 5000])
def test_config_sized_trees_match_oracle(n):
    import fpe_inputs
    inp = fpe_inputs.sparse_uni(n, npts=1)
    ex, co = inp.terms()
    for scheme in ["horner", "estrin", "balanced"]:
        compare([((int(e[0]),), float(c)) for e, c in zip(ex, co)], scheme)


def test_trivariate_dense_shape():
    import fpe_inputs
    inp = fpe_inputs.trivariate(npts=1)
    t = fpe.Tree(inp.exps, inp.coeffs, "estrin", fpe.MODP, fpe.P61)
    assert t.info.n_nodes == 12341 and t.info.n_terms == 12341   # no junction
    nodes = t.nodes()
    assert not np.any(nodes["flags"] & fpe.NODE_JUNCTION)


def test_threshold_and_table_schemes():
    rng = np.random.default_rng(4)
    c = rng.uniform(-1, 1, 200)
    ex = np.arange(200, dtype=np.int32).reshape(-1, 1)
    t = fpe.Tree(ex, c, "threshold", threshold=10)
    o = tree.build_tree(tree.dense_terms(c), schemes.threshold(10))
    assert [tuple(r) for r in t.node_exps()] == [n.exps for n in o]
    tab = [0] + [max(1, k // 3) for k in range(1, 400)]
    t = fpe.Tree(ex, c, "table", table=tab)
    o = tree.build_tree(tree.dense_terms(c), schemes.table(tab))
    par = t.nodes()["parent"]
    assert [p for p in par] == [n.parent.index if n.parent else -1 for n in o]


def test_errors_are_status_codes():
    ex = np.array([[0], [1]], dtype=np.int32)
    with pytest.raises(fpe.FpeError) as e:
        fpe.Tree(np.array([[1], [1]], dtype=np.int32), [1.0, 2.0], "horner")
    assert e.value.status == -1 and "duplicate" in str(e.value)
    with pytest.raises(fpe.FpeError):
        fpe.Tree(ex, [0.0, 0.0], "horner")                      # zero polynomial
    with pytest.raises(fpe.FpeError):
        fpe.Tree(ex, [1.0, float("nan")], "horner")             # non-finite
    with pytest.raises(fpe.FpeError):
        fpe.Tree(np.array([[-1]], dtype=np.int32), [1.0], "horner")
    with pytest.raises(fpe.FpeError):
        fpe.Tree(ex, [1, fpe.P61], "horner", fpe.MODP, fpe.P61)  # residue >= p
    with pytest.raises(fpe.FpeError) as e:
        fpe.Tree(ex, [1, 2], "horner", fpe.MODP, 1000003)
    assert e.value.status == -5
    with pytest.raises(fpe.FpeError):
        fpe.Tree(np.zeros((2, 9), dtype=np.int32), [1.0, 2.0], "horner")   # nvars > 8
    with pytest.raises(fpe.FpeError) as e:
        fpe.Tree(np.arange(20, dtype=np.int32).reshape(-1, 1), np.ones(20), "table",
                 table=[0, 1, 2, 5])                             # f(3) = 5 > 3
    assert "outside" in str(e.value)
    with pytest.raises(fpe.FpeError):
        fpe.Tree(np.arange(20, dtype=np.int32).reshape(-1, 1), np.ones(20), "table",
                 table=[0, 1, 1])                                # f(19) missing
    t = fpe.Tree(ex, [1.0, 2.0], "horner")
    with pytest.raises(fpe.FpeError):                            # not uploaded
        import ctypes
        fpe._check(fpe.lib.fpe_evaluate(t.handle, None, 1, None, None, None))


def test_zero_coefficients_dropped_and_single_term():
    t = fpe.Tree(np.array([[5], [3], [0]], dtype=np.int32), [2.0, 0.0, 0.0], "estrin")
    nodes = t.nodes()
    assert len(nodes) == 1 and nodes["pdeg"][0] == 5 and nodes["flags"][0] & fpe.NODE_ROOT


def test_serialize_roundtrip():
    rng = np.random.default_rng(6)
    ex = np.unique(rng.integers(0, 9, size=(50, 3)), axis=0).astype(np.int32)
    co = rng.uniform(-1, 1, len(ex))
    t = fpe.Tree(ex, co, "balanced", fpe.F32C)
    blob = t.serialize()
    t2 = fpe.Tree.deserialize(blob)
    assert t2.domain == fpe.F32C and t2.batch == 1
    assert t2.serialize() == blob
    assert np.array_equal(t2.nodes(), t.nodes())
    with pytest.raises(fpe.FpeError):
        fpe.Tree.deserialize(blob[:-3])
    bad = bytearray(blob)
    bad[0] ^= 0xFF
    with pytest.raises(fpe.FpeError):
        fpe.Tree.deserialize(bytes(bad))


def _op_arrays(blob, n):
    """Byte offsets of the FP64 and FP32 op records (n of each, 32 bytes) in a
    serialised compensated-FP32 tree: each array follows its u64 length, the
    FP32 one right after the FP64 one, and both carry the same info word at
    bytes 16-19 of each record (the deg words at 20-23 differ where the
    double-float walk's deeper LDS tier changes an entry's power class)."""
    u64 = lambda q: int.from_bytes(blob[q:q + 8], "little")
    hits = []
    for q in range(0, len(blob) - 16 - 64 * n):
        if u64(q) == n and u64(q + 8 + 32 * n) == n:
            a, b = q + 8, q + 16 + 32 * n
            if all(blob[a + 32 * k + 16:a + 32 * k + 20] == blob[b + 32 * k + 16:b + 32 * k + 20] for k in range(n)):
                hits.append((a, b))
    assert len(hits) == 1
    return hits[0]


def test_deserialize_checks_the_dispatch_codes():
    """A serialised program whose dispatch code disagrees with its record (the
    code selects the kernel's load of the power), or whose FP32 records differ
    from the FP64 ones, is refused."""
    inp = fpe_inputs.sparse_uni(3000, npts=1)
    e = np.nonzero(inp.coeffs)[0]
    t = fpe.Tree(e.astype(np.int32).reshape(-1, 1), inp.coeffs[e], "balanced", fpe.F32C)
    assert t.info.n_table > 8          # entries in registers, in the LDS tier and beyond it
    blob = t.serialize()
    a, b = _op_arrays(blob, len(t.nodes()))
    fpe.Tree.deserialize(blob)
    codes = [int.from_bytes(blob[a + 32 * k + 20:a + 32 * k + 24], "little") >> 26 for k in range(len(t.nodes()))]
    codes32 = [int.from_bytes(blob[b + 32 * k + 20:b + 32 * k + 24], "little") >> 26 for k in range(len(t.nodes()))]
    assert {4, 6} <= set(codes)        # power classes: LDS-tier and private entries
    # the FP64 records put entries 4-7 in the LDS tier, the FP32 ones 4-10
    assert t.info.n_table > 11 and {4, 6} <= set(codes32)
    moved = [k for k in range(len(codes)) if codes[k] == 6 and codes32[k] == 4]
    assert moved and all(codes32[k] == codes[k] for k in range(len(codes)) if codes[k] != 6)
    k = codes.index(6)
    for arrays in ((a, b), (b,)):
        bad = bytearray(blob)
        for base in arrays:            # private-table class -> LDS-tier class
            w = int.from_bytes(bad[base + 32 * k + 20:base + 32 * k + 24], "little")
            bad[base + 32 * k + 20:base + 32 * k + 24] = (w ^ (2 << 26)).to_bytes(4, "little")
        with pytest.raises(fpe.FpeError):
            fpe.Tree.deserialize(bytes(bad))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "fpe.h")).read()
    names = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(fpe_\w+)\s*\(", hdr, flags=re.M))
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(fpe.lib, n), n
    assert set(fpe.EXPORTED) <= names
    assert fpe.lib.fpe_version().decode().startswith("fpe")


def test_package_binds_to_one_hip_runtime():
    # Importing the package before torch must not load a second HIP runtime
    # next to the one PyTorch brings (that second copy finds no device once
    # PyTorch's has opened it).  Checked in a fresh process.
    import subprocess
    import sys
    code = ("import paper_1307_5655_amd\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced", "direct"])
def test_interval_trees_share_the_shape_and_take_no_power_products(scheme):
    """An interval tree has the FP64 tree's nodes; its powers come from the
    table or are computed on the fly, never as products of two entries, and
    every MUL step of its chain names its variable and degree parity."""
    g = np.random.default_rng(5)
    c = g.uniform(-1, 1, 700)
    c[g.choice(699, 70, replace=False)] = 0.0
    e = np.nonzero(c)[0].astype(np.int32).reshape(-1, 1)
    t64 = fpe.Tree(e, c[e[:, 0]], scheme, fpe.F64)
    tiv = fpe.Tree(e, c[e[:, 0]], scheme, fpe.IVAL)
    assert np.array_equal(t64.nodes(), tiv.nodes())
    assert tiv.info.n_pair_ops == 0
    assert tiv.info.walk_depth == t64.info.walk_depth
    assert tiv.info.n_table <= 48
    back = fpe.Tree.deserialize(tiv.serialize())
    assert np.array_equal(back.nodes(), tiv.nodes())
    assert back.domain == fpe.IVAL


def test_tree_info_reports_domain_modulus_and_batch():
    e = np.array([[0], [3], [5]], dtype=np.int32)
    t = fpe.Tree(e, np.array([[1, 2, 3], [4, 5, 6]], dtype=np.uint64), "estrin", fpe.MODP, fpe.P31)
    assert (t.info.domain, t.info.modulus, t.info.batch) == (fpe.MODP, fpe.P31, 2)
    back = fpe.Tree.deserialize(t.serialize())
    assert (back.domain, back.modulus, back.batch) == (fpe.MODP, fpe.P31, 2)


def _hdr_field(blob, off, fmt):
    import struct
    return struct.unpack_from(fmt, blob, off)[0]


def _set_field(blob, off, fmt, v):
    import struct
    b = bytearray(blob)
    struct.pack_into(fmt, b, off, v)
    return bytes(b)


# byte offsets of the serialised header: magic, nvars, domain, modulus,
# batch, n_terms, n_table, n_powers, depth, max_slot, max_lh, n_offtable, n_pairs
_OFF_BATCH, _OFF_NOFFT, _OFF_NPAIRS, _OFF_MOD, _OFF_DOMAIN = 24, 60, 64, 16, 12


def test_deserialize_rejects_corrupt_counts_and_batch():
    """Fields that select kernels or drive device indexing are checked against
    the data: the on-the-fly power count (a kernel without that path would read
    a table entry that does not exist), the batch and the coefficient rows of a
    composition tree, the modulus, and the node indices of a composition
    program.  Per-kind step counts are recomputed."""
    # a direct-scheme tree with powers beyond the table
    ex = np.sort(np.random.default_rng(4).choice(100_000, 300, replace=False)).astype(np.int32).reshape(-1, 1)
    t = fpe.Tree(ex, np.linspace(-1, 1, 300), "direct", fpe.F64)
    assert t.info.n_offtable > 0
    blob = t.serialize()
    assert _hdr_field(blob, _OFF_NOFFT, "<i") == t.info.n_offtable
    with pytest.raises(fpe.FpeError):
        fpe.Tree.deserialize(_set_field(blob, _OFF_NOFFT, "<i", 0))
    with pytest.raises(fpe.FpeError):
        fpe.Tree.deserialize(_set_field(blob, _OFF_NPAIRS, "<i", t.info.n_pair_ops + 1))
    back = fpe.Tree.deserialize(blob)
    assert list(back.info.n_ops_kind) == list(t.info.n_ops_kind)
    assert back.info.n_offtable == t.info.n_offtable
    # a batch of 4 rows mod 2^31 - 1 whose batch field claims 10^6
    rows = np.random.default_rng(5).integers(0, fpe.P31, size=(4, 32)).astype(np.uint64)
    tc = fpe.Tree(np.arange(32, dtype=np.int32).reshape(-1, 1), rows, "balanced", fpe.MODP, fpe.P31)
    blob = tc.serialize()
    assert _hdr_field(blob, _OFF_BATCH, "<q") == 4
    for bad in (10 ** 6, 0, -3, 5):
        with pytest.raises(fpe.FpeError):
            fpe.Tree.deserialize(_set_field(blob, _OFF_BATCH, "<q", bad))
    # the modulus must be one the kernels implement, and hold every residue
    with pytest.raises(fpe.FpeError):
        fpe.Tree.deserialize(_set_field(blob, _OFF_MOD, "<Q", 1000))
    # an FP64 tree claiming to be a batch composition tree
    with pytest.raises(fpe.FpeError):
        fpe.Tree.deserialize(_set_field(t.serialize(), _OFF_DOMAIN, "<i", fpe.MODP))
    assert fpe.Tree.deserialize(blob).info.batch == 4


def test_probe_library_exports_its_header():
    import ctypes
    hdr = open(os.path.join(ROOT, "include", "fpe_probe.h")).read()
    names = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(fpe_\w+)\s*\(", hdr, flags=re.M))
    assert names == {"fpe_probe_launch"}
    L = ctypes.CDLL(os.path.join(ROOT, "paper_1307_5655_amd", "libfpe_probe.so"))
    for n in names:
        assert hasattr(L, n), n
