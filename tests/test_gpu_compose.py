"""GPU composition p(q(x)) mod 2^31 - 1 through the evaluation tree, bit-exact
against the oracle's schoolbook expansion; at full size every instance is
checked by Schwartz-Zippel evaluation at random points and a sample of
instances coefficient by coefficient."""
import numpy as np
import pytest
import torch

import fpe_inputs
import paper_1307_5655_amd as fpe
from oracle import compose as ocomp
from oracle import native

pytestmark = pytest.mark.gpu
P31 = fpe.P31


def say(msg):
    print(msg, flush=True)


def gpu_compose(P, Q, scheme, dev):
    b, dp1 = P.shape
    ex = np.arange(dp1, dtype=np.int32).reshape(-1, 1)
    t = fpe.Tree(ex, P.astype(np.uint64), scheme, fpe.MODP, P31).upload(dev)
    q = torch.from_numpy(np.ascontiguousarray(Q.astype(np.int32))).to(dev)
    out = fpe.compose(t, q)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_compose_small_batch_exact(dev, scheme):
    say(f"compose 48 x (255 o 15) {scheme}")
    inp = fpe_inputs.compose_batch(batch=48)
    got = gpu_compose(inp.p, inp.q, scheme, dev)
    want = native.compose_modp(inp.p, inp.q, P31)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dp,dq", [(1, 1), (7, 3), (20, 1), (33, 5), (64, 2)])
def test_compose_shapes_exact(dev, dp, dq):
    say(f"compose shapes dp={dp} dq={dq}")
    g = np.random.default_rng([dp, dq])
    P = g.integers(0, P31, size=(5, dp + 1), dtype=np.uint32)
    Q = g.integers(0, P31, size=(5, dq + 1), dtype=np.uint32)
    for scheme in ["horner", "estrin", "balanced", "balanced_floor"]:
        got = gpu_compose(P, Q, scheme, dev)
        for b in range(5):
            assert got[b].tolist() == ocomp.compose(P[b].tolist(), Q[b].tolist(), P31), (scheme, b)


def test_compose_special_cases(dev):
    say("compose special cases")
    g = np.random.default_rng(5)
    P = g.integers(0, P31, size=(3, 17), dtype=np.uint32)
    # q = x gives p
    Q = np.zeros((3, 2), dtype=np.uint32)
    Q[:, 1] = 1
    assert np.array_equal(gpu_compose(P, Q, "balanced", dev)[:, :17], P)
    # sparse p (zero coefficients, zero constant term): p = x^k gives q^k
    P2 = np.zeros((2, 9), dtype=np.uint32)
    P2[:, 8] = 1
    Q2 = g.integers(0, P31, size=(2, 4), dtype=np.uint32)
    got = gpu_compose(P2, Q2, "estrin", dev)
    for b in range(2):
        for t in [3, 77, P31 - 5]:
            assert ocomp.horner_at(got[b].tolist(), t, P31) == pow(ocomp.horner_at(Q2[b].tolist(), t, P31), 8, P31)


def test_compose_full_size_schwartz_zippel(dev):
    say("compose 4096 x (255 o 15) balanced + horner, Schwartz-Zippel on every instance")
    inp = fpe_inputs.compose_batch()
    for scheme in ["balanced", "horner"]:
        got = gpu_compose(inp.p, inp.q, scheme, dev)
        assert got.shape == (4096, 255 * 15 + 1)
        rng = np.random.default_rng(17)
        for b in range(4096):
            t = int(rng.integers(2, P31 - 1))
            assert ocomp.horner_at(got[b].tolist(), t, P31) == ocomp.compose_at(inp.p[b].tolist(), inp.q[b].tolist(), t, P31), (scheme, b)
        idx = [0, 1, 2047, 4095]
        want = native.compose_modp(inp.p[idx], inp.q[idx], P31)
        assert np.array_equal(got[idx], want)


def gpu_compose_method(P, Q, scheme, dev, product):
    b, dp1 = P.shape
    ex = np.arange(dp1, dtype=np.int32).reshape(-1, 1)
    t = fpe.Tree(ex, P.astype(np.uint64), scheme, fpe.MODP, P31).upload(dev)
    q = torch.from_numpy(np.ascontiguousarray(Q.astype(np.int32))).to(dev)
    out = fpe.compose(t, q, product=product)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("scheme", ["balanced", "estrin", "horner", "balanced_floor"])
def test_compose_product_methods_agree_exactly(dev, scheme):
    """The fused walk, the op-by-op walk with schoolbook products, the
    op-by-op walk with transform products and the level walk with matrix-core
    products give the same residues, equal to the oracle's expansion (sparse
    p with a zero constant term included)."""
    say(f"compose product methods {scheme}")
    g = np.random.default_rng([13075655, 930])
    for b, dp, dq in [(37, 255, 15), (9, 130, 7), (5, 64, 63), (4, 300, 1), (3, 273, 15)]:
        P = g.integers(0, P31, size=(b, dp + 1), dtype=np.uint32)
        P[:, 0] = 0
        P[:, g.choice(dp, dp // 10, replace=False)] = 0
        Q = g.integers(0, P31, size=(b, dq + 1), dtype=np.uint32)
        got = {m: gpu_compose_method(P, Q, scheme, dev, m) for m in ("fused", "schoolbook", "ntt", "mfma")}
        assert np.array_equal(got["fused"], got["ntt"]), (b, dp, dq)
        assert np.array_equal(got["fused"], got["schoolbook"]), (b, dp, dq)
        assert np.array_equal(got["fused"], got["mfma"]), (b, dp, dq)
        want = native.compose_modp(P[:3], Q[:3], P31)
        assert np.array_equal(got["ntt"][:3], want), (b, dp, dq)


def test_compose_ntt_beyond_the_fused_walk(dev):
    """Outputs longer than the fused walk takes (deg 1023 o 15: 15,346
    coefficients) go to the transform products: exact against the oracle on
    two instances, Schwartz-Zippel on all, the same for every scheme."""
    say("compose 12 x (1023 o 15) by transforms")
    g = np.random.default_rng([13075655, 931])
    P = g.integers(0, P31, size=(12, 1024), dtype=np.uint32)
    Q = g.integers(0, P31, size=(12, 16), dtype=np.uint32)
    res = {s: gpu_compose_method(P, Q, s, dev, "auto") for s in ("balanced", "estrin", "horner")}
    assert res["balanced"].shape == (12, 1023 * 15 + 1)
    assert np.array_equal(res["balanced"], res["estrin"]) and np.array_equal(res["balanced"], res["horner"])
    want = native.compose_modp(P[:2], Q[:2], P31)
    assert np.array_equal(res["balanced"][:2], want)
    rng = np.random.default_rng(3)
    for b in range(12):
        t = int(rng.integers(2, P31 - 1))
        assert ocomp.horner_at(res["balanced"][b].tolist(), t, P31) == \
            ocomp.compose_at(P[b].tolist(), Q[b].tolist(), t, P31), b


def test_compose_mfma_digit_extremes_and_shapes(dev):
    """The level walk's matrix-core products on residues at the ends of the
    balanced-digit range (0, 1, (p - 1) / 2, (p + 1) / 2, p - 2, p - 1: every
    digit at -128 or 127 somewhere), a constant p, a single term c x^k (a
    leaf root with its own power), outputs ending exactly on a tile (4096 =
    273 * 15 + 1) and one past it with the long node on the schoolbook
    kernel, each bit-exact against the oracle's expansion."""
    say("compose mfma: digit extremes, constant and monomial p, tile edges")
    g = np.random.default_rng([13075655, 932])
    ext = np.array([0, 1, (P31 - 1) // 2, (P31 + 1) // 2, P31 - 2, P31 - 1, 0x7F7F7F7F, 0x80808080 % P31],
                   dtype=np.uint32)
    for b, dp, dq in [(4, 255, 15), (3, 273, 15), (2, 70, 63)]:
        P = ext[g.integers(0, len(ext), size=(b, dp + 1))]
        Q = ext[g.integers(0, len(ext), size=(b, dq + 1))]
        Q[:, dq] = P31 - 1
        P[:, dp] = P31 - 1
        for scheme in ("balanced", "estrin"):
            got = gpu_compose_method(P, Q, scheme, dev, "mfma")
            assert np.array_equal(got, native.compose_modp(P, Q, P31)), (b, dp, dq, scheme)
    # p = c (constant) and p = c x^k
    Q = g.integers(0, P31, size=(2, 8), dtype=np.uint32)
    t = fpe.Tree(np.zeros((1, 1), np.int32), np.array([[12345], [678]], np.uint64), "balanced", fpe.MODP,
                 P31).upload(dev)
    out = fpe.compose(t, torch.from_numpy(Q.astype(np.int32)).to(dev), product="mfma")
    torch.cuda.synchronize()
    assert out.cpu().numpy().view(np.uint32).tolist() == [[12345], [678]]
    t = fpe.Tree(np.array([[9]], np.int32), np.array([[5], [P31 - 1]], np.uint64), "estrin", fpe.MODP,
                 P31).upload(dev)
    out = fpe.compose(t, torch.from_numpy(Q.astype(np.int32)).to(dev), product="mfma")
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    for b, c in enumerate([5, P31 - 1]):
        pk = [0] * 9 + [c]
        assert got[b].tolist() == ocomp.compose(pk, Q[b].tolist(), P31), b
    # past four tiles: the root's products on the schoolbook kernel
    P = g.integers(0, P31, size=(2, 301), dtype=np.uint32)
    Q = g.integers(0, P31, size=(2, 16), dtype=np.uint32)
    got = gpu_compose_method(P, Q, "balanced", dev, "mfma")
    assert np.array_equal(got, native.compose_modp(P, Q, P31))


def test_compose_mfma_full_size_matches_fused(dev):
    """4096 x (255 o 15), the composition benchmark: the level walk equals the
    fused walk bit for bit on every instance (Estrin and balanced), and the
    oracle's expansion on a sample."""
    say("compose 4096 x (255 o 15): mfma vs fused")
    inp = fpe_inputs.compose_batch()
    for scheme in ("estrin", "balanced"):
        a = gpu_compose_method(inp.p, inp.q, scheme, dev, "mfma")
        b = gpu_compose_method(inp.p, inp.q, scheme, dev, "fused")
        assert np.array_equal(a, b), scheme
    idx = [0, 1, 4095]
    assert np.array_equal(a[idx], native.compose_modp(inp.p[idx], inp.q[idx], P31))
