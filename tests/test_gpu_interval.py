"""GPU interval walk (FPE_IVAL) through the C-ABI against the interval oracle.

The oracle takes the tree's value over each box with exact interval
operations (Fractions).  The GPU result must contain it (every bound is
rounded outward) and exceed it by no more than the rounding slack
8 (nodes + chain steps + 8) 2^-52 M, with M = sum |c| prod max(1, |x_j|)^e_j
bounding every partial value.  At full size, where the exact oracle is too
slow, every thin box must contain the double-double value of p (the C oracle,
within its own error bound)."""
from fractions import Fraction

import numpy as np
import pytest
import torch

import fpe_inputs
import paper_1307_5655_amd as fpe
from oracle import interval, native, schemes
from oracle import tree as otree

pytestmark = pytest.mark.gpu

SCHEMES = {"horner": schemes.horner, "estrin": schemes.estrin, "balanced": schemes.balanced,
           "direct": schemes.direct}


def say(msg):
    print(msg, flush=True)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def gpu_boxes(exps, coeffs, scheme, boxes, dev):
    """boxes: float64 [nvars, npts, 2]."""
    t = fpe.Tree(exps, coeffs, scheme, fpe.IVAL).upload(dev)
    out = fpe.evaluate(t, [to_dev(boxes[v], dev) for v in range(boxes.shape[0])])
    torch.cuda.synchronize()
    return out.cpu().numpy(), t


def slack(t, terms, box):
    M = interval.magnitude_bound(terms, box)
    return Fraction(8 * (t.info.n_nodes + t.info.n_chain + 8)) * Fraction(2) ** -52 * M


def check_against_oracle(got, t, terms, scheme, boxes, idx):
    nodes = otree.build_tree(terms, SCHEMES[scheme])
    for i in idx:
        box = [(float(boxes[v, i, 0]), float(boxes[v, i, 1])) for v in range(boxes.shape[0])]
        L, H = interval.tree_interval(nodes, [(Fraction(lo), Fraction(hi)) for lo, hi in box])
        lo, hi = Fraction(float(got[i, 0])), Fraction(float(got[i, 1]))
        assert lo <= L and H <= hi, (i, box, float(L), float(H), got[i])
        s = slack(t, terms, box)
        assert L - lo <= s and hi - H <= s, (i, float(L - lo), float(hi - H), float(s))


def uni_terms(coeffs):
    e = np.nonzero(coeffs)[0]
    return e.astype(np.int32).reshape(-1, 1), coeffs[e], [((int(k),), float(coeffs[k])) for k in e]


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced", "direct"])
def test_interval_univariate_parity(dev, scheme):
    say(f"interval uni sparse n=120 {scheme}")
    inp = fpe_inputs.sparse_uni(120, npts=300 + 13)
    ex, co, terms = uni_terms(inp.coeffs)
    boxes = fpe_inputs.interval_boxes(inp.points, fpe_inputs.rng_for(6, 1))[None]
    got, t = gpu_boxes(ex, co, scheme, boxes, dev)
    assert t.info.n_pair_ops == 0
    # every third box, the ragged tail included
    check_against_oracle(got, t, terms, scheme, boxes, list(range(0, boxes.shape[1], 3)) + [boxes.shape[1] - 1])


@pytest.mark.parametrize("scheme", ["horner", "estrin", "balanced"])
def test_interval_trivariate_parity(dev, scheme):
    say(f"interval trivariate 80 terms {scheme}")
    m = fpe_inputs.random_multi_f64(3, 80, 200 + 7, fpe_inputs.rng_for(6, 2), lo=-1.2, hi=1.2)
    boxes = fpe_inputs.interval_boxes(m.points, fpe_inputs.rng_for(6, 3))
    terms = [(tuple(int(v) for v in e), float(c)) for e, c in zip(m.exps, m.coeffs)]
    got, t = gpu_boxes(m.exps, m.coeffs, scheme, boxes, dev)
    check_against_oracle(got, t, terms, scheme, boxes, range(boxes.shape[1]))


def test_interval_powers_on_the_fly(dev):
    """The direct scheme gives every node its own partial degree: more than the
    48 table entries, so the rest are computed on the fly from the bounds."""
    say("interval direct n=400 (powers on the fly)")
    inp = fpe_inputs.sparse_uni(400, npts=128 + 5)
    ex, co, terms = uni_terms(inp.coeffs)
    boxes = fpe_inputs.interval_boxes(inp.points, fpe_inputs.rng_for(6, 4))[None]
    got, t = gpu_boxes(ex, co, "direct", boxes, dev)
    assert t.info.n_offtable > 0
    check_against_oracle(got, t, terms, "direct", boxes, range(0, boxes.shape[1], 16))


@pytest.mark.parametrize("log2n,depth", [(15, 8), (17, 9)])
def test_interval_deep_walks_contain_the_value(dev, log2n, depth):
    """Thin boxes on Estrin trees of walk depth 8 and 9: the enclosure holds
    the double-double value (error bound n 2^-100 ptilde + 2^-52 |y|)."""
    n = 1 << log2n
    say(f"interval estrin n=2^{log2n} depth {depth}")
    inp = fpe_inputs.dense_uni(npts=2048 + 37, degree=n - 1, seed_k=1)
    ex, co, _ = uni_terms(inp.coeffs)
    boxes = np.stack([inp.points, inp.points], axis=-1)[None]
    got, t = gpu_boxes(ex, co, "estrin", boxes, dev)
    assert t.info.walk_depth == depth
    ref = native.dd_value(inp.coeffs, inp.points)
    pt = native.ptilde(inp.coeffs, inp.points)
    eps = n * 2.0 ** -100 * pt + 2.0 ** -52 * np.abs(ref)
    assert np.all(got[:, 0] <= ref + eps) and np.all(ref - eps <= got[:, 1])
    M = np.abs(inp.coeffs).sum()
    assert np.all(got[:, 1] - got[:, 0] <= 16 * (t.info.n_nodes + t.info.n_chain + 8) * 2.0 ** -52 * M)


@pytest.mark.parametrize("scheme", ["horner", "balanced"])
def test_interval_full_size_thin_boxes(dev, scheme):
    """Degree 3000 at 1e6 boxes of the benchmark's point distribution: every
    thin box contains the double-double value of p, every box is ordered, and a
    sample of boxes of every width matches the exact interval oracle."""
    say(f"interval n=3000 1e6 boxes {scheme}")
    inp = fpe_inputs.sparse_uni(3000, npts=1_000_000)
    ex, co, terms = uni_terms(inp.coeffs)
    boxes = fpe_inputs.interval_boxes(inp.points, fpe_inputs.rng_for(6, 5))[None]
    got, t = gpu_boxes(ex, co, scheme, boxes, dev)
    assert np.all(got[:, 0] <= got[:, 1])
    thin = np.nonzero(boxes[0, :, 0] == boxes[0, :, 1])[0][:100_000]
    x = boxes[0, thin, 0]
    ref = native.dd_value(inp.coeffs, x)
    pt = native.ptilde(inp.coeffs, x)
    eps = 3000 * 2.0 ** -100 * pt + 2.0 ** -52 * np.abs(ref)
    assert np.all(got[thin, 0] <= ref + eps) and np.all(ref - eps <= got[thin, 1])
    g = np.random.default_rng(7)
    # the exact oracle takes seconds per box at this degree (Hörner's rationals grow)
    check_against_oracle(got, t, terms, scheme, boxes, g.choice(boxes.shape[1], 2 if scheme == "horner" else 4,
                                                                replace=False))


def test_interval_edge_cases(dev):
    say("interval edge cases")
    ex = np.array([[0], [1], [2]], dtype=np.int32)
    t = fpe.Tree(ex, np.array([1.0, -2.0, 1.0]), "horner", fpe.IVAL).upload(dev)
    # no points
    out = torch.empty((0, 2), dtype=torch.float64, device=dev)
    fpe.evaluate(t, [torch.empty((0, 2), dtype=torch.float64, device=dev)], out=out)
    # (x - 1)^2 over [1, 1] is exactly 0; over [0, 2] Hörner gives
    # ((x - 2) x + 1) = [-2, 0] [0, 2] + 1 = [-3, 1]
    b = to_dev(np.array([[1.0, 1.0], [0.0, 2.0]]), dev)
    got = fpe.evaluate(t, [b]).cpu().numpy()
    assert got[0, 0] <= 0.0 <= got[0, 1] and got[0, 1] - got[0, 0] < 1e-14
    assert got[1, 0] <= -3.0 and got[1, 1] >= 1.0 and got[1, 1] - got[1, 0] < 4.0 + 1e-12
    # overflow: the whole line
    t2 = fpe.Tree(np.array([[0], [40]], dtype=np.int32), np.array([1.0, 1e300]), "horner", fpe.IVAL).upload(dev)
    got = fpe.evaluate(t2, [to_dev(np.array([[1e10, 1e10]]), dev)]).cpu().numpy()
    assert got[0, 0] == -np.inf and got[0, 1] == np.inf
    # an interval array not 16-byte aligned is refused
    raw = torch.zeros(2 * 8 + 1, dtype=torch.float64, device=dev)
    with pytest.raises(fpe.FpeError):
        fpe.evaluate(t, [raw[1:].view(8, 2)])


def test_interval_subnormal_and_huge_magnitudes(dev):
    """Bounds that land in the subnormal range or near the top of the FP64
    range still enclose the exact interval value."""
    say("interval subnormal / huge magnitudes")
    cases = [
        ([[0], [1], [2]], [1e-300, 1e-160, 3e-150], [(1e-160, 1e-160), (-2e-160, 1e-161), (-1e-155, -1e-156)]),
        ([[0], [1], [3]], [1.0, -1e150, 1e100], [(1e50, 1e50), (-1e50, 2e50), (-3e50, -1e50)]),
    ]
    for ex, co, boxes in cases:
        ex = np.array(ex, dtype=np.int32)
        co = np.array(co)
        terms = [((int(e[0]),), float(c)) for e, c in zip(ex, co)]
        for scheme in ("horner", "estrin"):
            b = np.array(boxes, dtype=np.float64)[None]
            got, t = gpu_boxes(ex, co, scheme, b, dev)
            check_against_oracle(got, t, terms, scheme, b, range(b.shape[1]))
