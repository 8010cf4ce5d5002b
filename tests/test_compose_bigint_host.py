"""Host logic of the composition at one big point (no GPU): the slot width
fpe_compose_bigint_coef_limbs picks is the Kronecker bound (every
coefficient of p(q(X)) is at most p(q(1)) < 2^B, B = bitlen(sum c_m) +
deg p * bitlen(q(1)), slots of max(4, ceil(B / 16)) limbs), the output size is
(deg p * dq + 1) slots, and unsupported sizes are refused with 0."""
import ctypes

import numpy as np

import paper_1307_5655_amd as fpe
from oracle import bigint


def plan(coeffs, q, scheme="balanced"):
    exps = [e for e, c in enumerate(coeffs) if c]
    t = fpe.Tree(np.asarray(exps, dtype=np.int32).reshape(-1, 1),
                 np.asarray([coeffs[e] for e in exps], dtype=np.uint64), scheme, fpe.BIGINT)
    qa = np.asarray(q, dtype=np.uint64)
    qp = ctypes.c_void_p(qa.ctypes.data)
    return (int(fpe.lib.fpe_compose_bigint_coef_limbs(t.handle, qp, len(q) - 1)),
            int(fpe.lib.fpe_compose_bigint_out_limbs(t.handle, qp, len(q) - 1)),
            int(fpe.lib.fpe_compose_bigint_workspace_bytes(t.handle, qp, len(q) - 1)))


def test_slot_width_is_the_kronecker_bound():
    rng = np.random.default_rng([13075655, 11])
    for dp, dq in ((0, 3), (1, 0), (5, 1), (12, 3), (20, 2)):
        p = [int(c) for c in rng.integers(1, 2 ** 63, dp + 1, dtype=np.uint64)]
        q = [int(c) for c in rng.integers(0, 2 ** 63, dq + 1, dtype=np.uint64)]
        lc, nout, ws = plan(p, q)
        bits = sum(p).bit_length() + dp * sum(q).bit_length()
        assert lc == max(4, -(-bits // 16))
        assert nout == (dp * dq + 1) * lc
        assert ws > 0
        # the bound holds: every coefficient of the composition fits its slot
        r = bigint.compose_int([((e,), c) for e, c in enumerate(p)], q)
        assert max(r).bit_length() <= 16 * lc


def test_unsupported_sizes_are_refused():
    assert plan([1, 2, 3], [1] * 65)[0] == 0                 # q longer than 64 coefficients
    assert plan([2 ** 63] * 200, [2 ** 63] * 8)[0] == 0      # products beyond 2^14 limbs
    assert plan([1, 2, 3], [1, 1])[0] > 0
