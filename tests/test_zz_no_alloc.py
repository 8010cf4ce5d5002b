"""fpe_evaluate_noalloc (the allocation-free variant of fpe_evaluate) against
fpe_evaluate with a caller workspace: the same kernels, so the results,
fallback flags and fallback counts must be the same bits; and both within
the compensated form's bar (1e-12 relative) of the oracle on a sample.
Two calls in a row, the second smaller, so that the static scratch keeps the
first call's contents when the second runs."""
import numpy as np
import pytest

import fpe_inputs

pytestmark = pytest.mark.gpu


def _run(fpe, torch, dev, t, x, force, noalloc):
    n = x.numel()
    out = torch.empty(n, dtype=torch.float64, device=dev)
    cond = torch.empty(n, dtype=torch.float32, device=dev)
    flags = torch.zeros((n + 31) // 32, dtype=torch.int32, device=dev)
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)
    if noalloc:
        fpe.evaluate_noalloc(t, [x], out, force=force, cond_out=cond, flags_out=flags, nfallback_out=nfb)
    else:
        fpe.evaluate(t, [x], out=out, force=force, cond_out=cond, flags_out=flags, nfallback_out=nfb)
    torch.cuda.synchronize()
    return out.cpu().numpy(), cond.cpu().numpy(), flags.cpu().numpy(), int(nfb.item())


@pytest.mark.parametrize("scheme", ["balanced", "horner"])
def test_noalloc_matches_workspace_entry_point(dev, scheme):
    import torch

    import paper_1307_5655_amd as fpe
    from oracle import native

    print(f"noalloc: scheme {scheme}", flush=True)
    inp = fpe_inputs.sparse_uni(300, npts=200_003)
    ex, co = inp.terms()
    t = fpe.Tree(ex, co, scheme, fpe.F32C).upload(dev)
    xs_all = torch.from_numpy(inp.points).to(dev)
    # two calls in a row, the second with fewer points (ragged sizes), each
    # with the bound deciding the fallback and with every point re-evaluated
    for n in (200_003, 4_097):
        x = xs_all[:n].contiguous()
        for force in (0, 1):
            a = _run(fpe, torch, dev, t, x, force, noalloc=True)
            b = _run(fpe, torch, dev, t, x, force, noalloc=False)
            assert np.array_equal(a[0].view(np.uint64), b[0].view(np.uint64))
            assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
            assert np.array_equal(a[2], b[2])
            assert a[3] == b[3]
            if force == 1:
                assert a[3] == n
            idx = np.arange(0, n, max(1, n // 997))
            ref = native.dd_value(inp.coeffs, inp.points[idx])
            assert np.max(np.abs(a[0][idx] - ref) / np.abs(ref)) <= 1e-12


def test_noalloc_other_domains_and_limits(dev):
    import torch

    import paper_1307_5655_amd as fpe

    print("noalloc: F64 and the size limit", flush=True)
    inp = fpe_inputs.sparse_uni(300, npts=10_001)
    ex, co = inp.terms()
    x = torch.from_numpy(inp.points).to(dev)
    t64 = fpe.Tree(ex, co, "estrin", fpe.F64).upload(dev)
    a = torch.empty(x.numel(), dtype=torch.float64, device=dev)
    fpe.evaluate_noalloc(t64, [x], a)
    b = fpe.evaluate(t64, [x])
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int64), b.view(torch.int64))
    # beyond the stated maximum: a clear error before anything is launched
    t32 = fpe.Tree(ex, co, "estrin", fpe.F32C).upload(dev)
    big = fpe.NOALLOC_MAX_POINTS + 1
    xb = torch.empty(big, dtype=torch.float64, device=dev)
    yb = torch.empty(big, dtype=torch.float64, device=dev)
    with pytest.raises(fpe.FpeError) as e:
        fpe.evaluate_noalloc(t32, [xb], yb)
    assert "FPE_NOALLOC_MAX_POINTS" in str(e.value)
