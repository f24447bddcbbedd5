"""The allocation-free forward pass of the quadrature network
(ltmp2_mlp_forward_noalloc, called through the C ABI on device tensors)
against the allocating entry point ltmp2_mlp_forward: two calls in a row,
the second with fewer rows, each compared element by element."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_noalloc_forward_matches_allocating_forward():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_06797_amd import ltmp2 as L
    p = L.mlp_init(3)
    pd = torch.from_numpy(p).cuda()
    for n, seed in ((5000, 31), (777, 32)):
        _say("noalloc forward, rows", n)
        X, _, _, _ = L.mlp_dataset(n, seed)
        ref = L.mlp_forward(p, X)
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.full((n, 24), float("nan"), dtype=torch.float32, device="cuda")
        L.mlp_forward_noalloc(pd, Xd, Yd)
        torch.cuda.synchronize()
        out = Yd.cpu().numpy()
        assert np.isfinite(out).all()
        assert np.array_equal(out, ref)


def test_noalloc_forward_rejects_oversize():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_06797_amd import ltmp2 as L
    n = L.MLP_NOALLOC_MAX_ROWS + 1
    pd = torch.zeros(L.MLP_NPARAM, dtype=torch.float32, device="cuda")
    Xd = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    Yd = torch.zeros((n, 24), dtype=torch.float32, device="cuda")
    with pytest.raises(L.LTMP2Error) as e:
        L.mlp_forward_noalloc(pd, Xd, Yd)
    assert e.value.status == 1
