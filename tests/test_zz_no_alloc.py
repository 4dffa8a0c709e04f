"""The allocation-free network forward pass (nce_mlp_forward_noalloc) against
nce_mlp_forward through the C ABI: two calls in a row on the same GPU, the
first spanning several workspace chunks (8192 rows each at width 256), the
second smaller, each output compared element by element with the allocating
entry point's."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_mlp_forward_noalloc_matches_forward():
    import torch
    import paper_1906_04209_amd as nce
    assert torch.cuda.is_available()
    lib = nce.load()
    net = nce.Mlp(seed=3)
    g = torch.Generator().manual_seed(11)
    for B in (20000, 777):
        print(f"noalloc forward: B = {B}", flush=True)
        x = torch.randn(B, nce.FEATURES, generator=g).float().cuda()
        ref = net.forward(x)
        y = torch.full((B, 136), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        rc = lib.nce_mlp_forward_noalloc(net.h, ctypes.c_void_p(x.data_ptr()), B, ctypes.c_void_p(y.data_ptr()),
                                         None)
        torch.cuda.synchronize()
        assert rc == 0, lib.nce_last_error()
        assert bool(torch.isfinite(y).all())
        err = float((y - ref).abs().max() / ref.abs().max())
        print(f"  max relative difference {err:.2e}, bit-identical {bool(torch.equal(y, ref))}")
        assert err <= 1e-6
    # the binding's method writes the caller's tensor the same way
    y2 = torch.empty_like(ref)
    net.forward_noalloc(x, y2)
    torch.cuda.synchronize()
    assert float((y2 - ref).abs().max() / ref.abs().max()) <= 1e-6
    net.close()
