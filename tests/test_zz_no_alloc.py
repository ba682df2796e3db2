"""The allocation-free gradient entry point (bbx_mlp_grad_static) against the
allocating one (bbx_mlp_grad): same loss and gradient, bit for bit (the same
kernels in the same order), on two calls in a row, the second with a smaller
batch; batches beyond the static scratch are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NIN = NOUT = 21


def test_static_gradient_equals_allocating_gradient():
    import torch
    from paper_1605_06015_amd import bbx as B
    torch.cuda.set_device(0)
    m = B.Mlp(NIN, NOUT, seed=9)
    rng = np.random.default_rng(3)
    m.set_params((rng.standard_normal(m.nparams) * 0.1).astype(np.float32))
    for n in (4000, 333):          # a large batch, then a smaller ragged one
        X = torch.from_numpy(rng.standard_normal((n, NIN)).astype(np.float32)).cuda()
        T = torch.from_numpy(rng.standard_normal((n, NOUT)).astype(np.float32)).cuda()
        loss_ref, g_ref = m.grad(X, T)
        g_dev = torch.full((m.nparams,), float("nan"), dtype=torch.float32, device="cuda")
        l_dev = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        B.bbx_mlp_grad_static(m.handle, X, T, n, g_dev, l_dev)
        torch.cuda.synchronize()
        g = g_dev.cpu().numpy()
        loss = float(l_dev.cpu().numpy()[0])
        print(n, "loss", loss, loss_ref)
        assert loss == loss_ref
        assert np.array_equal(g, g_ref)


def test_static_gradient_rejects_large_batch():
    import torch
    from paper_1605_06015_amd import bbx as B
    torch.cuda.set_device(0)
    m = B.Mlp(NIN, NOUT, seed=1)
    X = torch.zeros((4097, NIN), dtype=torch.float32, device="cuda")
    with pytest.raises(B.BBXError) as ei:
        B.bbx_mlp_grad_static(m.handle, X, X, 4097)
    assert ei.value.code == B.BBX_EINVAL
    assert "4096" in str(ei.value)
