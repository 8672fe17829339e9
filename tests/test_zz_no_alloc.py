"""The allocation-free masked MSE (lbm_cnn_masked_mse_noalloc) against lbm_cnn_masked_mse, through
the C ABI: two calls in a row, the second on a smaller input, each compared with the entry point
that takes its scratch as an argument.  Both run the same kernels in the same order, so loss and
gradient must agree bitwise."""

import numpy as np
import pytest


pytestmark = pytest.mark.gpu


def _case(B, C, H, W, seed):
    import torch
    rng = np.random.default_rng(seed)
    pred = torch.tensor(rng.standard_normal((B, C, H, W)), dtype=torch.float32, device="cuda")
    tgt = torch.tensor(rng.standard_normal((B, C, H, W)), dtype=torch.float32, device="cuda")
    fluid = torch.tensor((rng.random((B, H, W)) > 0.4).astype(np.float32), device="cuda")
    return pred, tgt, fluid


def test_noalloc_mse_matches_scratch_argument_version():
    import torch
    from paper_1809_01600_amd import cnn
    # the large call fills many scratch slots; the smaller one that follows reuses fewer of them
    for shape, seed in (((3, 2, 301, 257), 11), ((1, 2, 37, 29), 12)):
        print("noalloc mse", shape, flush=True)
        pred, tgt, fluid = _case(*shape, seed)
        net = cnn.WarmStartNet(seed=0)
        loss_ref, grad_ref = net.loss_and_grad(pred, tgt, fluid)
        grad = torch.empty_like(pred)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        cnn.masked_mse_noalloc(pred, tgt, fluid, grad, loss)
        torch.cuda.synchronize()
        assert loss.item() == loss_ref.item()
        assert torch.equal(grad, grad_ref)
        # and both against the definition (float64 on the host)
        p, t, m = (x.double().cpu().numpy() for x in (pred, tgt, fluid))
        mm = m[:, None]
        ref = (mm * (p - t) ** 2).sum() / (shape[1] * m.sum())
        assert abs(loss.item() - ref) <= 1e-6 * ref


def test_noalloc_mse_rejects_bad_arguments():
    import ctypes
    from paper_1809_01600_amd import cnn
    rc = cnn.lib().lbm_cnn_masked_mse_noalloc(None, None, None, 1, 1, 1, 1, None, None, None)
    assert rc == -1
