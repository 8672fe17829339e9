"""Warm-start network kernels against the FP64 NumPy reference (which finite differences pin)."""

import numpy as np
import pytest

from oracle import cnn as ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_01600_amd import cnn  # noqa: E402


def _net_and_data(B=2, H=21, W=37, seed=0):
    net = cnn.WarmStartNet(seed=seed)
    rng = np.random.default_rng(seed + 1)
    feat = rng.normal(size=(B, cnn.CIN, H, W)).astype(np.float32)
    target = rng.normal(size=(B, cnn.OUT, H, W)).astype(np.float32)
    fluid = (rng.random((B, H, W)) < 0.6).astype(np.float32)
    return net, feat, target, fluid


def _layers(net):
    return [(w.cpu().double().numpy(), b.cpu().double().numpy(), relu)
            for (ci, co, relu), w, b in zip(cnn.LAYERS, net.w, net.b)]


def test_forward_matches_reference():
    net, feat, _, _ = _net_and_data()
    acts = net.forward(torch.tensor(feat, device="cuda"))
    refs = ref.forward(_layers(net), feat.astype(np.float64))
    for a, r in zip(acts, refs):
        a = a.cpu().double().numpy()
        assert np.max(np.abs(a - r)) <= 2e-5 * max(1.0, np.max(np.abs(r)))


def test_backward_matches_reference():
    net, feat, target, fluid = _net_and_data(B=2, H=19, W=35, seed=3)
    ft = torch.tensor(feat, device="cuda")
    acts = net.forward(ft)
    loss, g = net.loss_and_grad(acts[-1], torch.tensor(target, device="cuda"),
                                torch.tensor(fluid, device="cuda"))
    gws, gbs = net.backward(ft, acts, g)
    L = _layers(net)
    racts = ref.forward(L, feat.astype(np.float64))
    rloss, rg = ref.masked_mse(racts[-1], target.astype(np.float64), fluid.astype(np.float64))
    assert abs(float(loss.item()) - rloss) <= 1e-5 * rloss
    rgrads = ref.backward(L, feat.astype(np.float64), racts, rg)
    for li, ((rgw, rgb), gw, gb) in enumerate(zip(rgrads, gws, gbs)):
        gw = gw.cpu().double().numpy()
        gb = gb.cpu().double().numpy()
        scale = max(np.max(np.abs(rgw)), 1e-12)
        assert np.max(np.abs(gw - rgw)) <= 1e-4 * scale, li
        assert np.max(np.abs(gb - rgb)) <= 1e-4 * max(np.max(np.abs(rgb)), 1e-12), li


def test_bf16_inference_close_to_fp32():
    net, feat, _, _ = _net_and_data(B=1, H=40, W=70, seed=5)
    ft = torch.tensor(feat, device="cuda")
    p32 = net.forward(ft)[-1].cpu().numpy()
    p16 = net.predict_bf16(ft).cpu().numpy()
    assert np.max(np.abs(p16 - p32)) <= 0.05 * max(1.0, np.max(np.abs(p32)))


def test_training_reduces_loss():
    net, feat, target, fluid = _net_and_data(B=4, H=32, W=32, seed=7)
    ft, tt, fl = (torch.tensor(a, device="cuda") for a in (feat, target * 0.1, fluid))
    losses = [float(net.train_step(ft, tt, fl, lr=3e-3).item()) for _ in range(60)]
    assert losses[-1] < 0.7 * losses[0]


def test_adam_matches_definition():
    net = cnn.WarmStartNet(seed=1)
    p0 = [t.clone() for t in net.params()]
    grads = [torch.full_like(t, 0.5) for t in net.params()]
    net.adam(grads, lr=1e-2)
    # first Adam step moves every parameter by -lr * sign(g) (bias-corrected moments)
    for a, b in zip(net.params(), p0):
        assert torch.allclose(a - b, torch.full_like(a, -1e-2), atol=1e-7)
