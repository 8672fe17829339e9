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


def test_bf16_inference_against_the_fp64_reference():
    """BF16 activations and weights with FP32 accumulation, against the FP64 reference forward.
    Each layer rounds its inputs and weights to 8 significant bits (relative 2^-9 each) and sums
    up to 288 products of random sign, so a layer's output carries about 2^-9 sqrt(2) = 2.8e-3 of
    its typical magnitude, plus 2^-9 for its own rounding; over five layers that is about 1e-2,
    and the bound allows twice that."""
    net, feat, _, _ = _net_and_data(B=1, H=40, W=70, seed=5)
    ft = torch.tensor(feat, device="cuda")
    p16 = net.predict_bf16(ft).cpu().double().numpy()
    r = ref.forward(_layers(net), feat.astype(np.float64))[-1]
    err = np.max(np.abs(p16 - r)) / np.max(np.abs(r))
    print("BF16 inference vs FP64 reference: max error %.2e of max |output|" % err)
    assert err <= 2e-2
    # and the FP32 forward is far closer
    p32 = net.forward(ft)[-1].cpu().double().numpy()
    assert np.max(np.abs(p32 - r)) <= 2e-5 * np.max(np.abs(r))


@pytest.mark.parametrize("cin", [8, 32])
@pytest.mark.parametrize("relu", [0, 1])
def test_bf16_layer_on_the_matrix_cores(cin, relu):
    """One 32-output-channel BF16 layer (the matrix-core path) against the FP64 convolution of the
    same BF16-rounded inputs and weights: the FP32 accumulation of at most 288 products is exact
    to about 1e-6 relative, so each output must be the FP64 value rounded to BF16 (relative 2^-8)
    up to that.  Ragged 16x16 tiles (21 x 37) and two images."""
    B, H, W, cout = 2, 21, 37, 32
    rng = np.random.default_rng(11 + cin + relu)
    x = torch.tensor(rng.normal(size=(B, cin, H, W)), dtype=torch.bfloat16, device="cuda")
    w = torch.tensor(rng.normal(size=(cout, cin, 3, 3)) / np.sqrt(9 * cin), dtype=torch.bfloat16,
                     device="cuda")
    b = torch.tensor(rng.normal(size=cout) * 0.1, dtype=torch.float32, device="cuda")
    out = torch.empty((B, cout, H, W), dtype=torch.bfloat16, device="cuda")
    p = lambda t: t.data_ptr()  # noqa: E731
    rc = cnn.lib().lbm_cnn_conv_forward_bf16(p(x), B, cin, H, W, p(w), p(b), cout, relu, p(out),
                                             torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    got = out.float().cpu().double().numpy()
    xd = x.float().cpu().double().numpy()
    wd = w.float().cpu().double().numpy()
    xp = np.pad(xd, ((0, 0), (0, 0), (1, 1), (1, 1)))
    r = np.zeros((B, cout, H, W)) + b.cpu().double().numpy()[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            r += np.einsum("oc,bchw->bohw", wd[:, :, ky, kx], xp[:, :, ky:ky + H, kx:kx + W])
    if relu:
        r = np.maximum(r, 0.0)
    scale = np.max(np.abs(r))
    err = np.abs(got - r)
    print("cin %d relu %d: max |out - ref| %.3e, max |ref| %.3e" % (cin, relu, err.max(), scale))
    assert np.all(err <= 2.0 ** -8 * np.abs(r) + 1e-5 * scale)


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


def test_features_match_reference():
    rng = np.random.default_rng(11)
    B, H, W = 3, 37, 50
    solid = (rng.random((B, H, W)) < 0.45).astype(np.uint8)
    X_in = rng.dirichlet((6.0, 3.0, 1.0), size=B)
    j = rng.uniform(0.0, 2.0, B)
    prof = X_in[:, :2, None] + np.cumsum(rng.normal(0.0, 1e-3, (B, 2, W)), axis=2)
    prof[:, :, 0] = X_in[:, :2]
    dev = lambda a, t: torch.tensor(a, dtype=t, device="cuda")  # noqa: E731
    for case in range(2):
        if case == 1:
            solid[1, :, 7] = 1  # a column of solid only: phi clamps at 1/H
        feat, base = cnn.features(dev(solid, torch.uint8), dev(X_in, torch.float64),
                                  dev(j, torch.float64), dev(prof, torch.float64))
        rf, rb = ref.features(solid, X_in, j, prof)
        assert np.max(np.abs(base.cpu().numpy() - rb)) <= 1e-14
        feat = feat.cpu().double().numpy()
        assert np.max(np.abs(feat - rf)) <= 2e-6 * max(1.0, np.max(np.abs(rf))), case


def test_assemble_matches_reference():
    rng = np.random.default_rng(12)
    B, H, W = 2, 9, 30
    pred = rng.normal(0.0, 3.0, (B, 2, H, W)).astype(np.float32)
    prof = rng.dirichlet((6.0, 3.0, 1.0), size=(B, W)).transpose(0, 2, 1)[:, :2].copy()
    X = cnn.assemble(torch.tensor(pred, device="cuda"),
                     torch.tensor(prof, device="cuda")).cpu().numpy()
    r = ref.assemble(pred.astype(np.float64), prof, cnn.SCALE, 1e-6)
    assert np.max(np.abs(X - r)) <= 1e-7
    assert np.all(X >= 1e-6 - 1e-15) and np.allclose(X.sum(axis=1), 1.0, atol=1e-14)
