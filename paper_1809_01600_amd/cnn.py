"""Warm-start network: five 3x3 convolution layers (8 -> 32 -> 32 -> 32 -> 32 -> 2 channels, ReLU
between), trained and run with the hand-written HIP kernels of include/lbm_cnn.h.

The paper starts its runs from a one-dimensional profile along x (Section 4.1): the flux equal to
the electrode flux everywhere, in an open channel.  In a porous slice the same flux passes through
a narrower and tortuous cross-section, so the steady depletion is several times larger.  The
features carry a porosity-weighted version of that profile (its increments divided by the fluid
fraction of each column), scaled to order one, together with the fluid indicator, X_in,1, X_in,2,
j / 2 A cm^-2, normalized x and the column fluid fraction.  The network predicts the correction on
the porosity-weighted profile: X_s = P_s + SCALE * output_s (s = 1, 2), X_3 by closure, kept on
the simplex.  Its 11 x 11 receptive field learns the tortuosity factor and the pore-scale
deviation; the profile carries the domain-scale trend.

Argument marshalling only: the arithmetic runs in the library's kernels, on the current torch
stream.
"""

from __future__ import annotations

import ctypes
from typing import List, Sequence

import numpy as np

from . import lbm_ms

CIN = 8
HID = 32
OUT = 2
LAYERS = [(CIN, HID, True), (HID, HID, True), (HID, HID, True), (HID, HID, True), (HID, OUT, False)]
SCALE = 0.1

_VP = ctypes.c_void_p
_I = ctypes.c_int
_CNN_SIGNATURES = [
    ("lbm_cnn_conv_forward", _I, [_VP, _VP, _I, _I, _I, _I, _VP, _VP, _I, _I, _VP, _VP]),
    ("lbm_cnn_conv_forward_bf16", _I, [_VP, _I, _I, _I, _I, _VP, _VP, _I, _I, _VP, _VP]),
    ("lbm_cnn_conv_backward_data", _I, [_VP, _VP, _I, _I, _I, _I, _VP, _I, _VP, _VP, _VP]),
    ("lbm_cnn_backward_weight_scratch", ctypes.c_size_t, [_I, _I, _I, _I, _I]),
    ("lbm_cnn_conv_backward_weight", _I, [_VP, _VP, _VP, _I, _I, _I, _I, _I, _VP, _VP, _VP, _VP]),
    ("lbm_cnn_masked_mse", _I, [_VP, _VP, _VP, _I, _I, _I, _I, _VP, _VP, _VP, _VP]),
    ("lbm_cnn_masked_mse_noalloc", _I, [_VP, _VP, _VP, _I, _I, _I, _I, _VP, _VP, _VP]),
    ("lbm_cnn_adam", _I, [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                          ctypes.c_float, ctypes.c_float, _I, _VP]),
    ("lbm_cnn_to_bf16", _I, [_VP, _VP, ctypes.c_int64, _VP]),
    ("lbm_cnn_from_bf16", _I, [_VP, _VP, ctypes.c_int64, _VP]),
    ("lbm_cnn_features", _I, [_VP, _VP, _VP, _VP, _I, _I, _I, _VP, _VP, _VP]),
    ("lbm_cnn_assemble", _I, [_VP, _VP, _I, _I, _I, ctypes.c_float, ctypes.c_double, _VP, _VP]),
]
CNN_SYMBOLS = [s[0] for s in _CNN_SIGNATURES]
_bound = False


def lib():
    global _bound
    L = lbm_ms.lib()
    if not _bound:
        for name, res, args in _CNN_SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ok(rc, what):
    if rc != 0:
        raise lbm_ms.LbmMsError(rc, what)


class WarmStartNet:
    """Parameters, Adam state and the forward / backward passes."""

    def __init__(self, seed: int = 0, device: str = "cuda"):
        import torch
        self.device = torch.device(device)
        rng = np.random.Generator(np.random.PCG64(seed))
        self.w, self.b = [], []
        for ci, co, _ in LAYERS:
            std = np.sqrt(2.0 / (9 * ci))
            self.w.append(torch.tensor(rng.normal(0.0, std, (co, ci, 3, 3)), dtype=torch.float32,
                                       device=self.device))
            self.b.append(torch.zeros(co, dtype=torch.float32, device=self.device))
        self.w[-1].mul_(0.1)  # start near the profile
        self.m = [torch.zeros_like(t) for t in self.w + self.b]
        self.v = [torch.zeros_like(t) for t in self.w + self.b]
        self.t = 0

    # -- parameters --------------------------------------------------------------------------
    def params(self):
        return self.w + self.b

    def state_dict(self):
        return {"w%d" % i: w.cpu().numpy() for i, w in enumerate(self.w)} | \
               {"b%d" % i: b.cpu().numpy() for i, b in enumerate(self.b)}

    def load_state_dict(self, d):
        import torch
        for i in range(len(LAYERS)):
            self.w[i] = torch.tensor(d["w%d" % i], dtype=torch.float32, device=self.device)
            self.b[i] = torch.tensor(d["b%d" % i], dtype=torch.float32, device=self.device)

    def save(self, path):
        np.savez(path, **self.state_dict())

    def load(self, path):
        with np.load(path, allow_pickle=False) as d:
            self.load_state_dict({k: d[k] for k in d.files})

    # -- passes ------------------------------------------------------------------------------
    def forward(self, feat) -> List:
        """FP32 forward; returns every layer's output (the last is the prediction)."""
        import torch
        B, _, H, W = feat.shape
        acts = []
        h = feat.contiguous()
        for (ci, co, relu), w, b in zip(LAYERS, self.w, self.b):
            out = torch.empty((B, co, H, W), dtype=torch.float32, device=self.device)
            _ok(lib().lbm_cnn_conv_forward(_p(h), None, B, ci, H, W, _p(w), _p(b), co,
                                           1 if relu else 0, _p(out), _stream()), "conv forward")
            acts.append(out)
            h = out
        return acts

    def predict_bf16(self, feat):
        """Inference with bfloat16 activations and weights (FP32 accumulation)."""
        import torch
        B, _, H, W = feat.shape
        h = torch.empty(feat.shape, dtype=torch.int16, device=self.device)
        _ok(lib().lbm_cnn_to_bf16(_p(feat.contiguous()), _p(h), feat.numel(), _stream()), "to bf16")
        for (ci, co, relu), w, b in zip(LAYERS, self.w, self.b):
            wb = torch.empty(w.shape, dtype=torch.int16, device=self.device)
            _ok(lib().lbm_cnn_to_bf16(_p(w), _p(wb), w.numel(), _stream()), "to bf16")
            out = torch.empty((B, co, H, W), dtype=torch.int16, device=self.device)
            _ok(lib().lbm_cnn_conv_forward_bf16(_p(h), B, ci, H, W, _p(wb), _p(b), co,
                                                1 if relu else 0, _p(out), _stream()), "bf16 conv")
            h = out
        pred = torch.empty(h.shape, dtype=torch.float32, device=self.device)
        _ok(lib().lbm_cnn_from_bf16(_p(h), _p(pred), h.numel(), _stream()), "from bf16")
        return pred

    def backward(self, feat, acts, gout):
        """Gradients (gw list, gb list) given dL/d(prediction)."""
        import torch
        B, _, H, W = feat.shape
        gws = [None] * len(LAYERS)
        gbs = [None] * len(LAYERS)
        g = gout.contiguous()
        for li in range(len(LAYERS) - 1, -1, -1):
            ci, co, relu = LAYERS[li]
            inp = feat if li == 0 else acts[li - 1]
            act = acts[li] if relu else None
            gw = torch.empty_like(self.w[li])
            gb = torch.empty_like(self.b[li])
            scratch = torch.empty(lib().lbm_cnn_backward_weight_scratch(B, ci, co, H, W),
                                  dtype=torch.float32, device=self.device)
            _ok(lib().lbm_cnn_conv_backward_weight(_p(inp), _p(g), _p(act), B, ci, co, H, W,
                                                   _p(gw), _p(gb), _p(scratch), _stream()),
                "backward weight")
            gws[li], gbs[li] = gw, gb
            if li > 0:
                gin = torch.empty((B, ci, H, W), dtype=torch.float32, device=self.device)
                wt = torch.empty(ci * co * 9, dtype=torch.float32, device=self.device)
                _ok(lib().lbm_cnn_conv_backward_data(_p(g), _p(act), B, co, H, W, _p(self.w[li]),
                                                     ci, _p(gin), _p(wt), _stream()),
                    "backward data")
                g = gin
        return gws, gbs

    def loss_and_grad(self, pred, target, fluid):
        import torch
        B, C, H, W = pred.shape
        grad = torch.empty_like(pred)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        part = torch.empty(2 * 1024 + 1, dtype=torch.float64, device=self.device)
        _ok(lib().lbm_cnn_masked_mse(_p(pred), _p(target.contiguous()), _p(fluid.contiguous()),
                                     B, C, H, W, _p(grad), _p(loss), _p(part), _stream()), "mse")
        return loss, grad

    def adam(self, grads, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        for p, g, m, v in zip(self.params(), grads, self.m, self.v):
            _ok(lib().lbm_cnn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, beta1, beta2, eps,
                                   self.t, _stream()), "adam")

    def train_step(self, feat, target, fluid, lr=1e-3):
        acts = self.forward(feat)
        loss, g = self.loss_and_grad(acts[-1], target, fluid)
        gws, gbs = self.backward(feat, acts, g)
        self.adam(gws + gbs, lr=lr)
        return loss


def features(solid, X_in, j_A_cm2, prof):
    """Device tensors: solid uint8 [B,H,W], X_in f64 [B,3], j f64 [B], prof f64 [B,2,W] ->
    (features f32 [B,8,H,W], baseline f64 [B,2,W]: the porosity-weighted profile)."""
    import torch
    B, H, W = solid.shape
    feat = torch.empty((B, CIN, H, W), dtype=torch.float32, device=solid.device)
    base = torch.empty((B, 2, W), dtype=torch.float64, device=solid.device)
    _ok(lib().lbm_cnn_features(_p(solid.contiguous()), _p(X_in.contiguous()), _p(j_A_cm2.contiguous()),
                               _p(prof.contiguous()), B, H, W, _p(feat), _p(base), _stream()),
        "features")
    return feat, base


def assemble(pred, base, x_min=1e-6):
    """Prediction [B,2,H,W] + baseline [B,2,W] -> initial field [B,3,H,W] float64 on the device."""
    import torch
    B, _, H, W = pred.shape
    X = torch.empty((B, 3, H, W), dtype=torch.float64, device=pred.device)
    _ok(lib().lbm_cnn_assemble(_p(pred.contiguous()), _p(base.contiguous()), B, H, W, SCALE, x_min,
                               _p(X), _stream()), "assemble")
    return X


def targets(X, base):
    """Training targets (X_s - base_s) / SCALE for s = 1, 2 (torch, device)."""
    return ((X[:, :2] - base[:, :, None, :]) / SCALE).float().contiguous()


def masked_mse_noalloc(pred, target, fluid, grad, loss):
    """Masked MSE and its gradient into caller-provided device tensors (contiguous float32 pred,
    target, grad [B,C,H,W], fluid [B,H,W], loss: one float64), using the library's fixed scratch:
    nothing is allocated by this call."""
    B, C, H, W = pred.shape
    for t in (pred, target, fluid, grad, loss):
        if not t.is_contiguous():
            raise ValueError("masked_mse_noalloc takes contiguous tensors")
    _ok(lib().lbm_cnn_masked_mse_noalloc(_p(pred), _p(target), _p(fluid), B, C, H, W, _p(grad),
                                         _p(loss), _stream()), "mse (no alloc)")
    return loss, grad
