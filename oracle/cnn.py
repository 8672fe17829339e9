"""FP64 NumPy reference of the warm-start network's layers (test infrastructure only).

conv3x3 with one pixel of zero padding, ReLU, masked mean squared error, and their gradients,
written from the definitions; pinned by finite differences in the tests.
"""

import numpy as np


def conv3x3(x, w, b):
    """x [B,Ci,H,W], w [Co,Ci,3,3], b [Co] -> [B,Co,H,W]:
    y[b,o,i,j] = b[o] + sum_c sum_{u,v} w[o,c,u,v] x[b,c,i+u-1,j+v-1] (zero outside)."""
    B, Ci, H, W = x.shape
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, w.shape[0], H, W)) + b[None, :, None, None]
    for u in range(3):
        for v in range(3):
            y += np.einsum("oc,bcij->boij", w[:, :, u, v], xp[:, :, u:u + H, v:v + W])
    return y


def conv3x3_backward(x, w, gy):
    """Gradients of conv3x3 w.r.t. x, w, b given dL/dy."""
    B, Ci, H, W = x.shape
    xp = np.zeros((B, Ci, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for u in range(3):
        for v in range(3):
            gw[:, :, u, v] = np.einsum("boij,bcij->oc", gy, xp[:, :, u:u + H, v:v + W])
            gxp[:, :, u:u + H, v:v + W] += np.einsum("oc,boij->bcij", w[:, :, u, v], gy)
    return gxp[:, :, 1:-1, 1:-1], gw, gy.sum(axis=(0, 2, 3))


def forward(layers, x):
    """layers: list of (w, b, relu).  Returns the list of layer outputs."""
    acts = []
    h = x
    for w, b, relu in layers:
        h = conv3x3(h, w, b)
        if relu:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return acts


def masked_mse(pred, target, fluid):
    """loss = sum m (p - t)^2 / (C sum m); returns (loss, dloss/dpred)."""
    m = fluid[:, None, :, :]
    cnt = m.sum() * pred.shape[1]
    d = (pred - target) * m
    return float((d * (pred - target)).sum() / cnt), 2.0 * d / cnt


def backward(layers, x, acts, gout):
    """Gradients of every (w, b) given dL/d(last output)."""
    grads = [None] * len(layers)
    g = gout
    for li in range(len(layers) - 1, -1, -1):
        w, b, relu = layers[li]
        if relu:
            g = g * (acts[li] > 0)
        inp = x if li == 0 else acts[li - 1]
        gx, gw, gb = conv3x3_backward(inp, w, g)
        grads[li] = (gw, gb)
        g = gx
    return grads


def features(solid, X_in, j_A_cm2, prof):
    """Network inputs [B,8,H,W] and baseline [B,2,W] from solid [B,H,W] (nonzero = solid), X_in
    [B,3], j [B] (A/cm^2) and the one-dimensional profile prof [B,2,W].  With phi(x) the column
    fluid fraction (at least 1/H), P_s(x) = X_in,s + sum_{x'<=x} (prof_s(x') - prof_s(x'-1)) /
    phi(x'), prof_s(-1) = X_in,s.  Channels: fluid indicator, X_in,1, X_in,2, j/2, x/(W-1),
    (P_1 - X_in,1)/0.01, (P_2 - X_in,2)/0.01, phi.  The baseline is P."""
    B, H, W = solid.shape
    fl = (solid == 0).astype(np.float64)
    out = np.zeros((B, 8, H, W))
    base = np.zeros((B, 2, W))
    for b in range(B):
        phi = np.maximum(fl[b].sum(axis=0), 1.0) / H
        out[b, 0] = fl[b]
        out[b, 1] = X_in[b][0]
        out[b, 2] = X_in[b][1]
        out[b, 3] = 0.5 * j_A_cm2[b]
        out[b, 4] = np.arange(W) / (W - 1) if W > 1 else 0.0
        for s in range(2):
            steps = np.diff(np.concatenate([[X_in[b][s]], prof[b, s]]))
            base[b, s] = X_in[b][s] + np.cumsum(steps / phi)
            out[b, 5 + s] = ((base[b, s] - X_in[b][s]) / 0.01)[None, :]
        out[b, 7] = phi[None, :]
    return out, base


def assemble(pred, prof, scale, x_min):
    """Initial field [B,3,H,W]: X_s = max(prof_s + scale pred_s, x_min) (s = 1, 2); where
    X_3 = 1 - X_1 - X_2 would fall below x_min, the parts of X_1, X_2 above x_min are scaled so
    that X_3 = x_min."""
    X12 = np.maximum(prof[:, :, None, :] + scale * pred, x_min)
    s = X12.sum(axis=1)
    fix = (1.0 - s) < x_min
    f = np.where(fix, (1.0 - 3.0 * x_min) / np.where(fix, s - 2.0 * x_min, 1.0), 1.0)
    X12 = x_min + (X12 - x_min) * f[:, None]
    return np.concatenate([X12, (1.0 - X12.sum(axis=1))[:, None]], axis=1)
