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
