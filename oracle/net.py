"""Learned correction network (oracle; test infrastructure only).

The correction added after each ADI preconditioner application inside the
flexible CG of Sec. 7 (a learned addition; the paper has plain ADI-PCG):

    z <- z + s_z * NN([z / s_z, r / s_r, log a]),   s = root-mean-square value.

NN is a stack of 3x3 convolutions with zero padding on the (element, slot)
coefficient image, 3 -> 32 -> 32 -> 32 -> 1 channels, each hidden layer followed
by the tanh form of GELU, gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))
(Hendrycks and Gimpel).  Arrays are NHWC: x[b, h, w, c]; weights W[dy, dx, c_in,
c_out] act as out[h, w] = b + sum W[dy, dx] x[h + dy - 1, w + dx - 1].

Training loss of a batch (weights w_p >= 0 per pixel, targets t = e / s_z, the
normalised error the corrected z should equal, zn = z / s_z):

    L = (1 / B) sum_b  sum_p w_p (zn_p + NN_p - t_p)^2 / sum_p w_p t_p^2.

Everything here is FP64 and written for clarity; ``grad`` is checked against
central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (3, 32, 32, 32, 1)
_C = np.sqrt(2.0 / np.pi)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(_C * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = _C * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    du = _C * (1.0 + 3.0 * 0.044715 * x ** 2)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


def init_params(seed: int, channels=CHANNELS):
    """He-style normal initialisation (std sqrt(2 / fan_in)), zero biases; the last
    layer is scaled by 1/10 so an untrained network makes a small correction."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(len(channels) - 1):
        cin, cout = channels[l], channels[l + 1]
        W = rng.standard_normal((3, 3, cin, cout)) * np.sqrt(2.0 / (9 * cin))
        if l == len(channels) - 2:
            W *= 0.1
        params.append((W, np.zeros(cout)))
    return params


def conv3x3(x, W, b):
    B, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (B, H, Wd, W.shape[3])).copy()
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("bhwc,cd->bhwd", xp[:, dy:dy + H, dx:dx + Wd, :], W[dy, dx])
    return out


def conv3x3_backward(x, W, g):
    """Gradients of sum(g * conv3x3(x, W, b)) w.r.t. x, W and b."""
    B, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            dW[dy, dx] = np.einsum("bhwc,bhwd->cd", xp[:, dy:dy + H, dx:dx + Wd, :], g)
            dxp[:, dy:dy + H, dx:dx + Wd, :] += np.einsum("bhwd,cd->bhwc", g, W[dy, dx])
    return dxp[:, 1:-1, 1:-1, :], dW, g.sum(axis=(0, 1, 2))


def forward(params, x):
    """Returns the output (B, H, W, 1) and the cache of layer inputs and pre-activations."""
    cache = []
    h = x
    for l, (W, b) in enumerate(params):
        pre = conv3x3(h, W, b)
        cache.append((h, pre))
        h = gelu(pre) if l < len(params) - 1 else pre
    return h, cache


def loss(params, x, zn, t, w):
    out, _ = forward(params, x)
    return _loss_from_out(out[..., 0], zn, t, w)


def _loss_from_out(o, zn, t, w):
    num = np.sum(w * (zn + o - t) ** 2, axis=(1, 2))
    den = np.sum(w * t ** 2, axis=(1, 2))
    return float(np.mean(num / den))


def grad(params, x, zn, t, w):
    """Loss and its gradients [(dW, db) per layer]."""
    out, cache = forward(params, x)
    o = out[..., 0]
    B = o.shape[0]
    den = np.sum(w * t ** 2, axis=(1, 2))
    L = float(np.mean(np.sum(w * (zn + o - t) ** 2, axis=(1, 2)) / den))
    g = (2.0 / B) * w * (zn + o - t) / den[:, None, None]
    g = g[..., None]
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        h_in, pre = cache[l]
        if l < len(params) - 1:
            g = g * gelu_grad(pre)
        dx, dW, db = conv3x3_backward(h_in, params[l][0], g)
        grads[l] = (dW, db)
        g = dx
    return L, grads
