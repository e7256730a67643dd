"""Pins of the learned-correction network oracle (oracle/net.py).

* the 3x3 convolution against a direct quadruple loop on a tiny image;
* the tanh-form GELU and its derivative against their formula and a central
  difference;
* the full gradient (all layers, weights and biases) against central finite
  differences of the loss in FP64.
"""
import numpy as np

from oracle import net


def test_conv_against_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 5, 3))
    W = rng.standard_normal((3, 3, 3, 2))
    b = rng.standard_normal(2)
    out = net.conv3x3(x, W, b)
    ref = np.zeros((2, 4, 5, 2))
    for bb in range(2):
        for h in range(4):
            for w in range(5):
                for co in range(2):
                    s = b[co]
                    for dy in range(3):
                        for dx in range(3):
                            hh, ww = h + dy - 1, w + dx - 1
                            if 0 <= hh < 4 and 0 <= ww < 5:
                                s += np.dot(x[bb, hh, ww], W[dy, dx, :, co])
                    ref[bb, h, w, co] = s
    assert np.abs(out - ref).max() < 1e-13


def test_gelu_and_derivative():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(net.gelu(x), 0.5 * x * (1 + np.tanh(np.sqrt(2 / np.pi) * (x + 0.044715 * x ** 3))))
    h = 1e-6
    fd = (net.gelu(x + h) - net.gelu(x - h)) / (2 * h)
    assert np.abs(fd - net.gelu_grad(x)).max() < 1e-8
    assert abs(net.gelu(np.array([0.0]))[0]) == 0.0 and abs(net.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_gradient_against_finite_differences():
    rng = np.random.default_rng(1)
    ch = (3, 4, 4, 1)
    params = net.init_params(2, channels=ch)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for (W, b) in params]
    B, H, Wd = 2, 5, 6
    x = rng.standard_normal((B, H, Wd, 3))
    zn = rng.standard_normal((B, H, Wd))
    t = rng.standard_normal((B, H, Wd))
    w = rng.uniform(0.5, 2.0, (B, H, Wd))
    L, grads = net.grad(params, x, zn, t, w)
    assert abs(L - net.loss(params, x, zn, t, w)) < 1e-14 * max(1.0, L)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                Lp = net.loss(params, x, zn, t, w)
                flat[idx] = old - h
                Lm = net.loss(params, x, zn, t, w)
                flat[idx] = old
                fd = (Lp - Lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx, fd, g.reshape(-1)[idx])
