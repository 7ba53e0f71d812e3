"""FP64 reference of the surrogate MLP (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The surrogate is not part of the paper; it is the learned extension of the
pricing engine (an MLP n_in -> W -> W -> W -> 1 with GELU activations,
mean-squared-error loss on price / y_scale, Adam).  This module is the plain
numpy reference the GPU kernels are checked against:

* parameters are flat in the order W1 b1 W2 b2 W3 b3 W4 b4, each W row-major
  [out][in] (the library's layout);
* inputs are min-max scaled to [-1, 1]: 2 (x - lo) / (hi - lo) - 1;
* GELU is the tanh form of Hendrycks and Gimpel,
  0.5 z (1 + tanh(u)), u = sqrt(2/pi) (z + 0.044715 z^3), with derivative
  0.5 (1 + tanh u) + 0.5 z (1 - tanh^2 u) u'(z) (within 4.8e-4 of the erf
  form z Phi(z) everywhere);
* loss = mean((yhat - y / y_scale)^2); gradients by reverse-mode chain rule;
* Adam (Kingma & Ba) with bias correction.
"""
from __future__ import annotations

import math

import numpy as np


def layer_shapes(n_in=8, width=256):
    return [(width, n_in), (width, width), (width, width), (1, width)]


def n_params(n_in=8, width=256):
    return sum(o * i + o for o, i in layer_shapes(n_in, width))


def unflatten(p, n_in=8, width=256):
    p = np.asarray(p, dtype=np.float64)
    out, off = [], 0
    for o, i in layer_shapes(n_in, width):
        W = p[off:off + o * i].reshape(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        out.append((W, b))
    assert off == p.size
    return out


_C = math.sqrt(2.0 / math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(_C * (z + 0.044715 * z ** 3))
    du = _C * (1.0 + 3.0 * 0.044715 * z * z)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * du


def scale_inputs(x, lo, hi):
    x = np.asarray(x, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return 2.0 * (x - lo) / (hi - lo) - 1.0


def forward(p, xs, n_in=8, width=256):
    """Network output (scaled units) for scaled inputs xs [n][n_in]; also the
    per-layer pre-activations and activations."""
    layers = unflatten(p, n_in, width)
    h = np.asarray(xs, dtype=np.float64)
    zs, hs = [], [h]
    for W, b in layers[:3]:
        z = h @ W.T + b
        h = gelu(z)
        zs.append(z)
        hs.append(h)
    W4, b4 = layers[3]
    y = (h @ W4.T + b4)[:, 0]
    return y, zs, hs


def loss_and_grad(p, x, y, lo, hi, y_scale, n_in=8, width=256):
    """(loss, flat gradient) of mean((yhat - y/y_scale)^2)."""
    xs = scale_inputs(x, lo, hi)
    yhat, zs, hs = forward(p, xs, n_in, width)
    n = yhat.size
    e = yhat - np.asarray(y, dtype=np.float64) / y_scale
    loss = float(np.mean(e * e))
    layers = unflatten(p, n_in, width)
    grads = [None] * 4
    d = (2.0 / n) * e[:, None]                       # dL/d(out) [n][1]
    W4, _ = layers[3]
    grads[3] = (d.T @ hs[3], d.sum(0))
    dh = d @ W4                                      # [n][width]
    for l in (2, 1, 0):
        dz = dh * gelu_grad(zs[l])
        grads[l] = (dz.T @ hs[l], dz.sum(0))
        dh = dz @ layers[l][0]
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb.reshape(-1)]) for gW, gb in grads])
    return loss, flat


def predict(p, x, lo, hi, y_scale, n_in=8, width=256):
    """Prices predicted for raw inputs x."""
    y, _, _ = forward(p, scale_inputs(x, lo, hi), n_in, width)
    return y * y_scale


def adam_step(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def cosine_lr(step, total, lr_max, lr_min):
    frac = min(1.0, step / total)
    return lr_min + 0.5 * (lr_max - lr_min) * (1 + math.cos(math.pi * frac))
