"""Pins for the FP64 surrogate reference (CPU only): torch's float64
autograd and Adam (library), central finite differences, GELU identities."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp


def _setup(width=32, n=40, seed=0):
    g = np.random.default_rng(seed)
    p = g.normal(0, 0.3, size=mlp.n_params(8, width))
    lo, hi = np.zeros(8), np.ones(8) * 2.0
    x = g.uniform(0, 2, size=(n, 8))
    y = g.normal(80, 10, size=n)
    return p, x, y, lo, hi


def _torch_loss(p, x, y, lo, hi, y_scale, width):
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    xs = 2 * (torch.tensor(x) - torch.tensor(lo)) / (torch.tensor(hi) - torch.tensor(lo)) - 1
    off, h = 0, xs
    for li, (o, i) in enumerate(mlp.layer_shapes(8, width)):
        W = pt[off:off + o * i].view(o, i)
        off += o * i
        b = pt[off:off + o]
        off += o
        h = h @ W.T + b
        if li < 3:
            h = torch.nn.functional.gelu(h, approximate="tanh")
    loss = torch.mean((h[:, 0] - torch.tensor(y) / y_scale) ** 2)
    loss.backward()
    return loss.item(), pt.grad.numpy()


def test_param_count():
    assert mlp.n_params(8, 256) == 134145


def test_gelu_identities():
    """The tanh form of GELU: torch's implementation of the same formula,
    the odd-part identity gelu(z) - gelu(-z) = z, closeness to the erf form
    z Phi(z) (the function it approximates, within 4.8e-4), its limits, and
    its derivative against central differences and torch's autograd."""
    from scipy.special import ndtr
    z = np.linspace(-6, 6, 1001)
    ref = torch.nn.functional.gelu(torch.tensor(z), approximate="tanh").numpy()
    assert np.allclose(mlp.gelu(z), ref, rtol=1e-14, atol=1e-15)
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-14)
    assert np.max(np.abs(mlp.gelu(z) - z * ndtr(z))) < 4.8e-4
    assert mlp.gelu(np.array([40.0]))[0] == 40.0 and abs(mlp.gelu(np.array([-40.0]))[0]) < 1e-300
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)
    zt = torch.tensor(z, requires_grad=True)
    torch.nn.functional.gelu(zt, approximate="tanh").sum().backward()
    assert np.allclose(mlp.gelu_grad(z), zt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_gradient_matches_torch_autograd():
    p, x, y, lo, hi = _setup()
    loss, g = mlp.loss_and_grad(p, x, y, lo, hi, 100.0, width=32)
    tl, tg = _torch_loss(p, x, y, lo, hi, 100.0, 32)
    assert loss == pytest.approx(tl, rel=1e-12)
    assert np.allclose(g, tg, rtol=1e-10, atol=1e-13)


def test_gradient_matches_finite_differences():
    p, x, y, lo, hi = _setup(seed=1)
    _, g = mlp.loss_and_grad(p, x, y, lo, hi, 100.0, width=32)
    idx = np.random.default_rng(2).choice(p.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, x, y, lo, hi, 100.0, width=32)[0] -
              mlp.loss_and_grad(pm, x, y, lo, hi, 100.0, width=32)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9)


def test_adam_matches_torch():
    g = np.random.default_rng(3)
    w0 = g.normal(size=50)
    grads = [g.normal(size=50) for _ in range(5)]
    wt = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t, gr in enumerate(grads, 1):
        opt.zero_grad()
        wt.grad = torch.tensor(gr)
        opt.step()
        w, m, v = mlp.adam_step(w, m, v, gr, t, 1e-2)
    assert np.allclose(w, wt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_cosine_schedule_endpoints():
    assert mlp.cosine_lr(0, 100, 1e-3, 1e-5) == pytest.approx(1e-3)
    assert mlp.cosine_lr(100, 100, 1e-3, 1e-5) == pytest.approx(1e-5)
    assert mlp.cosine_lr(50, 100, 1e-3, 1e-5) == pytest.approx(0.5 * (1e-3 + 1e-5))
