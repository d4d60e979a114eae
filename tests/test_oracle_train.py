"""Pins of the oracle's MLP backward and Adam: torch autograd in FP64 (an
independent implementation), central finite differences, closed forms."""
import numpy as np
import torch

import synth
from oracle import train

WIDTHS = (19, 24, 16, 12, 17)


def _problem(seed=0, B=40):
    rng = np.random.default_rng(seed)
    W, b = synth.xavier_weights(rng, WIDTHS, bias_scale=0.2)
    p = train.flatten(W, b).astype(np.float64)
    x = rng.standard_normal((WIDTHS[0], B))
    t = rng.standard_normal((WIDTHS[-1], B))
    return p, x, t


def _torch_loss_grad(p, x, t):
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    off, a = 0, xt
    for l in range(len(WIDTHS) - 1):
        fi, fo = WIDTHS[l], WIDTHS[l + 1]
        Wl = pt[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        bl = pt[off:off + fo]
        off += fo
        a = Wl @ a + bl[:, None]
        if l < len(WIDTHS) - 2:
            a = torch.nn.functional.gelu(a, approximate="tanh")
    loss = ((a - torch.tensor(t)) ** 2).mean()
    loss.backward()
    return loss.item(), pt.grad.numpy(), xt.grad.numpy()


def test_backward_matches_torch_autograd():
    p, x, t = _problem()
    o, zs = train.forward(x, p, WIDTHS)
    loss, go = train.mse(o, t)
    g, gx = train.backward(x, p, WIDTHS, zs, go)
    tl, tg, tgx = _torch_loss_grad(p, x, t)
    assert abs(loss - tl) <= 1e-14 * tl
    np.testing.assert_allclose(g, tg, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(gx, tgx, rtol=1e-11, atol=1e-15)


def test_backward_central_differences():
    p, x, t = _problem(1)
    o, zs = train.forward(x, p, WIDTHS)
    _, go = train.mse(o, t)
    g, _ = train.backward(x, p, WIDTHS, zs, go)
    rng = np.random.default_rng(2)
    for i in rng.choice(p.size, 256, replace=False):
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (train.mse(train.forward(x, pp, WIDTHS)[0], t)[0]
              - train.mse(train.forward(x, pm, WIDTHS)[0], t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-6), (i, fd, g[i])


def test_linear_least_squares_closed_form():
    rng = np.random.default_rng(3)
    B, D, S = 50, 6, 4
    W = rng.standard_normal((S, D))
    b = rng.standard_normal(S)
    x = rng.standard_normal((D, B))
    t = rng.standard_normal((S, B))
    p = train.flatten([W], [b])
    o, zs = train.forward(x, p, (D, S))
    _, go = train.mse(o, t)
    g, _ = train.backward(x, p, (D, S), zs, go)
    r = W @ x + b[:, None] - t
    np.testing.assert_allclose(g[:S * D].reshape(S, D), 2 * r @ x.T / (B * S), rtol=1e-13)
    np.testing.assert_allclose(g[S * D:], 2 * r.sum(axis=1) / (B * S), rtol=1e-13)


def test_zero_gradient_at_target():
    p, x, _ = _problem(4)
    o, zs = train.forward(x, p, WIDTHS)
    loss, go = train.mse(o, o)
    g, _ = train.backward(x, p, WIDTHS, zs, go)
    assert loss == 0.0 and np.all(g == 0.0)


def test_adam_first_step_closed_form_and_torch():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(300)
    g = rng.standard_normal(300) * 10.0 ** rng.integers(-6, 2, 300)
    p1, m1, v1 = train.adam(p, g, np.zeros(300), np.zeros(300), 1, lr=1e-3)
    # bias-corrected moments of step 1 are g and g^2
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # several steps against torch.optim.Adam (FP64)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    q, m, v = p.copy(), np.zeros(300), np.zeros(300)
    for k in range(1, 6):
        gk = g * (1.0 + 0.1 * k)
        pt.grad = torch.tensor(gk)
        opt.step()
        q, m, v = train.adam(q, gk, m, v, k, lr=1e-3)
    np.testing.assert_allclose(q, pt.detach().numpy(), rtol=1e-13, atol=1e-16)


def test_train_step_lowers_loss():
    p, x, _ = _problem(6, B=256)
    t = np.tanh(x[:17] * 0.5) * 0.3          # a smooth, learnable target
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for k in range(1, 51):
        r = train.train_step(x, t, p, m, v, k, WIDTHS, lr=3e-3)
        p, m, v = r["params"], r["m"], r["v"]
        losses.append(r["loss"])
    assert losses[-1] < 0.5 * losses[0]
