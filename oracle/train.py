"""FP64 oracle of one training step of the chemistry net (test infrastructure).

Forward: z_l = W_l a_(l-1) + b_l, a_l = GELU(z_l) for hidden layers, linear
output.  Loss: mean squared error over all outputs of the batch.  Backward:
the chain rule written out per layer; Adam as published by Kingma and Ba
(2015, Algorithm 1) with bias correction.  Arrays are feature-major
([features][batch]); parameters use the flat layout [W1 (out x in), b1, ...].
"""
from __future__ import annotations

import numpy as np

from .chem import gelu, gelu_grad


def unflatten(params, widths):
    params = np.asarray(params, dtype=np.float64)
    W, b, off = [], [], 0
    for i in range(len(widths) - 1):
        fi, fo = widths[i], widths[i + 1]
        W.append(params[off:off + fo * fi].reshape(fo, fi))
        off += fo * fi
        b.append(params[off:off + fo])
        off += fo
    assert off == params.size
    return W, b


def flatten(W, b):
    parts = []
    for w, v in zip(W, b):
        parts += [np.asarray(w).reshape(-1), np.asarray(v).reshape(-1)]
    return np.concatenate(parts)


def forward(x, params, widths):
    """Returns (output [S][B], list of pre-activations z_1..z_L)."""
    W, b = unflatten(params, widths)
    a = np.asarray(x, dtype=np.float64)
    zs = []
    for l in range(len(W)):
        z = W[l] @ a + b[l][:, None]
        zs.append(z)
        a = gelu(z) if l < len(W) - 1 else z
    return a, zs


def mse(o, t):
    """L = (1/(B S)) sum (o - t)^2 and dL/do = 2 (o - t)/(B S)."""
    o = np.asarray(o, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    d = o - t
    return float(np.sum(d * d) / d.size), 2.0 * d / d.size


def backward(x, params, widths, zs, grad_out):
    """Gradient of a scalar loss given dL/do.  Returns (grad_params flat, grad_x).

    dZ_L = dL/do;  for l = L..1:  dW_l = dZ_l a_(l-1)^T,  db_l = sum_batch dZ_l,
    dA_(l-1) = W_l^T dZ_l,  dZ_(l-1) = dA_(l-1) * GELU'(z_(l-1)).
    """
    W, b = unflatten(params, widths)
    L = len(W)
    x = np.asarray(x, dtype=np.float64)
    acts = [x] + [gelu(z) for z in zs[:-1]]
    dZ = np.asarray(grad_out, dtype=np.float64)
    gW, gb = [None] * L, [None] * L
    dA = None
    for l in range(L - 1, -1, -1):
        gW[l] = dZ @ acts[l].T
        gb[l] = dZ.sum(axis=1)
        dA = W[l].T @ dZ
        if l > 0:
            dZ = dA * gelu_grad(zs[l - 1])
    return flatten(gW, gb), dA


def adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update (step counts from 1); returns new (params, m, v)."""
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def train_step(x, t, params, m, v, step, widths, lr=1e-3):
    """Forward, MSE, backward and Adam on one batch.  Returns a dict."""
    o, zs = forward(x, params, widths)
    loss, go = mse(o, t)
    g, _ = backward(x, params, widths, zs, go)
    p, m2, v2 = adam(params, g, m, v, step, lr)
    return {"loss": loss, "grads": g, "params": p, "m": m2, "v": v2, "out": o}
