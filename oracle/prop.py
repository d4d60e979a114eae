"""FP64 oracle of the property networks (test infrastructure; see package doc).

For flames at supercritical pressure the paper's solver evaluates a second
kind of fully connected network per cell, PRNet (Sec. 2), that maps a few
thermodynamic state variables to the mixture's density, temperature and
transport properties in place of the real-fluid equation of state; its sizes
are 3-1024-512-256-1 (density) and 3-2048-1024-512-4 (temperature and
transport properties), Sec. 4.  Per cell: the Z-score normalisation of the
inputs (Sec. 3.3.1), the network with tanh-form GELU hidden layers and a
linear output layer (Sec. 3.3.2; ``chem.mlp``), and the output scaling
y = o sigma_out + mu_out (a reading: the paper states no output transform).

Layout: inputs [n_in][cells], outputs [n_out][cells].
"""
from __future__ import annotations

import numpy as np

from . import chem


def features(x, in_mean, in_std):
    """z = (x - mu_in) / sigma_in per input field (Sec. 3.3.1)."""
    x = np.asarray(x, dtype=np.float64)
    return (x - np.asarray(in_mean, np.float64)[:, None]) / np.asarray(in_std, np.float64)[:, None]


def outputs(o, out_mean, out_std):
    """y = o sigma_out + mu_out."""
    o = np.asarray(o, dtype=np.float64)
    return o * np.asarray(out_std, np.float64)[:, None] + np.asarray(out_mean, np.float64)[:, None]


def evaluate(x, net, fmt=None):
    """Property outputs of every cell.  ``net`` has the attributes of
    ``synth.Net``; ``fmt`` as in ``chem.mlp`` (None: exact FP64, else the
    operands of every layer rounded to that narrow format, scales 1).
    Returns dict(y, o)."""
    z = features(x, net.in_mean, net.in_std)
    W = [np.asarray(w, dtype=np.float64) for w in net.W]
    b = [np.asarray(v, dtype=np.float64) for v in net.b]
    o = chem.mlp(z, W, b, fmt)
    return {"y": outputs(o, net.out_mean, net.out_std), "o": o}
