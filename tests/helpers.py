"""Shared helpers of the GPU tests: seeded workloads on the device and the
comparison metrics.  Imports the oracle (tests may) and the binding."""
from __future__ import annotations

import numpy as np

import synth

LAM = synth.BOXCOX_LAMBDA


def dev_state(st, device="cuda", ld=None):
    """Copies a synth.State to the device; optional padded leading dimension."""
    import torch
    n = st.n
    ld = n if ld is None else ld
    T = torch.tensor(st.T, dtype=torch.float64, device=device)
    P = torch.tensor(st.P, dtype=torch.float64, device=device)
    Yb = torch.full((st.S, ld), -7.0, dtype=torch.float64, device=device)   # poison padding
    Yb[:, :n] = torch.tensor(st.Y, dtype=torch.float64, device=device)
    return T, P, Yb[:, :n] if ld == n else Yb.narrow(1, 0, n)


def make_handle(net, precision, thermo=None, act_amax=None, max_batch=0, device="cuda",
                gelu="tanh", molar_mass=None, recompute_chunk=0):
    import torch
    from paper_2508_18969_amd import ChemDNN
    params = torch.tensor(net.flat_params(), dtype=torch.float32, device=device)
    h = ChemDNN(net.widths, precision, params, net.in_mean, net.in_std, net.out_mean, net.out_std,
                act_amax=act_amax, thermo=thermo, max_batch=max_batch, lam=net.lam, gelu=gelu,
                molar_mass=molar_mass, recompute_chunk=recompute_chunk)
    h._params = params
    return h


def rel_err(got, ref, floor=1e-10):
    """max_i |got - ref| / max(|ref|, floor)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), floor))) if got.size else 0.0
