"""Benchmark of the fused chemistry update on one MI355X.

Workload: 2^20 cells, 29 species, network 31-1600-800-400-29 with GELU,
synthetic seeded states (T ~ U(300, 3000) K, P lognormal around 10 MPa,
Y ~ Dirichlet(0.5)) and Xavier weights.  A step is one chem_dnn_step over the
whole batch with state resident in HBM.  `value` is BF16-operand cells/s;
FP32, FP16 and FP8 are timed the same way and listed under `precisions`,
each with its max-abs dY and T error against the FP64 oracle on a sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Counter runs: `--copy-probe BYTES` adds one plain device-to-device copy of that
many bytes before the timed region, whose FETCH_SIZE / WRITE_SIZE readings
calibrate the counters; `--traffic FETCH.csv WRITE.csv` turns two rocprofv3
--pmc counter files of such a run into the stored per-launch traffic record.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_CELL = 2 * (31 * 1600 + 1600 * 800 + 800 * 400 + 400 * 29)     # 3,322,400
STATE_BYTES_PER_CELL = 8 * (2 + 29) + 8 * (29 + 1)                       # in + out, FP64
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "fp8": 5000.0}
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2508_18969_amd/csrc/step_kernel.h", "paper_2508_18969_amd/csrc/step_bf16.hip",
                  "paper_2508_18969_amd/csrc/common.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_chem_step_bf16_2p20.json")
BLOCK_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_chem_step_block_2p27.json")


def _log(msg):
    """Progress on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(n_cells):
    """HBM bytes per launch from the committed counter runs, if they were
    taken on the current kernel source; else None."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha() or t.get("cells") != n_cells:
        return None
    return float(t["hbm_bytes_per_launch"])


def stored_block_traffic():
    """HBM bytes per launch of the 512^3-block launches (per precision) from
    the committed counter runs, if taken on the current kernel source."""
    try:
        t = json.load(open(BLOCK_TRAFFIC_FILE))
    except (OSError, ValueError):
        return {}
    return t if t.get("kernel_sha") == kernel_sha() else {}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=1 << 20)
    ap.add_argument("--precisions", default="fp32,bf16,fp16,fp8,bf16+table,fp16+table16",
                    help="'+table' / '+table16' select the tabulated GELU with FP32 / FP16 "
                         "coefficients")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--workloads",
                    default="fp8_bimodal_2p24,block_2p27,train_b65536,source_2p20,odenet_2p20,"
                            "prnet_2p20",
                    help="further workloads timed after the headline one ('' for none)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="bytes of one plain device copy run before the timed region")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-launch HBM traffic record from two counter runs")
    args = ap.parse_args()
    if args.traffic:
        write_traffic(args.traffic[0], args.traffic[1], args.cells, args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the chemistry update needs no communication "
              "between GPUs (cells are independent) - run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2508_18969_amd import ChemDNN

    dev = torch.device("cuda:0")
    n = args.cells
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    st = synth.make_state(2, n)
    T = torch.tensor(st.T, device=dev)
    P = torch.tensor(st.P, device=dev)
    Y = torch.tensor(st.Y, device=dev)
    params = torch.tensor(net.flat_params(), device=dev)
    Yo = torch.empty_like(Y)
    To = torch.empty_like(T)

    def handle(prec, act_amax=None):
        base, _, form = prec.partition("+")
        return ChemDNN(net.widths, base, params, net.in_mean, net.in_std, net.out_mean,
                       net.out_std, act_amax=act_amax, thermo=thermo, lam=net.lam,
                       gelu=form or "tanh")

    precs = [p for p in args.precisions.split(",") if p]
    results = {}
    outputs = {}
    sample = synth.subsample_indices(2, n, 1 << 12)
    sample_t = torch.tensor(sample, device=dev)
    for prec in precs:
        act_amax = None
        if prec == "fp8":
            # calibration on a separate seeded draw, FP32 forward on the GPU
            cal = synth.make_state(2, 1 << 16, stream="calibration")
            h32 = handle("fp32")
            amax = h32.calibrate(torch.tensor(cal.T, device=dev), torch.tensor(cal.P, device=dev),
                                 torch.tensor(cal.Y, device=dev))
            act_amax = amax.cpu().numpy()
            h32.close()
        try:
            h = handle(prec, act_amax)
        except Exception as e:          # a precision the library lacks
            results[prec] = {"error": str(e)}
            continue
        for _ in range(args.warmup):
            h.step(T, P, Y, Y_out=Yo, T_out=To)
        torch.cuda.synchronize()
        k = args.steps if prec != "fp32" else max(3, args.steps // 4)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(k):
            h.step(T, P, Y, Y_out=Yo, T_out=To)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / k
        _log(f"{prec}: {ms:.3f} ms per step")
        outputs[prec] = (Yo[:, sample_t].cpu().numpy(), To[sample_t].cpu().numpy())
        tflops = FLOP_PER_CELL * n / (ms * 1e-3) * 1e-12
        results[prec] = {"ms_per_step": ms, "cells_per_s": n / (ms * 1e-3), "tflops": tflops,
                         "mfma_frac": tflops / PEAK_TFLOPS[prec.partition("+")[0]], "steps": k}
        h.close()

    if args.copy_probe:
        src = torch.empty(args.copy_probe // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # timed headline run: BF16, exactly K steps between synchronisations
    h = handle("bf16")
    for _ in range(args.warmup):
        h.step(T, P, Y, Y_out=Yo, T_out=To)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        h.step(T, P, Y, Y_out=Yo, T_out=To)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = ev0.elapsed_time(ev1) / args.steps       # one kernel launch per step
    ms_per_step = wall / args.steps * 1e3
    value = n / (ms_per_step * 1e-3)
    achieved = FLOP_PER_CELL * n / (kern_ms * 1e-3) * 1e-12
    traffic = stored_traffic(n)

    torch_ref = _torch_reference_step_ms(torch, net, T, P, Y)
    # the headline state is no longer needed on the device
    del T, P, Y, Yo, To
    torch.cuda.empty_cache()
    extra = {}
    sampled = {}
    for wl in [w for w in args.workloads.split(",") if w]:
        extra[wl], sampled[wl] = WORKLOADS[wl](torch, synth, ChemDNN)
        _log(f"workload {wl} done")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(st, net, thermo, sample, outputs, results, sampled, extra)

    line = {
        "metric": "DNN-chemistry cells/s (BF16 MFMA operands, FP32 accumulate, FP64 update)",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "chemistry update, 2^20 cells, 29 species, MLP 31-1600-800-400-29 "
                               "GELU, Xavier weights, T~U(300,3000) K, P lognormal 10 MPa, "
                               "Y~Dirichlet(0.5)",
                   "cells": n, "species": 29, "widths": list(net.widths)},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["bf16"],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["bf16"],
                     "traffic": traffic, "kernel_ms": kern_ms,
                     "flop_per_cell": FLOP_PER_CELL,
                     "state_GBps": STATE_BYTES_PER_CELL * n / (kern_ms * 1e-3) * 1e-9},
        "precisions": results,
        "workloads": extra,
        "cpu_baseline": cpu,
        "torch_reference": torch_ref,
    }
    print(json.dumps(line), flush=True)


def _time_steps(torch, h, T, P, Y, Yo, To, steps, warmup):
    for _ in range(warmup):
        h.step(T, P, Y, Y_out=Yo, T_out=To)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        h.step(T, P, Y, Y_out=Yo, T_out=To)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _rate(n, ms, prec):
    tf = FLOP_PER_CELL * n / (ms * 1e-3) * 1e-12
    return {"ms_per_step": ms, "cells_per_s": n / (ms * 1e-3), "tflops": tf,
            "mfma_frac": tf / PEAK_TFLOPS[prec],
            "state_GBps": STATE_BYTES_PER_CELL * n / (ms * 1e-3) * 1e-9}


def _fp8_amax(torch, ChemDNN, net, thermo, T, P, Y):
    """Per-layer input amax from the library's FP32 calibration pass."""
    params = torch.tensor(net.flat_params(), device="cuda")
    h = ChemDNN(net.widths, "fp32", params, net.in_mean, net.in_std, net.out_mean, net.out_std,
                thermo=thermo, lam=net.lam)
    amax = h.calibrate(T, P, Y).cpu().numpy()
    h.close()
    return amax


def wl_fp8_bimodal(torch, synth, ChemDNN, n=1 << 24):
    """FP8 e4m3 over 2^24 cells with bimodal T (N(800,100) | N(2800,150) K),
    scales from a 2^16-cell calibration draw; the FP32 and BF16 paths run on
    the same batch for comparison."""
    net = synth.make_net(3)
    thermo = synth.make_thermo(3, 29)
    st = synth.make_state(3, n)
    cal = synth.make_state(3, 1 << 16, stream="calibration")
    dev = torch.device("cuda")
    amax = _fp8_amax(torch, ChemDNN, net, thermo, torch.tensor(cal.T, device=dev),
                     torch.tensor(cal.P, device=dev), torch.tensor(cal.Y, device=dev))
    idx = synth.subsample_indices(3, n, 1 << 10)
    T, P, Y = (torch.tensor(a, device=dev) for a in (st.T, st.P, st.Y))
    idx_t = torch.tensor(idx, device=dev)
    Yo, To = torch.empty_like(Y), torch.empty_like(T)
    params = torch.tensor(net.flat_params(), device=dev)
    io = synth.subsample_indices(3, n, 1 << 16)
    out, samp = {}, {"state": (st.T[idx], st.P[idx], st.Y[:, idx]), "net": net, "thermo": thermo,
                     "oracle_state": (st.T[io], st.P[io], np.ascontiguousarray(st.Y[:, io]))}
    for prec in ("fp8", "bf16", "fp32"):
        h = ChemDNN(net.widths, prec, params, net.in_mean, net.in_std, net.out_mean, net.out_std,
                    act_amax=amax if prec == "fp8" else None, thermo=thermo, lam=net.lam)
        ms = _time_steps(torch, h, T, P, Y, Yo, To, 3 if prec == "fp32" else 10, 2)
        h.close()
        out[prec] = _rate(n, ms, prec)
        samp[prec] = (Yo[:, idx_t].cpu().numpy(), To[idx_t].cpu().numpy())
    for prec in ("bf16", "fp32"):
        out["fp8"][f"max_abs_dY_vs_{prec}"] = float(np.max(np.abs(samp["fp8"][0] - samp[prec][0])))
        out["fp8"][f"max_abs_dT_K_vs_{prec}"] = float(np.max(np.abs(samp["fp8"][1] - samp[prec][1])))
    out["config"] = {"cells": n, "T": "bimodal N(800,100) | N(2800,150) K", "P": "lognormal 10 MPa",
                     "Y": "Dirichlet(0.5)", "calibration_cells": 1 << 16}
    del T, P, Y, Yo, To
    torch.cuda.empty_cache()
    return out, samp


def wl_block(torch, synth, ChemDNN, edge=512):
    """The 512^3 block (seeded smooth fields, LOX/CH4-like compositions), BF16
    and FP8, state drawn on the device."""
    n = edge ** 3
    net = synth.make_net(5)
    thermo = synth.make_thermo(5, 29)
    T, P, Y = synth.make_block_state_device(5, edge, 29, device="cuda")
    dev = torch.device("cuda")
    cal_t = torch.tensor(synth.subsample_indices(5, n, 1 << 16), device=dev)
    amax = _fp8_amax(torch, ChemDNN, net, thermo, T[cal_t].contiguous(), P[cal_t].contiguous(),
                     Y[:, cal_t].contiguous())
    idx_t = torch.tensor(synth.subsample_indices(5, n, 1 << 10), device=dev)
    io_t = torch.tensor(synth.subsample_indices(5, n, 1 << 16), device=dev)
    samp = {"state": (T[idx_t].cpu().numpy(), P[idx_t].cpu().numpy(), Y[:, idx_t].cpu().numpy()),
            "net": net, "thermo": thermo,
            "oracle_state": (T[io_t].cpu().numpy(), P[io_t].cpu().numpy(),
                             Y[:, io_t].contiguous().cpu().numpy())}
    Yo, To = torch.empty_like(Y), torch.empty_like(T)
    params = torch.tensor(net.flat_params(), device=dev)
    out = {}
    for prec in ("bf16", "fp8"):
        h = ChemDNN(net.widths, prec, params, net.in_mean, net.in_std, net.out_mean, net.out_std,
                    act_amax=amax if prec == "fp8" else None, thermo=thermo, lam=net.lam)
        ms = _time_steps(torch, h, T, P, Y, Yo, To, 3, 1)
        h.close()
        out[prec] = _rate(n, ms, prec)
        tr = stored_block_traffic().get(prec)
        # HBM bytes counted by FETCH_SIZE / WRITE_SIZE for this launch, per second
        out[prec]["hbm_GBps"] = tr["hbm_bytes_per_launch"] / (ms * 1e-3) * 1e-9 if tr else None
        samp[prec] = (Yo[:, idx_t].cpu().numpy(), To[idx_t].cpu().numpy())
    out["config"] = {"cells": n, "block": f"{edge}^3", "T": "300 + 2900 c K", "P": "5 + 15 p MPa",
                     "Y": "mix of LOX-like / CH4-like compositions and Dirichlet(0.5)"}
    del T, P, Y, Yo, To
    torch.cuda.empty_cache()
    return out, samp


def wl_train(torch, synth, ChemDNN, B=65536, steps=20, chunk=8192):
    """One Adam training step of the 19-400-200-100-17 net over a batch of
    65,536 states (features, FP32 forward, MSE, backward, Adam), timed with
    the pre-activations of the whole batch saved, and with activation
    recomputation in chunks of 8,192 samples (forward and backward chunk by
    chunk, gradient accumulated; the workspace holds one chunk's
    pre-activations); targets are seeded normal draws (the step's work does
    not depend on their values)."""
    net = synth.make_net(4)
    st = synth.make_state(4, B)
    dev = torch.device("cuda")
    T, P, Y = (torch.tensor(a, device=dev) for a in (st.T, st.P, st.Y))
    rng = synth.streams(4)["extra"]
    tgt = torch.tensor(rng.standard_normal((17, B)), dtype=torch.float32, device=dev)
    p0 = torch.tensor(net.flat_params(), device=dev)
    out = {}
    for name, rc in (("saved", 0), (f"recompute_chunk_{chunk}", chunk)):
        p = p0.clone()
        g, m, v = torch.empty_like(p), torch.zeros_like(p), torch.zeros_like(p)
        h = ChemDNN(net.widths, "fp32", p, net.in_mean, net.in_std, net.out_mean, net.out_std,
                    lam=net.lam, max_batch=B, recompute_chunk=rc)
        for k in range(1, 3):
            h.train_step(T, P, Y, tgt, p, g, m, v, k, lr=1e-3)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(3, 3 + steps):
            h.train_step(T, P, Y, tgt, p, g, m, v, k, lr=1e-3)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        fl = 3 * 2 * sum(a * b for a, b in zip(net.widths[:-1], net.widths[1:])) * B
        out[name] = {"ms_per_step": ms, "samples_per_s": B / (ms * 1e-3),
                     "tflops_fwd_bwd": fl / (ms * 1e-3) * 1e-12,
                     "workspace_bytes": int(h.workspace.numel())}
        h.close()
    out["torch_reference"] = _torch_train_step_ms(torch, net.widths, B, steps)
    out["config"] = {"batch": B, "widths": list(net.widths), "optimizer": "Adam lr 1e-3",
                     "targets": "seeded normal draws of the label shape"}
    return out, None


def _time_ms(torch, f, reps=10, warm=3):
    for _ in range(warm):
        f()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        f()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _torch_reference_step_ms(torch, net, T, P, Y):
    """Context for the headline: the same chemistry update written with torch
    on the GPU (library BF16 matrix products with FP32 bias and GELU, the
    transforms and the update as elementwise torch operations in FP64), and
    its network alone in pure BF16 (products with bias, GELU in BF16)."""
    lam = net.lam
    dev = T.device
    mu = torch.tensor(net.in_mean, device=dev)
    sd = torch.tensor(net.in_std, device=dev)
    Ws = [torch.tensor(w, device=dev).to(torch.bfloat16) for w in net.W]
    bs = [torch.tensor(b, device=dev).float() for b in net.b]

    def mlp(a, fp32_epilogue):
        for l in range(len(Ws)):
            if fp32_epilogue:
                h = torch.nn.functional.linear(a, Ws[l]).float() + bs[l]
                a = torch.nn.functional.gelu(h, approximate="tanh").to(torch.bfloat16) if l < len(Ws) - 1 else h
            else:
                h = torch.nn.functional.linear(a, Ws[l], bs[l].to(torch.bfloat16))
                a = torch.nn.functional.gelu(h, approximate="tanh") if l < len(Ws) - 1 else h
        return a

    def step():
        yl = Y.clamp_min(0) ** lam
        x = torch.cat([T[None], P[None], (yl - 1) / lam], 0)
        z = ((x - mu[:, None]) / sd[:, None]).float().t().contiguous().to(torch.bfloat16)
        o = mlp(z, True).t().double()
        yh = (Y + ((yl + lam * o).clamp_min(0) ** (1 / lam) - Y)).clamp_min(0)
        return yh / yh.sum(0, keepdim=True)

    z0 = torch.zeros((T.shape[0], net.widths[0]), dtype=torch.bfloat16, device=dev)
    out = {"step_ms": _time_ms(torch, step), "mlp_bf16_ms": _time_ms(torch, lambda: mlp(z0, False)),
           "what": "torch on the GPU, library BF16 products (context only)"}
    torch.cuda.empty_cache()
    return out


def _torch_train_step_ms(torch, widths, B, steps):
    """Context for the training step: the same network and step written with
    torch.nn on the GPU (FP32 library matrix products, tanh GELU, MSE, fused
    Adam, no TF32), normalised features given."""
    torch.backends.cuda.matmul.allow_tf32 = False
    layers = []
    for i in range(len(widths) - 1):
        layers.append(torch.nn.Linear(widths[i], widths[i + 1]))
        if i < len(widths) - 2:
            layers.append(torch.nn.GELU(approximate="tanh"))
    net = torch.nn.Sequential(*layers).to("cuda").float()
    opt = torch.optim.Adam(net.parameters(), lr=1e-3, fused=True)
    gen = torch.Generator(device="cuda").manual_seed(18969)
    x = torch.randn(B, widths[0], device="cuda", generator=gen)
    t = torch.randn(B, widths[-1], device="cuda", generator=gen)

    def step():
        opt.zero_grad(set_to_none=True)
        torch.nn.functional.mse_loss(net(x), t).backward()
        opt.step()

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del net, opt, x, t
    return {"ms_per_step": ms, "samples_per_s": B / (ms * 1e-3),
            "what": "torch.nn eager, FP32 library products, fused Adam (context only)"}


def wl_source(torch, synth, ChemDNN, n=1 << 20, dt=1e-6):
    """The headline batch (2^20 cells, 29 species) through chem_dnn_step_source
    in BF16: the update plus the species source terms rho (Y_new - Y)/dt, with
    seeded molar masses (232 more bytes written per cell)."""
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    W = synth.make_molar_masses(2, 29)
    st = synth.make_state(2, n)
    dev = torch.device("cuda")
    T, P, Y = (torch.tensor(a, device=dev) for a in (st.T, st.P, st.Y))
    Yo, To, om = torch.empty_like(Y), torch.empty_like(T), torch.empty_like(Y)
    params = torch.tensor(net.flat_params(), device=dev)
    h = ChemDNN(net.widths, "bf16", params, net.in_mean, net.in_std, net.out_mean, net.out_std,
                thermo=thermo, lam=net.lam, molar_mass=W)
    for _ in range(3):
        h.step_source(T, P, Y, dt, Y_out=Yo, T_out=To, omega=om)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        h.step_source(T, P, Y, dt, Y_out=Yo, T_out=To, omega=om)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    h.close()
    out = {"bf16": _rate(n, ms, "bf16")}
    out["bf16"]["state_GBps"] = (STATE_BYTES_PER_CELL + 8 * 29) * n / (ms * 1e-3) * 1e-9
    out["config"] = {"cells": n, "dt_s": dt, "molar_mass": "log-uniform 2-200 g/mol",
                     "density": "ideal gas of the state before the step"}
    del T, P, Y, Yo, To, om
    torch.cuda.empty_cache()
    return out, None


def wl_odenet(torch, synth, ChemDNN, n=1 << 20):
    """The ODENet size of the paper's runs, 19-2048-4096-2048-1024-512-17
    (38.9 MFLOP per cell), over 2^20 cells of the 17-species distribution, in
    BF16 and FP16 on the layer-by-layer path (chunks of 32,768 cells, one
    matrix-core kernel per layer)."""
    net = synth.make_net(6)
    thermo = synth.make_thermo(6, 17)
    st = synth.make_state(6, n)
    dev = torch.device("cuda")
    T, P, Y = (torch.tensor(a, device=dev) for a in (st.T, st.P, st.Y))
    Yo, To = torch.empty_like(Y), torch.empty_like(T)
    params = torch.tensor(net.flat_params(), device=dev)
    flop = 2 * sum(a * b for a, b in zip(net.widths[:-1], net.widths[1:]))
    out = {}
    for prec in ("bf16", "fp16"):
        h = ChemDNN(net.widths, prec, params, net.in_mean, net.in_std, net.out_mean, net.out_std,
                    thermo=thermo, lam=net.lam)
        ms = _time_steps(torch, h, T, P, Y, Yo, To, 3, 1)
        h.close()
        tf = flop * n / (ms * 1e-3) * 1e-12
        out[prec] = {"ms_per_step": ms, "cells_per_s": n / (ms * 1e-3), "tflops": tf,
                     "mfma_frac": tf / PEAK_TFLOPS[prec]}
    out["config"] = {"cells": n, "widths": list(net.widths), "flop_per_cell": flop,
                     "chunk_cells": 32768}
    del T, P, Y, Yo, To
    torch.cuda.empty_cache()
    return out, None


def wl_prnet(torch, synth, ChemDNN, n=1 << 20):
    """The property networks of the supercritical flame (the paper's PRNet
    sizes 3-1024-512-256-1 for the density and 3-2048-1024-512-4 for the
    temperature and transport properties) over 2^20 cells of the LOX/CH4
    mixing-layer inputs, in BF16 and FP16, through chem_prop_eval."""
    from paper_2508_18969_amd import PropNet
    dev = torch.device("cuda")
    out = {}
    for cfg, name in ((7, "density"), (8, "transport")):
        net = synth.make_prop_net(cfg)
        x = torch.tensor(synth.make_prop_inputs(cfg, n), device=dev)
        y = torch.empty((net.widths[-1], n), dtype=torch.float64, device=dev)
        params = torch.tensor(net.flat_params(), device=dev)
        flop = 2 * sum(a * b for a, b in zip(net.widths[:-1], net.widths[1:]))
        res = {"widths": list(net.widths), "flop_per_cell": flop}
        for prec in ("bf16", "fp16"):
            h = PropNet(net.widths, prec, params, net.in_mean, net.in_std, net.out_mean, net.out_std)
            for _ in range(3):
                h.eval(x, y)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                h.eval(x, y)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 10
            h.close()
            tf = flop * n / (ms * 1e-3) * 1e-12
            res[prec] = {"ms_per_step": ms, "cells_per_s": n / (ms * 1e-3), "tflops": tf,
                         "mfma_frac": tf / PEAK_TFLOPS[prec]}
        out[name] = res
        del x, y, params
    out["config"] = {"cells": n, "inputs": "E, p, mixture fraction (seeded LOX/CH4 mixing layer)"}
    torch.cuda.empty_cache()
    return out, None


WORKLOADS = {"fp8_bimodal_2p24": wl_fp8_bimodal, "block_2p27": wl_block, "train_b65536": wl_train,
             "source_2p20": wl_source, "odenet_2p20": wl_odenet, "prnet_2p20": wl_prnet}


def _counter_means(path, name_parts):
    """Mean of each counter over the dispatches of the headline kernel (BF16
    operands, tanh GELU) at the headline size: kernel names containing every
    string of name_parts, values within 4x of the smallest (larger launches
    of the same kernel, e.g. the 512^3 block, are left out; rocprofv3
    counter_collection CSV, values in KiB)."""
    import csv
    acc = {}
    for r in csv.DictReader(open(path)):
        if all(p in r["Kernel_Name"] for p in name_parts):
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = {}
    for k, v in acc.items():
        sel = [x for x in v if x <= 4 * min(v)]
        out[k] = sum(sel) / len(sel)
    return out


def write_traffic(fetch_csv, write_csv, n_cells, copy_bytes):
    """HBM bytes per launch of the chemistry kernel: FETCH_SIZE + WRITE_SIZE,
    each scaled by bytes/reading of the plain copy of copy_bytes bytes (which
    reads and writes copy_bytes each)."""
    if copy_bytes <= 0:
        sys.exit("--traffic needs --copy-probe BYTES of the counter runs")
    kern = ("chem_step_kernel<chemdnn::Cfg<chemdnn::OpBF16,", "1600, 800, 400>, false, 0,")
    f_k = _counter_means(fetch_csv, kern)["FETCH_SIZE"]
    w_k = _counter_means(write_csv, kern)["WRITE_SIZE"]
    # the probe is the largest plain copy of the run
    import csv
    f_c = max(float(r["Counter_Value"]) for r in csv.DictReader(open(fetch_csv))
              if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == "FETCH_SIZE")
    w_c = max(float(r["Counter_Value"]) for r in csv.DictReader(open(write_csv))
              if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == "WRITE_SIZE")
    fs, ws = copy_bytes / f_c, copy_bytes / w_c
    rec = {"kernel_sha": kernel_sha(), "cells": n_cells,
           "fetch_kib_per_launch": f_k, "write_kib_per_launch": w_k,
           "copy_bytes": copy_bytes, "copy_fetch_kib": f_c, "copy_write_kib": w_c,
           "fetch_bytes_per_reading": fs, "write_bytes_per_reading": ws,
           "hbm_bytes_per_launch": f_k * fs + w_k * ws,
           "algorithmic_state_bytes": STATE_BYTES_PER_CELL * n_cells}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def _median_s(f, reps=3, warm=None):
    """Median wall time of `reps` calls of f, after one untimed call of warm
    (a smaller instance of the same work; f itself if None)."""
    (warm or f)()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        f()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def cpu_baseline(st, net, thermo, sample, outputs, results, sampled=None, extra=None,
                 n_oracle=1 << 16):
    """The FP64 oracle on the host cores: the headline workload on a seeded
    2^16-cell subsample (median of 3 after a warm-up), and beside it the
    4096-cell 17-species step, the training step at batch 65,536 and 2^16-cell
    subsamples of the 2^24-cell bimodal and the 512^3 block workloads.  Its
    results on the error samples are also the reference of the stated errors
    (of the headline workload and, on their own samples, of the further
    workloads)."""
    import synth
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import chem, train
    idx = np.asarray(sample)
    ref = chem.step(st.T[idx], st.P[idx], st.Y[:, idx], net, thermo=thermo)
    for prec, (Yg, Tg) in outputs.items():
        results[prec]["max_abs_dY"] = float(np.max(np.abs(Yg - ref["Y_new"])))
        results[prec]["max_abs_dT_K"] = float(np.max(np.abs(Tg - ref["T_new"])))
    for wl, sm in (sampled or {}).items():
        if not sm:
            continue
        Tw, Pw, Yw = sm["state"]
        refw = chem.step(Tw, Pw, Yw, sm["net"], thermo=sm["thermo"])
        for prec, val in sm.items():
            if prec in ("state", "net", "thermo", "oracle_state"):
                continue
            extra[wl][prec]["max_abs_dY"] = float(np.max(np.abs(val[0] - refw["Y_new"])))
            extra[wl][prec]["max_abs_dT_K"] = float(np.max(np.abs(val[1] - refw["T_new"])))
            extra[wl][prec]["error_sample_cells"] = int(len(Tw))
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])

    # headline: 2^16 seeded cells of the same workload
    io = synth.subsample_indices(2, len(st.T), n_oracle)
    To_, Po_, Yo_ = st.T[io], st.P[io], np.ascontiguousarray(st.Y[:, io])
    _log("oracle timings on the host")
    sec = _median_s(lambda: chem.step(To_, Po_, Yo_, net, thermo=thermo),
                    warm=lambda: chem.step(To_[:1024], Po_[:1024], Yo_[:, :1024], net,
                                           thermo=thermo))
    # the same oracle on one thread, on 1024 cells of that subsample
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        chem.step(To_[:1024], Po_[:1024], Yo_[:, :1024], net, thermo=thermo)
        one = 1024 / (time.perf_counter() - t1)
    others = {}
    # 4096 cells, 17 species, 19-400-200-100-17 (all cells)
    net1, th1, st1 = synth.make_net(1), synth.make_thermo(1, 17), synth.make_state(1, 4096)
    s1 = _median_s(lambda: chem.step(st1.T, st1.P, st1.Y, net1, thermo=th1))
    others["step_4096_17sp"] = {"cells_per_s": 4096 / s1, "median_s": s1, "cells": 4096}
    # one Adam step of the 19-400-200-100-17 net at batch 65,536
    net4, st4 = synth.make_net(4), synth.make_state(4, 65536)
    x4 = chem.features(st4.T, st4.P, st4.Y, net4.in_mean, net4.in_std, net4.lam)
    t4 = synth.streams(4)["extra"].standard_normal((17, 65536))
    q4 = net4.flat_params().astype(np.float64)
    z4 = np.zeros_like(q4)
    s4 = _median_s(lambda: train.train_step(x4, t4, q4, z4, z4, 1, list(net4.widths)),
                   warm=lambda: train.train_step(x4[:, :4096], t4[:, :4096], q4, z4, z4, 1,
                                                 list(net4.widths)))
    others["train_step_b65536"] = {"samples_per_s": 65536 / s4, "median_s": s4, "batch": 65536}
    # 2^16-cell subsamples of the larger workloads
    for wl in ("fp8_bimodal_2p24", "block_2p27"):
        sm = (sampled or {}).get(wl)
        if not sm or "oracle_state" not in sm:
            continue
        Tw, Pw, Yw = sm["oracle_state"]
        sw = _median_s(lambda: chem.step(Tw, Pw, Yw, sm["net"], thermo=sm["thermo"]),
                       warm=lambda: chem.step(Tw[:1024], Pw[:1024], Yw[:, :1024], sm["net"],
                                              thermo=sm["thermo"]))
        others[wl] = {"cells_per_s": len(Tw) / sw, "median_s": sw, "cells": int(len(Tw))}
        _log(f"oracle {wl}: {sw:.2f} s")
    return {"value": len(io) / sec, "unit": "cells/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{len(io)} seeded cells of the same workload, FP64 numpy oracle "
                      f"(BLAS matmul), median of 3 runs after a warm-up ({sec:.2f} s each)",
            "single_thread_value": one, "workloads": others}


if __name__ == "__main__":
    main()
