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
KERNEL_SOURCES = ["paper_2508_18969_amd/csrc/step.hip", "paper_2508_18969_amd/csrc/common.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_chem_step_bf16_2p20.json")


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=1 << 20)
    ap.add_argument("--precisions", default="fp32,bf16,fp16,fp8")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="bytes of one plain device copy run before the timed region")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the per-launch HBM traffic record from two counter runs")
    args = ap.parse_args()
    if args.traffic:
        write_traffic(args.traffic[0], args.traffic[1], args.cells, args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; the chemistry update needs no "
              "communication (cells are independent) - run with --gpus 1", file=sys.stderr)
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
        return ChemDNN(net.widths, prec, params, net.in_mean, net.in_std, net.out_mean,
                       net.out_std, act_amax=act_amax, thermo=thermo, lam=net.lam)

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
        except Exception as e:          # a precision this build lacks
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
        outputs[prec] = (Yo[:, sample_t].cpu().numpy(), To[sample_t].cpu().numpy())
        tflops = FLOP_PER_CELL * n / (ms * 1e-3) * 1e-12
        results[prec] = {"ms_per_step": ms, "cells_per_s": n / (ms * 1e-3), "tflops": tflops,
                         "mfma_frac": tflops / PEAK_TFLOPS[prec], "steps": k}
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

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(st, net, thermo, sample, outputs, results)

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
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def _counter_means(path, name_part):
    """Mean of each counter over the dispatches whose kernel name contains
    name_part (rocprofv3 counter_collection CSV, values in KiB)."""
    import csv
    acc = {}
    for r in csv.DictReader(open(path)):
        if name_part in r["Kernel_Name"]:
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def write_traffic(fetch_csv, write_csv, n_cells, copy_bytes):
    """HBM bytes per launch of the chemistry kernel: FETCH_SIZE + WRITE_SIZE,
    each scaled by bytes/reading of the plain copy of copy_bytes bytes (which
    reads and writes copy_bytes each)."""
    if copy_bytes <= 0:
        sys.exit("--traffic needs --copy-probe BYTES of the counter runs")
    f_k = _counter_means(fetch_csv, "chem_step")["FETCH_SIZE"]
    w_k = _counter_means(write_csv, "chem_step")["WRITE_SIZE"]
    # the copy is the largest other dispatch of the run
    import csv
    f_c = max(float(r["Counter_Value"]) for r in csv.DictReader(open(fetch_csv))
              if "chem_step" not in r["Kernel_Name"] and r["Counter_Name"] == "FETCH_SIZE")
    w_c = max(float(r["Counter_Value"]) for r in csv.DictReader(open(write_csv))
              if "chem_step" not in r["Kernel_Name"] and r["Counter_Name"] == "WRITE_SIZE")
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


def cpu_baseline(st, net, thermo, sample, outputs, results):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload; its results are also the reference of the stated errors."""
    from threadpoolctl import threadpool_info
    from oracle import chem
    idx = np.asarray(sample)
    Ts, Ps, Ys = st.T[idx], st.P[idx], st.Y[:, idx]
    ref = chem.step(Ts, Ps, Ys, net, thermo=thermo)           # warm-up, also the reference
    reps, t0 = 0, time.perf_counter()
    while True:
        chem.step(Ts, Ps, Ys, net, thermo=thermo)
        reps += 1
        el = time.perf_counter() - t0
        if el >= 10.0 or reps >= 200:
            break
    for prec, (Yg, Tg) in outputs.items():
        results[prec]["max_abs_dY"] = float(np.max(np.abs(Yg - ref["Y_new"])))
        results[prec]["max_abs_dT_K"] = float(np.max(np.abs(Tg - ref["T_new"])))
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": reps * len(idx) / el, "unit": "cells/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{len(idx)} seeded cells of the same workload, FP64 numpy oracle "
                      f"(BLAS matmul), {reps} repetitions in {el:.1f} s"}


if __name__ == "__main__":
    main()
