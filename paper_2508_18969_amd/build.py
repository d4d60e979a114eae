"""Compiles the HIP sources of the chemistry-update library for gfx950 into
``libchemdnn.so`` next to this file (in-tree, so a copied tree carries it).

    python -m paper_2508_18969_amd.build

Each source is compiled to an object file in its own hipcc process (in
parallel), then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libchemdnn.so")
SOURCES = ["step_fp32.hip", "step_bf16.hip", "step_fp16.hip", "step_fp8.hip", "step.hip",
           "layered.hip", "train.hip", "capi.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 (v_pk_*_f32) code generation
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _filter(stderr: str) -> str:
    # hipcc's host pass does not know the packed-FP32 feature: harmless
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False, extra=()) -> str:
    with tempfile.TemporaryDirectory(prefix="chemdnn_build_") as tmpd:
        objs, procs = [], []
        for s in SOURCES:
            obj = os.path.join(tmpd, os.path.splitext(s)[0] + ".o")
            cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                              text=True)))
            objs.append(obj)
        failed = []
        for s, p in procs:
            _, err = p.communicate()
            err = _filter(err)
            if p.returncode != 0:
                failed.append(f"{s} ({p.returncode}):\n{err}")
            elif verbose and err.strip():
                print(err)
        if failed:
            raise RuntimeError("hipcc failed: " + "\n".join(failed))
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed ({res.returncode}):\n{_filter(res.stderr)}")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
    print(LIB)
