"""Full-size workloads on the GPU, checked on a seeded sample of cells.

The whole batch runs in one launch, in the configuration the benchmark
times; the oracle then recomputes a seeded sample of cells one by one (the
oracle is exact FP64 or rounds operands like the kernel) and the sample is
held to the same statistical bar as the small-batch parity tests.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import chem
from tests.helpers import make_handle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(a, b, floor=1e-10):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def _check_against_emulation(Yg, Tg, emu, ex, tag):
    """The bar of the narrow-format parity tests: the GPU's deviation from the
    emulation is a small fraction of the quantisation error itself."""
    ge, ee = Yg - emu["Y_new"], emu["Y_new"] - ex["Y_new"]
    rg, re = _rel(Yg, emu["Y_new"]), _rel(emu["Y_new"], ex["Y_new"])
    rms_g, rms_e = np.sqrt(np.mean(ge ** 2)), np.sqrt(np.mean(ee ** 2))
    _note(f"  {tag} gpu-emu: rms {rms_g:.2e} med {np.median(rg):.2e} p99 {np.quantile(rg, .99):.2e} "
          f"max {rg.max():.2e} | emu-fp64: rms {rms_e:.2e} med {np.median(re):.2e} "
          f"p99 {np.quantile(re, .99):.2e} max {re.max():.2e} | gpu-fp64 max abs dY "
          f"{np.abs(Yg - ex['Y_new']).max():.2e} T {np.abs(Tg - ex['T_new']).max():.2e} K")
    assert rms_g <= 0.25 * rms_e
    assert np.median(rg) <= 0.05 * np.median(re)
    assert np.quantile(rg, 0.99) <= 0.5 * np.quantile(re, 0.99)
    assert rg.max() <= 0.5 * re.max()
    tg, te = Tg - emu["T_new"], emu["T_new"] - ex["T_new"]
    assert np.sqrt(np.mean(tg ** 2)) <= 0.25 * np.sqrt(np.mean(te ** 2))
    assert np.abs(tg).max() <= np.abs(te).max()


def _sample_run(h, T, P, Y, idx_t):
    Yo = torch.empty_like(Y)
    To = torch.empty_like(T)
    nbad = torch.zeros(1, dtype=torch.int32, device="cuda")
    h.step(T, P, Y, Y_out=Yo, T_out=To, n_bad=nbad)
    torch.cuda.synchronize()
    out = Yo[:, idx_t].cpu().numpy(), To[idx_t].cpu().numpy(), int(nbad.item())
    del Yo, To
    return out


@pytest.mark.parametrize("prec,fmt", [("fp32", None), ("bf16", "bf16"), ("fp16", "f16")])
def test_headline_2p20_sampled(prec, fmt):
    """The benchmark's headline batch: 2^20 cells of the 29-species net in
    one launch; 1,024 sampled cells against the exact oracle (FP32: 1e-5
    relative on Y_new and T_new) or against the oracle with the same operand
    rounding (BF16, FP16: the bars of the small-batch test)."""
    n = 1 << 20
    _note(f"case headline 2^20 {prec}")
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    st = synth.make_state(2, n)
    idx = synth.subsample_indices(2, n, 1024)
    h = make_handle(net, prec, thermo=thermo)
    dev = torch.device("cuda")
    T, P, Y = (torch.tensor(a, device=dev) for a in (st.T, st.P, st.Y))
    Yg, Tg, nbad = _sample_run(h, T, P, Y, torch.tensor(idx, device=dev))
    assert nbad == 0
    sub = (st.T[idx], st.P[idx], st.Y[:, idx])
    ex = chem.step(*sub, net, thermo=thermo)
    if fmt is None:
        e_y = float(_rel(Yg, ex["Y_new"]).max())
        e_t = float(_rel(Tg, ex["T_new"], floor=1.0).max())
        _note(f"  rel err Y {e_y:.3e}  T {e_t:.3e}")
        assert e_y <= 1e-5 and e_t <= 1e-5
    else:
        emu = chem.step(*sub, net, fmt=fmt, thermo=thermo)
        _check_against_emulation(Yg, Tg, emu, ex, prec)


def test_fp8_bimodal_2p24_sampled():
    """FP8 e4m3 over 2^24 cells with bimodal temperatures; scales from a
    separate calibration draw.  4096 sampled cells against the oracle's FP8
    emulation; FP32 and BF16 runs of the same batch are compared too."""
    n = 1 << 24
    _note(f"case fp8 bimodal n={n}: drawing states")
    net = synth.make_net(3)
    thermo = synth.make_thermo(3, 29)
    st = synth.make_state(3, n)
    cal = synth.make_state(3, 1 << 14, stream="calibration")
    amax = chem.layer_input_amax(cal.T, cal.P, cal.Y, net).astype(np.float32)
    act_s = chem.pow2_scale(amax.astype(np.float64))
    w_s = chem.pow2_scale(chem.weight_amax(net))
    idx = synth.subsample_indices(3, n, 4096)
    T = torch.tensor(st.T, device="cuda")
    P = torch.tensor(st.P, device="cuda")
    Y = torch.tensor(st.Y, device="cuda")
    idx_t = torch.tensor(idx, device="cuda")
    Ts, Ps, Ys = st.T[idx], st.P[idx], st.Y[:, idx]
    del st
    ex = chem.step(Ts, Ps, Ys, net, thermo=thermo)
    res = {}
    for prec in ("fp8", "bf16", "fp32"):
        _note(f"  running {prec}")
        h = make_handle(net, prec, thermo=thermo, act_amax=amax if prec == "fp8" else None)
        res[prec] = _sample_run(h, T, P, Y, idx_t)
        h.close()
        assert res[prec][2] == 0
        _note(f"  {prec}: max abs dY vs FP64 {np.abs(res[prec][0] - ex['Y_new']).max():.2e}, "
              f"dT {np.abs(res[prec][1] - ex['T_new']).max():.2e} K")
    emu = chem.step(Ts, Ps, Ys, net, fmt="e4m3", act_scale=act_s, w_scale=w_s, thermo=thermo)
    _check_against_emulation(res["fp8"][0], res["fp8"][1], emu, ex, "fp8")
    # the FP32 path stays within the small-batch FP32 bound on the sample
    e32 = np.max(_rel(res["fp32"][0], ex["Y_new"]))
    assert e32 <= 1e-5, e32
    # FP8 is further from FP64 than BF16, and the difference FP8 - BF16 is
    # of the size of the FP8 quantisation error
    d8 = np.abs(res["fp8"][0] - ex["Y_new"]).max()
    d16 = np.abs(res["bf16"][0] - ex["Y_new"]).max()
    _note(f"  max abs dY: fp8 {d8:.2e}  bf16 {d16:.2e}  fp8-bf16 "
          f"{np.abs(res['fp8'][0] - res['bf16'][0]).max():.2e}")
    assert d16 <= d8


def test_block_2p27_sampled():
    """The 512^3 block (smooth fields, LOX/CH4-like compositions), BF16 and
    FP8, drawn on the device; 2048 sampled cells against the emulation."""
    edge = 512
    n = edge ** 3
    free, total = torch.cuda.mem_get_info()
    need = n * (29 + 2) * 8 * 2 + (1 << 34)
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} free")
    _note(f"case block n={n}: drawing states on the device")
    net = synth.make_net(5)
    thermo = synth.make_thermo(5, 29)
    T, P, Y = synth.make_block_state_device(5, edge, 29, device="cuda")
    idx = synth.subsample_indices(5, n, 2048)
    idx_t = torch.tensor(idx, device="cuda")
    Ts, Ps, Ys = T[idx_t].cpu().numpy(), P[idx_t].cpu().numpy(), Y[:, idx_t].cpu().numpy()
    cal_idx = synth.subsample_indices(5, n, 1 << 14)
    cal_t = torch.tensor(cal_idx, device="cuda")
    Tc, Pc, Yc = T[cal_t].cpu().numpy(), P[cal_t].cpu().numpy(), Y[:, cal_t].cpu().numpy()
    amax = chem.layer_input_amax(Tc, Pc, Yc, net).astype(np.float32)
    act_s = chem.pow2_scale(amax.astype(np.float64))
    w_s = chem.pow2_scale(chem.weight_amax(net))
    ex = chem.step(Ts, Ps, Ys, net, thermo=thermo)
    for prec, fmt in (("bf16", "bf16"), ("fp8", "e4m3")):
        _note(f"  running {prec}")
        h = make_handle(net, prec, thermo=thermo, act_amax=amax if prec == "fp8" else None)
        Yg, Tg, nbad = _sample_run(h, T, P, Y, idx_t)
        h.close()
        assert nbad == 0
        emu = chem.step(Ts, Ps, Ys, net, fmt=fmt, act_scale=act_s if prec == "fp8" else None,
                        w_scale=w_s if prec == "fp8" else None, thermo=thermo)
        _check_against_emulation(Yg, Tg, emu, ex, prec)
        np.testing.assert_allclose(Yg.sum(axis=0), 1.0, atol=1e-13)
