"""GPU parity of the property networks (the paper's PRNet sizes,
3-1024-512-256-1 and 3-2048-1024-512-4) through chem_prop_eval against the
FP64 oracle (oracle/prop.py).  The density net (workload 7) runs in the fused
kernel's property mode, the transport net (workload 8) layer by layer."""
import sys

import numpy as np
import pytest

import synth
from oracle import prop

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _handle(net, prec, params=None):
    from paper_2508_18969_amd import PropNet
    if params is None:
        params = torch.tensor(net.flat_params(), device="cuda")
    return PropNet(net.widths, prec, params, net.in_mean, net.in_std, net.out_mean, net.out_std)


def _o(y, net):
    """Network output recovered from the scaled outputs (FP64)."""
    return (y - net.out_mean[:, None]) / net.out_std[:, None]


@pytest.mark.parametrize("cfg", [7, 8])
def test_fp32_matches_fp64_oracle(cfg):
    """FP32 operands: per cell |o - o_ref| <= 1e-5 max(1, max_k |o_ref,k|), the
    chemistry path's FP32 bar, on a ragged batch."""
    net = synth.make_prop_net(cfg)
    n = 1000 + 7
    _note(f"case prop fp32 cfg={cfg} widths={net.widths} n={n}")
    x = synth.make_prop_inputs(cfg, n)
    h = _handle(net, "fp32")
    y = h.eval(torch.tensor(x, device="cuda"))
    torch.cuda.synchronize()
    ref = prop.evaluate(x, net)
    og = _o(y.cpu().numpy(), net)
    err = np.abs(og - ref["o"]).max(axis=0) / np.maximum(1.0, np.abs(ref["o"]).max(axis=0))
    _note(f"  max rel err {err.max():.3e}")
    assert err.max() <= 1e-5


@pytest.mark.parametrize("cfg", [7, 8])
@pytest.mark.parametrize("prec,fmt", [("bf16", "bf16"), ("fp16", "f16")])
def test_narrow_matches_emulation(cfg, prec, fmt):
    """BF16 / FP16 operands against the oracle with the same operand rounding.
    As for the chemistry net's layer-by-layer path, activations whose exact
    value lies within the FP32 accumulation error of a rounding boundary round
    one ulp apart on the two sides (a fraction near 2 sqrt(K) 2^-24 / ulp), so
    the deviation from the emulation is a fraction of the quantisation error
    itself (expected near 0.1 for BF16 and 0.35 for FP16 in RMS at K = 2048).
    Bars: 0.6x in RMS and median, 1x at the 99th percentile, 1.5x at the
    maximum; a rounding mistake gives deviations of the quantisation error's
    own size or more."""
    net = synth.make_prop_net(cfg)
    n = 2048 + 5
    _note(f"case prop {prec} cfg={cfg} n={n}")
    x = synth.make_prop_inputs(cfg, n)
    h = _handle(net, prec)
    y = h.eval(torch.tensor(x, device="cuda"))
    torch.cuda.synchronize()
    og = _o(y.cpu().numpy(), net)
    emu = prop.evaluate(x, net, fmt=fmt)["o"]
    ex = prop.evaluate(x, net)["o"]
    ge, ee = np.abs(og - emu).ravel(), np.abs(emu - ex).ravel()
    _note(f"  gpu-emu rms {np.sqrt(np.mean(ge ** 2)):.2e} med {np.median(ge):.2e} max {ge.max():.2e} | "
          f"emu-fp64 rms {np.sqrt(np.mean(ee ** 2)):.2e} med {np.median(ee):.2e} max {ee.max():.2e}")
    assert np.sqrt(np.mean(ge ** 2)) <= 0.6 * np.sqrt(np.mean(ee ** 2))
    assert np.median(ge) <= 0.6 * np.median(ee)
    assert np.quantile(ge, 0.99) <= 1.0 * np.quantile(ee, 0.99)
    assert ge.max() <= 1.5 * ee.max()


@pytest.mark.parametrize("cfg", [7, 8])
def test_chunks_strides_and_cell_independence(cfg):
    """A batch over many tiles (fused) or past a chunk of 65,536 cells
    (layer by layer) with a ragged tail and a leading dimension above n: a
    cell's outputs do not depend on its batch (bit for bit), and a
    non-finite input spoils only its own cell."""
    net = synth.make_prop_net(cfg)
    n, ld = 65536 + 1300, 65536 + 1300 + 5
    _note(f"case prop chunks cfg={cfg} n={n} ld={ld}")
    x = synth.make_prop_inputs(cfg, n)
    bad = 66000
    x[1, bad] = np.nan
    xd = torch.zeros((3, ld), dtype=torch.float64, device="cuda")
    xd[:, :n] = torch.tensor(x, device="cuda")
    h = _handle(net, "bf16")
    y = h.eval(xd[:, :n])
    sub = slice(65000, 66600)
    ys = h.eval(xd[:, sub].contiguous())
    torch.cuda.synchronize()
    yc = y.cpu().numpy()
    assert y.stride(0) == ld
    assert np.array_equal(ys.cpu().numpy(), yc[:, sub], equal_nan=True)
    fin = np.isfinite(yc).all(axis=0)
    assert not fin[bad] and fin.sum() == n - 1
    # sampled cells against the exact oracle, within the BF16 emulation's own deviation
    idx = synth.subsample_indices(cfg, n, 512)
    idx = idx[idx != bad]
    og = _o(yc[:, idx], net)
    emu = prop.evaluate(x[:, idx], net, fmt="bf16")["o"]
    ex = prop.evaluate(x[:, idx], net)["o"]
    assert np.abs(og - ex).max() <= 1.5 * np.abs(emu - ex).max() + 1e-6


@pytest.mark.parametrize("cfg", [7, 8])
@pytest.mark.parametrize("prec,fmt", [("bf16", "bf16"), ("fp16", "f16")])
def test_full_batch_sampled(cfg, prec, fmt):
    """The benchmark's batch of 2^20 cells in BF16 and FP16, sampled cells
    against the oracle with the statistical bars of the emulation test."""
    net = synth.make_prop_net(cfg)
    n = 1 << 20
    _note(f"case prop full cfg={cfg} {prec} n={n}")
    x = synth.make_prop_inputs(cfg, n)
    h = _handle(net, prec)
    y = h.eval(torch.tensor(x, device="cuda"))
    torch.cuda.synchronize()
    idx = synth.subsample_indices(cfg, n, 1024)
    og = _o(y[:, torch.tensor(idx, device="cuda")].cpu().numpy(), net)
    emu = prop.evaluate(x[:, idx], net, fmt=fmt)["o"]
    ex = prop.evaluate(x[:, idx], net)["o"]
    ge, ee = np.abs(og - emu).ravel(), np.abs(emu - ex).ravel()
    _note(f"  gpu-emu rms {np.sqrt(np.mean(ge ** 2)):.2e} | emu-fp64 rms {np.sqrt(np.mean(ee ** 2)):.2e}")
    assert np.isfinite(y.cpu().numpy()).all()
    assert np.sqrt(np.mean(ge ** 2)) <= 0.6 * np.sqrt(np.mean(ee ** 2))
    assert np.quantile(ge, 0.99) <= 1.0 * np.quantile(ee, 0.99)
    assert ge.max() <= 1.5 * ee.max()


@pytest.mark.parametrize("cfg", [7, 8])
def test_single_cell_empty_and_set_params(cfg):
    """n = 1 and n = 0; set_params gives the outputs of a handle built from
    the new parameters (bit for bit), on both paths."""
    net = synth.make_prop_net(cfg)
    _note(f"case prop n=1, n=0, set_params cfg={cfg}")
    x = synth.make_prop_inputs(cfg, 300)
    h = _handle(net, "fp32")
    y1 = h.eval(torch.tensor(x[:, :1], device="cuda"))
    torch.cuda.synchronize()
    ref = prop.evaluate(x[:, :1], net)["o"]
    assert abs(_o(y1.cpu().numpy(), net) - ref).max() <= 1e-5 * max(1.0, abs(ref).max())
    h.eval(torch.empty((3, 0), dtype=torch.float64, device="cuda"))
    p2 = torch.tensor(net.flat_params() * np.float32(0.75), device="cuda")
    for prec in ("fp32", "bf16"):
        ha = _handle(net, prec)
        ha.set_params(p2)
        hb = _handle(net, prec, params=p2)
        xd = torch.tensor(x, device="cuda")
        ya, yb = ha.eval(xd), hb.eval(xd)
        torch.cuda.synchronize()
        assert torch.equal(ya, yb), prec


def test_binding_rejects_aliasing_and_layouts():
    from paper_2508_18969_amd import ChemDNNError
    net = synth.make_prop_net(8)
    h = _handle(net, "bf16")
    x = torch.zeros((3, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        h.eval(x.t().contiguous().t())                    # cell index not fastest
    buf = torch.zeros((8, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(ChemDNNError):
        h.eval(buf[:3], y=buf[2:6])                       # overlapping input and output


@pytest.mark.parametrize("widths", [(32, 1024, 512, 256, 30), (32, 1024, 512, 256, 32), (1, 256, 256, 1)])
def test_input_and_output_limits(widths):
    """The largest input and output counts: 32 inputs and 30 outputs still
    run in the fused kernel (its output rows are 2 .. 31), 32 outputs on the
    layer-by-layer path; and the smallest net, one input and one output.
    FP32 operands against the FP64 oracle (the FP32 bar), with random non-zero
    biases and input statistics of a seeded draw."""
    rng = np.random.default_rng(sum(widths))
    n = 777
    D, K = widths[0], widths[-1]
    _note(f"case prop limits widths={widths} n={n}")
    x = rng.normal(size=(D, n)) * rng.uniform(0.5, 5.0, size=(D, 1)) + rng.normal(size=(D, 1)) * 10
    net = synth.make_prop_net(7, widths=widths, bias_scale=0.1)
    net.in_mean, net.in_std = x.mean(axis=1), x.std(axis=1)
    net.out_mean, net.out_std = rng.normal(size=K), rng.uniform(0.5, 2.0, size=K)
    h = _handle(net, "fp32")
    y = h.eval(torch.tensor(x, device="cuda"))
    torch.cuda.synchronize()
    ref = prop.evaluate(x, net)
    og = _o(y.cpu().numpy(), net)
    err = np.abs(og - ref["o"]).max(axis=0) / np.maximum(1.0, np.abs(ref["o"]).max(axis=0))
    _note(f"  max rel err {err.max():.3e}")
    assert err.max() <= 1e-5
