"""GPU parity of the layer-by-layer path (networks outside the fused
kernel's shapes), on the ODENet size of the paper's runs,
19-2048-4096-2048-1024-512-17, against the FP64 oracle."""
import sys

import numpy as np
import pytest

import synth
from oracle import chem
from tests.helpers import dev_state, make_handle, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def net():
    return synth.make_net(6)


def _rel(a, b, floor=1e-10):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def test_fp32_matches_fp64_oracle(net):
    """FP32 operands through six layers with K up to 4096: the output carries
    about sqrt(K) 2^-24 relative error per layer; the bar on Y_new and T_new is
    the fused path's 1e-5 relative."""
    n = 1000 + 7
    _note(f"case layered fp32 n={n}")
    thermo = synth.make_thermo(6, 17)
    st = synth.make_state(6, n)
    h = make_handle(net, "fp32", thermo=thermo)
    T, P, Y = dev_state(st)
    nb = torch.zeros(1, dtype=torch.int32, device="cuda")
    Yn, Tn = h.step(T, P, Y, n_bad=nb)
    torch.cuda.synchronize()
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    e_y = rel_err(Yn.cpu().numpy(), ref["Y_new"])
    e_t = rel_err(Tn.cpu().numpy(), ref["T_new"], floor=1.0)
    _note(f"  rel err Y {e_y:.3e}  T {e_t:.3e}")
    assert int(nb.item()) == 0
    assert e_y <= 1e-5 and e_t <= 1e-5


@pytest.mark.parametrize("prec,fmt", [("bf16", "bf16"), ("fp16", "f16")])
def test_narrow_matches_emulation(net, prec, fmt):
    """BF16 / FP16 operands against the oracle with the same operand rounding.
    The two sides accumulate in FP32 and FP64, so an activation whose exact
    value lies within the FP32 accumulation error (about sqrt(K) 2^-24
    relative, K up to 4096) of a rounding boundary rounds one ulp apart: a
    fraction p of about 2 sqrt(K) 2^-24 / ulp of all activations (0.1 % for
    BF16, 0.8 % for FP16), against an error of ulp / sqrt(12) on every
    activation for the quantisation itself.  The deviation from the emulation
    is therefore expected near sqrt(12 p) of the quantisation error in RMS:
    0.11 for BF16 and 0.31 for FP16 (the fused path's shallower, narrower
    net stays under 0.25).  The bar: 0.6x in RMS and median, 1x at the 99th
    percentile, 1.5x at the maximum - a rounding mistake (truncation, a wrong
    format) gives deviations of the quantisation error's own size or more."""
    n = 1024 + 3
    _note(f"case layered {prec} n={n}")
    thermo = synth.make_thermo(6, 17)
    st = synth.make_state(6, n)
    h = make_handle(net, prec, thermo=thermo)
    T, P, Y = dev_state(st)
    Yn, Tn = h.step(T, P, Y)
    torch.cuda.synchronize()
    Yg, Tg = Yn.cpu().numpy(), Tn.cpu().numpy()
    emu = chem.step(st.T, st.P, st.Y, net, fmt=fmt, thermo=thermo)
    ex = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    for got, e, x, name in ((Yg, emu["Y_new"], ex["Y_new"], "Y"), (Tg, emu["T_new"], ex["T_new"], "T")):
        ge, ee = got - e, e - x
        rg, re = _rel(got, e), _rel(e, x)
        rms_g, rms_e = np.sqrt(np.mean(ge ** 2)), np.sqrt(np.mean(ee ** 2))
        _note(f"  {name}: gpu-emu rms {rms_g:.2e} med {np.median(rg):.2e} max {rg.max():.2e} | "
              f"emu-fp64 rms {rms_e:.2e} med {np.median(re):.2e} max {re.max():.2e}")
        assert rms_g <= 0.6 * rms_e
        assert np.median(rg) <= 0.6 * np.median(re)
        assert np.quantile(rg, 0.99) <= 1.0 * np.quantile(re, 0.99)
        assert rg.max() <= 1.5 * re.max()


def test_chunks_cells_independent_and_source_terms(net):
    """Past one chunk (32768 cells) and with a ragged tail: a cell's result
    does not depend on its batch (bit for bit), bad cells pass through, and
    the source terms are rho / dt times the step's own change."""
    n = 32768 + 1200
    _note(f"case layered chunks n={n}")
    thermo = synth.make_thermo(6, 17)
    W = synth.make_molar_masses(6, 17)
    st = synth.make_state(6, n)
    st.T[40000 - 8000] = np.nan
    h = make_handle(net, "bf16", thermo=thermo, molar_mass=W)
    T, P, Y = dev_state(st)
    nb = torch.zeros(1, dtype=torch.int32, device="cuda")
    Yo, To, om = h.step_source(T, P, Y, 1e-6, n_bad=nb)
    sub = slice(32000, 33968)
    Ts, Ps, Ys = T[sub].contiguous(), P[sub].contiguous(), Y[:, sub].contiguous()
    Ys_o, Ts_o = h.step(Ts, Ps, Ys)
    torch.cuda.synchronize()
    assert int(nb.item()) == 1
    assert torch.equal(Ys_o, Yo[:, sub])
    # (the bad cell's T is NaN on both sides: equal as bit patterns)
    assert torch.equal(Ts_o.view(torch.int64), To[sub].view(torch.int64))
    bad = 40000 - 8000
    assert torch.equal(Yo[:, bad], Y[:, bad]) and not torch.any(om[:, bad])
    ok = np.ones(n, bool)
    ok[bad] = False
    rho = chem.mixture_density(st.T[ok], st.P[ok], st.Y[:, ok], W)
    np.testing.assert_allclose(om.cpu().numpy()[:, ok] * 1e-6 / rho[None, :],
                               Yo.cpu().numpy()[:, ok] - st.Y[:, ok], rtol=1e-12, atol=1e-18)


def test_single_cell_and_empty(net):
    _note("case layered n=1 and n=0")
    st = synth.make_state(6, 1)
    h = make_handle(net, "fp32")
    T, P, Y = dev_state(st)
    Yn, _ = h.step(T, P, Y)
    torch.cuda.synchronize()
    ref = chem.step(st.T, st.P, st.Y, net)
    assert rel_err(Yn.cpu().numpy(), ref["Y_new"]) <= 1e-5
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    h.step(e, e, torch.empty((17, 0), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()


def test_training_is_not_offered(net):
    """Training entry points cover the fused shapes only."""
    from paper_2508_18969_amd import binding
    with pytest.raises(binding.ChemDNNError) as e:
        make_handle(net, "fp32", max_batch=1024)
    assert e.value.status == binding.EUNSUPPORTED


def test_set_params_repacks_every_layer(net):
    """chem_dnn_set_params on a layer-by-layer handle: the result equals a
    handle built from the new parameters, bit for bit."""
    import dataclasses
    _note("case layered set_params")
    st = synth.make_state(6, 300)
    rng = np.random.default_rng(5)
    W2 = [w * np.float32(1.0 + 0.1 * rng.standard_normal()) for w in net.W]
    b2 = [(x + np.float32(0.01) * rng.standard_normal(x.shape)).astype(np.float32) for x in net.b]
    other = dataclasses.replace(net, W=W2, b=b2)
    h = make_handle(net, "bf16")
    p2 = torch.tensor(other.flat_params(), device="cuda")
    h.set_params(p2)
    T, P, Y = dev_state(st)
    Ya, _ = h.step(T, P, Y)
    hb = make_handle(other, "bf16")
    Yb, _ = hb.step(T, P, Y)
    torch.cuda.synchronize()
    assert torch.equal(Ya, Yb)


def test_full_batch_sampled(net):
    """The benchmark's batch (2^20 cells, 32 chunks) in BF16: 512 sampled
    cells against the oracle with the same operand rounding, with the bars of
    the emulation test above, and no bad cells."""
    n = 1 << 20
    _note(f"case layered full batch bf16 n={n}")
    thermo = synth.make_thermo(6, 17)
    st = synth.make_state(6, n)
    h = make_handle(net, "bf16", thermo=thermo)
    T, P, Y = dev_state(st)
    nb = torch.zeros(1, dtype=torch.int32, device="cuda")
    Yn, Tn = h.step(T, P, Y, n_bad=nb)
    torch.cuda.synchronize()
    assert int(nb.item()) == 0
    idx = synth.subsample_indices(6, n, 512)
    it = torch.tensor(idx, device="cuda")
    Yg, Tg = Yn[:, it].cpu().numpy(), Tn[it].cpu().numpy()
    sub = (st.T[idx], st.P[idx], st.Y[:, idx])
    emu = chem.step(*sub, net, fmt="bf16", thermo=thermo)
    ex = chem.step(*sub, net, thermo=thermo)
    for got, e, x, name in ((Yg, emu["Y_new"], ex["Y_new"], "Y"), (Tg, emu["T_new"], ex["T_new"], "T")):
        ge, ee = got - e, e - x
        rg, re = _rel(got, e), _rel(e, x)
        rms_g, rms_e = np.sqrt(np.mean(ge ** 2)), np.sqrt(np.mean(ee ** 2))
        _note(f"  {name}: gpu-emu rms {rms_g:.2e} | emu-fp64 rms {rms_e:.2e}")
        assert rms_g <= 0.6 * rms_e
        assert np.median(rg) <= 0.6 * np.median(re)
        assert np.quantile(rg, 0.99) <= 1.0 * np.quantile(re, 0.99)
        assert rg.max() <= 1.5 * re.max()


def test_largest_species_count():
    """30 species, the most a description takes (32 inputs, output rows up to
    31), on the layer-by-layer path: FP32 against the FP64 oracle (1e-5) with
    the temperature update and the source terms, on a ragged batch."""
    S, n = 30, 777
    _note(f"case layered S={S} n={n}")
    net = synth.make_net(6, widths=(S + 2, 256, 512, S), bias_scale=0.05)
    thermo = synth.make_thermo(6, S)
    W = synth.make_molar_masses(6, S)
    st = synth.make_state(6, n, S=S)
    h = make_handle(net, "fp32", thermo=thermo, molar_mass=W)
    T, P, Y = dev_state(st)
    Yn, Tn, om = h.step_source(T, P, Y, 1e-6)
    torch.cuda.synchronize()
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    assert rel_err(Yn.cpu().numpy(), ref["Y_new"]) <= 1e-5
    assert rel_err(Tn.cpu().numpy(), ref["T_new"], floor=1.0) <= 1e-5
    rho = chem.mixture_density(st.T, st.P, st.Y, W)
    np.testing.assert_allclose(om.cpu().numpy() * 1e-6 / rho[None, :], Yn.cpu().numpy() - st.Y,
                               rtol=1e-12, atol=1e-18)
