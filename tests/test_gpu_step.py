"""GPU parity of the chemistry update (chem_dnn_step through the C ABI)
against the FP64 oracle on seeded inputs."""
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


def _run(h, st, ld=None):
    T, P, Y = dev_state(st, ld=ld)
    nbad = torch.zeros(1, dtype=torch.int32, device="cuda")
    Yn, Tn = h.step(T, P, Y, n_bad=nbad)
    torch.cuda.synchronize()
    return Yn.cpu().numpy(), (Tn.cpu().numpy() if Tn is not None else None), int(nbad.item())


# ------------------------------------------------------------------ FP32 paths vs FP64
@pytest.mark.parametrize("n", [4096, 4096 - 37, 1, 33])
def test_small_net_fp32_matches_fp64_oracle(n):
    """17-species net, FP32 operands: Y_new within 1e-5 relative (floor 1e-10)
    and T_new within 1e-5 relative of the FP64 oracle; several tiles and a
    ragged tail."""
    _note(f"case small fp32 n={n}")
    net = synth.make_net(1)
    thermo = synth.make_thermo(1, 17)
    st = synth.make_state(1, n)
    h = make_handle(net, "fp32", thermo=thermo)
    Yg, Tg, nbad = _run(h, st)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    assert nbad == 0
    e_y = rel_err(Yg, ref["Y_new"])
    e_t = rel_err(Tg, ref["T_new"], floor=1.0)
    _note(f"  rel err Y {e_y:.3e}  T {e_t:.3e}")
    assert e_y <= 1e-5
    assert e_t <= 1e-5
    np.testing.assert_allclose(Yg.sum(axis=0), 1.0, atol=1e-13)


def test_large_net_fp32_matches_fp64_oracle():
    _note("case large fp32 n=2048+5")
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    st = synth.make_state(2, 2048 + 5)
    h = make_handle(net, "fp32", thermo=thermo)
    Yg, Tg, _ = _run(h, st)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    e_y = rel_err(Yg, ref["Y_new"])
    e_t = rel_err(Tg, ref["T_new"], floor=1.0)
    _note(f"  rel err Y {e_y:.3e}  T {e_t:.3e}")
    assert e_y <= 1e-5
    assert e_t <= 1e-5


# ------------------------------------------------------------------ narrow formats
def _rel(a, b, floor=1e-10):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


@pytest.mark.parametrize("prec,fmt", [("bf16", "bf16"), ("fp16", "f16")])
def test_large_net_narrow_matches_emulation(prec, fmt):
    """29-species net with bf16 / fp16 operands against the oracle that rounds
    the same operands (FP64 arithmetic otherwise).

    The two sides round activations that differ by FP32 accumulation error, so
    an activation near a rounding boundary can land one narrow-format ulp apart
    (a "flip"); each flip moves a cell's output by a fraction of one ulp.  The
    bar: the GPU's deviation from the emulation is a small fraction of the
    quantisation error itself (emulation vs exact FP64) in RMS, median, 99th
    percentile and maximum.  The error against exact FP64 is printed."""
    _note(f"case large {prec} n=4096+11")
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    st = synth.make_state(2, 4096 + 11)
    h = make_handle(net, prec, thermo=thermo)
    Yg, Tg, _ = _run(h, st)
    emu = chem.step(st.T, st.P, st.Y, net, fmt=fmt, thermo=thermo)
    ex = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    ge, ee = Yg - emu["Y_new"], emu["Y_new"] - ex["Y_new"]
    rg, re = _rel(Yg, emu["Y_new"]), _rel(emu["Y_new"], ex["Y_new"])
    rms_g, rms_e = np.sqrt(np.mean(ge ** 2)), np.sqrt(np.mean(ee ** 2))
    _note(f"  gpu-emu: rms {rms_g:.2e} med {np.median(rg):.2e} p99 {np.quantile(rg, .99):.2e} "
          f"max {rg.max():.2e} T {np.abs(Tg - emu['T_new']).max():.2e} | "
          f"emu-fp64: rms {rms_e:.2e} med {np.median(re):.2e} p99 {np.quantile(re, .99):.2e} "
          f"max {re.max():.2e} | gpu-fp64 max abs dY {np.abs(Yg - ex['Y_new']).max():.2e} "
          f"T {np.abs(Tg - ex['T_new']).max():.2e} K")
    assert rms_g <= 0.25 * rms_e
    assert np.median(rg) <= 0.05 * np.median(re)
    assert np.quantile(rg, 0.99) <= 0.5 * np.quantile(re, 0.99)
    assert rg.max() <= 0.5 * re.max()
    tg, te = Tg - emu["T_new"], emu["T_new"] - ex["T_new"]
    assert np.sqrt(np.mean(tg ** 2)) <= 0.25 * np.sqrt(np.mean(te ** 2))
    assert np.abs(tg).max() <= np.abs(te).max()


def _fp8_setup(config, n_cal=1 << 14):
    """Net and its FP8 scales from the oracle: per-layer input amax of the
    exact forward over a separate calibration draw, weight amax, and the
    power-of-two scales of both.  The amax goes to the GPU as an input."""
    net = synth.make_net(config)
    cal = synth.make_state(config, n_cal, stream="calibration")
    amax = chem.layer_input_amax(cal.T, cal.P, cal.Y, net).astype(np.float32)
    act_s = chem.pow2_scale(amax.astype(np.float64))
    w_s = chem.pow2_scale(chem.weight_amax(net))
    return net, amax, act_s, w_s


@pytest.mark.parametrize("config", [1, 2])
def test_fp8_scales_match_oracle(config):
    """The library's power-of-two activation and weight scales equal the
    oracle's, bit for bit."""
    _note(f"case fp8 scales config={config}")
    net, amax, act_s, w_s = _fp8_setup(config)
    h = make_handle(net, "fp8", act_amax=amax)
    a, w = h.scales()
    np.testing.assert_array_equal(a.astype(np.float64), act_s)
    np.testing.assert_array_equal(w.astype(np.float64), w_s)


@pytest.mark.parametrize("config,n", [(1, 4096 - 5), (2, 4096 + 11)])
def test_fp8_matches_emulation(config, n):
    """FP8 e4m3 operands with per-layer scales against the oracle that rounds
    the same scaled operands; same statistical bar as the 16-bit formats
    (a rounding flip is rarer but larger in e4m3)."""
    _note(f"case fp8 config={config} n={n}")
    net, amax, act_s, w_s = _fp8_setup(config)
    S = 17 if config == 1 else 29
    thermo = synth.make_thermo(config, S)
    st = synth.make_state(config, n)
    h = make_handle(net, "fp8", thermo=thermo, act_amax=amax)
    Yg, Tg, nbad = _run(h, st)
    assert nbad == 0
    emu = chem.step(st.T, st.P, st.Y, net, fmt="e4m3", act_scale=act_s, w_scale=w_s, thermo=thermo)
    ex = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    ge, ee = Yg - emu["Y_new"], emu["Y_new"] - ex["Y_new"]
    rg, re = _rel(Yg, emu["Y_new"]), _rel(emu["Y_new"], ex["Y_new"])
    rms_g, rms_e = np.sqrt(np.mean(ge ** 2)), np.sqrt(np.mean(ee ** 2))
    _note(f"  gpu-emu: rms {rms_g:.2e} med {np.median(rg):.2e} p99 {np.quantile(rg, .99):.2e} "
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
    np.testing.assert_allclose(Yg.sum(axis=0), 1.0, atol=1e-13)


# ------------------------------------------------------------------ tabulated GELU
@pytest.mark.parametrize("config,n", [(1, 4096 - 3), (2, 2048 + 5)])
def test_gelu_table_fp32_matches_oracle(config, n):
    """FP32 operands with the tabulated GELU (Sec. 3.3.2) against the FP64
    oracle evaluating the same table: the same 1e-5 bound as the tanh form."""
    _note(f"case gelu table fp32 config={config} n={n}")
    net = synth.make_net(config)
    S = 17 if config == 1 else 29
    thermo = synth.make_thermo(config, S)
    st = synth.make_state(config, n)
    h = make_handle(net, "fp32", thermo=thermo, gelu="table")
    Yg, Tg, nbad = _run(h, st)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo, act=chem.gelu_table)
    assert nbad == 0
    e_y = rel_err(Yg, ref["Y_new"])
    e_t = rel_err(Tg, ref["T_new"], floor=1.0)
    exact = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    _note(f"  rel err Y {e_y:.3e}  T {e_t:.3e} | table vs tanh form (oracle): max abs dY "
          f"{np.abs(ref['Y_new'] - exact['Y_new']).max():.2e}")
    assert e_y <= 1e-5
    assert e_t <= 1e-5


def test_gelu_table_bf16_matches_emulation():
    """BF16 operands with the tabulated GELU against the emulation with the
    same table; the statistical bar of the narrow formats."""
    _note("case gelu table bf16 n=4096+11")
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    st = synth.make_state(2, 4096 + 11)
    h = make_handle(net, "bf16", thermo=thermo, gelu="table")
    Yg, Tg, _ = _run(h, st)
    emu = chem.step(st.T, st.P, st.Y, net, fmt="bf16", thermo=thermo, act=chem.gelu_table)
    ex = chem.step(st.T, st.P, st.Y, net, thermo=thermo, act=chem.gelu_table)
    ge, ee = Yg - emu["Y_new"], emu["Y_new"] - ex["Y_new"]
    rg, re = _rel(Yg, emu["Y_new"]), _rel(emu["Y_new"], ex["Y_new"])
    rms_g, rms_e = np.sqrt(np.mean(ge ** 2)), np.sqrt(np.mean(ee ** 2))
    _note(f"  gpu-emu: rms {rms_g:.2e} med {np.median(rg):.2e} max {rg.max():.2e} | "
          f"emu-fp64: rms {rms_e:.2e} med {np.median(re):.2e} max {re.max():.2e}")
    assert rms_g <= 0.25 * rms_e
    assert np.median(rg) <= 0.05 * np.median(re)
    assert np.quantile(rg, 0.99) <= 0.5 * np.quantile(re, 0.99)
    assert rg.max() <= 0.5 * re.max()


def _table_boundary_cells(st, net, delta=2e-6):
    """Cells with a hidden pre-activation (FP64 forward with the table)
    within delta of an interval boundary -3 + 0.01 k of the table (or of its
    ends): there the FP32 pre-activation may fall in the neighbouring
    interval.  The FP16 table jumps at a boundary by up to its coefficient
    rounding (about 1e-3), the FP32 table by about 1e-8."""
    a = chem.features(st.T, st.P, st.Y, net.in_mean, net.in_std, net.lam)
    near = np.zeros(st.n, bool)
    for l, (W, b) in enumerate(zip(net.W, net.b)):
        z = np.asarray(W, np.float64) @ a + np.asarray(b, np.float64)[:, None]
        if l == len(net.W) - 1:
            break
        u = (z + 3.0) * 100.0
        near |= np.any((np.abs(u - np.round(u)) < 100.0 * delta) & (np.abs(z) <= 3.0 + delta), axis=0)
        a = chem.gelu_table16(z)
    return near


@pytest.mark.parametrize("config,n", [(1, 4096 - 3), (2, 2048 + 5)])
def test_gelu_table16_fp32_matches_oracle(config, n):
    """FP32 operands with the FP16-coefficient table (Sec. 3.3.2: FP16
    tabulation) against the FP64 oracle evaluating the same FP16
    coefficients.  The table is discontinuous at its interval boundaries by
    up to the coefficient rounding (about 1e-3): a pre-activation that the
    FP32 accumulation leaves within about 1e-7 of a boundary may take the
    neighbouring interval's polynomial on one side.  So: 1e-5 relative on
    every cell without a pre-activation within 2e-6 of a boundary; the
    others (counted) must stay within the jump's effect, 1e-3 relative."""
    _note(f"case gelu table16 fp32 config={config} n={n}")
    net = synth.make_net(config)
    S = 17 if config == 1 else 29
    thermo = synth.make_thermo(config, S)
    st = synth.make_state(config, n)
    h = make_handle(net, "fp32", thermo=thermo, gelu="table16")
    Yg, Tg, nbad = _run(h, st)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo, act=chem.gelu_table16)
    assert nbad == 0
    near = _table_boundary_cells(st, net)
    ok = ~near
    e_y = rel_err(Yg[:, ok], ref["Y_new"][:, ok])
    e_t = rel_err(Tg[ok], ref["T_new"][ok], floor=1.0)
    e_near = rel_err(Yg[:, near], ref["Y_new"][:, near]) if near.any() else 0.0
    exact = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    _note(f"  {near.sum()} of {st.n} cells have a pre-activation near a table boundary (rel err Y "
          f"{e_near:.2e}); the others: rel err Y {e_y:.3e}  T {e_t:.3e} | FP16 table vs tanh form "
          f"(oracle): max abs dY {np.abs(ref['Y_new'] - exact['Y_new']).max():.2e}, "
          f"dT {np.abs(ref['T_new'] - exact['T_new']).max():.2e} K")
    assert e_y <= 1e-5
    assert e_t <= 1e-5
    assert e_near <= 1e-3


def test_gelu_table16_bf16_matches_emulation():
    """BF16 operands with the FP16-coefficient table against the emulation
    with the same table; the statistical bar of the narrow formats."""
    _note("case gelu table16 bf16 n=4096+11")
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    st = synth.make_state(2, 4096 + 11)
    h = make_handle(net, "bf16", thermo=thermo, gelu="table16")
    Yg, Tg, _ = _run(h, st)
    emu = chem.step(st.T, st.P, st.Y, net, fmt="bf16", thermo=thermo, act=chem.gelu_table16)
    ex = chem.step(st.T, st.P, st.Y, net, thermo=thermo, act=chem.gelu_table16)
    ge, ee = Yg - emu["Y_new"], emu["Y_new"] - ex["Y_new"]
    rg, re = _rel(Yg, emu["Y_new"]), _rel(emu["Y_new"], ex["Y_new"])
    rms_g, rms_e = np.sqrt(np.mean(ge ** 2)), np.sqrt(np.mean(ee ** 2))
    _note(f"  gpu-emu: rms {rms_g:.2e} med {np.median(rg):.2e} max {rg.max():.2e} | "
          f"emu-fp64: rms {rms_e:.2e} med {np.median(re):.2e} max {re.max():.2e}")
    assert rms_g <= 0.25 * rms_e
    assert np.median(rg) <= 0.05 * np.median(re)
    assert np.quantile(rg, 0.99) <= 0.5 * np.quantile(re, 0.99)
    assert rg.max() <= 0.5 * re.max()


# ------------------------------------------------------------------ source terms
@pytest.mark.parametrize("config,n", [(1, 4096 + 5), (2, 2053)])
def test_source_terms_match_oracle(config, n):
    """FP32: omega against the oracle's source terms of its own step.  omega dt
    / rho is Y_new - Y, so the bar is that of Y_new (1e-5 relative).  Y_out and
    T_out are those of chem_dnn_step, bit for bit."""
    _note(f"case source terms config={config} n={n}")
    net = synth.make_net(config)
    S = 17 if config == 1 else 29
    thermo = synth.make_thermo(config, S)
    W = synth.make_molar_masses(config, S)
    st = synth.make_state(config, n)
    h = make_handle(net, "fp32", thermo=thermo, molar_mass=W)
    T, P, Y = dev_state(st)
    dt = 1e-6
    Yo, To, om = h.step_source(T, P, Y, dt)
    Y2, T2 = h.step(T, P, Y)
    torch.cuda.synchronize()
    assert torch.equal(Yo, Y2) and torch.equal(To, T2)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    om_ref = chem.source_terms(st.T, st.P, st.Y, ref["Y_new"], W, dt)
    rho = chem.mixture_density(st.T, st.P, st.Y, W)
    omg = om.cpu().numpy()
    e = np.abs(omg - om_ref) * dt / rho[None, :]
    bound = 1e-5 * np.maximum(np.abs(ref["Y_new"]), 1e-10)
    _note(f"  max |d omega| dt/rho / bound = {np.max(e / bound):.3f}")
    assert np.all(e <= bound)
    # mass conservation of the exported terms, relative to rho / dt
    assert np.max(np.abs(omg.sum(axis=0)) * dt / rho) < 1e-12


def test_source_terms_narrow_and_bad_cells():
    """BF16: omega is the GPU's own Y change times rho / dt; cells passed
    through as bad get zero source terms."""
    _note("case source terms bf16 + bad cells")
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    W = synth.make_molar_masses(2, 29)
    st = synth.make_state(2, 1000)
    st.T[7] = np.nan
    st.Y[3, 11] = np.inf
    h = make_handle(net, "bf16", thermo=thermo, molar_mass=W)
    T, P, Y = dev_state(st)
    nb = torch.zeros(1, dtype=torch.int32, device="cuda")
    Yo, To, om = h.step_source(T, P, Y, 2e-6, n_bad=nb)
    torch.cuda.synchronize()
    assert int(nb.item()) == 2
    omg, yo = om.cpu().numpy(), Yo.cpu().numpy()
    assert not np.any(omg[:, [7, 11]])
    ok = np.ones(1000, bool)
    ok[[7, 11]] = False
    rho = chem.mixture_density(st.T[ok], st.P[ok], st.Y[:, ok], W)
    np.testing.assert_allclose(omg[:, ok] * 2e-6 / rho[None, :], yo[:, ok] - st.Y[:, ok],
                               rtol=1e-12, atol=1e-18)


def test_source_terms_full_batch():
    """The benchmark's source-term workload (2^20 cells, BF16): Y_out and
    T_out bit-identical to chem_dnn_step's; at 1,024 sampled cells omega is
    rho / dt times the kernel's own change (1e-12), the source terms of a
    cell sum to zero (mass conservation of the renormalised update)."""
    n, dt = 1 << 20, 1e-6
    _note(f"case source terms full batch bf16 n={n}")
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    W = synth.make_molar_masses(2, 29)
    st = synth.make_state(2, n)
    h = make_handle(net, "bf16", thermo=thermo, molar_mass=W)
    T, P, Y = dev_state(st)
    Yo, To, om = h.step_source(T, P, Y, dt)
    Ys, Ts = h.step(T, P, Y)
    torch.cuda.synchronize()
    assert torch.equal(Yo, Ys) and torch.equal(To, Ts)
    idx = synth.subsample_indices(2, n, 1024)
    it = torch.tensor(idx, device="cuda")
    omg, yo = om[:, it].cpu().numpy(), Yo[:, it].cpu().numpy()
    rho = chem.mixture_density(st.T[idx], st.P[idx], st.Y[:, idx], W)
    np.testing.assert_allclose(omg * dt / rho[None, :], yo - st.Y[:, idx], rtol=1e-12, atol=1e-18)
    assert np.all(np.abs(omg.sum(axis=0)) <= 1e-12 * rho / dt)


# ------------------------------------------------------------------ properties
def test_cells_are_independent_and_runs_deterministic():
    _note("case independence bf16")
    net = synth.make_net(2)
    st = synth.make_state(2, 300)
    h = make_handle(net, "bf16")
    Y1, _, _ = _run(h, st)
    Y2, _, _ = _run(h, st)
    assert np.array_equal(Y1, Y2)
    one = synth.State(st.T[17:18].copy(), st.P[17:18].copy(), st.Y[:, 17:18].copy())
    Yo, _, _ = _run(h, one)
    assert np.array_equal(Yo[:, 0], Y1[:, 17])


def test_padded_leading_dimension_and_in_place():
    _note("case ld/in-place fp32 small")
    net = synth.make_net(1)
    st = synth.make_state(1, 200)
    h = make_handle(net, "fp32")
    Yref, _, _ = _run(h, st)
    T, P, Y = dev_state(st, ld=256)
    assert Y.stride(0) == 256
    h.step(T, P, Y, Y_out=Y)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Y.cpu().numpy(), Yref)


def test_bad_cells_pass_through():
    _note("case bad cells")
    net = synth.make_net(1)
    thermo = synth.make_thermo(1, 17)
    st = synth.make_state(1, 64)
    st.T[3] = np.nan
    st.Y[5, 9] = np.inf
    st.P[20] = -np.inf
    h = make_handle(net, "fp32", thermo=thermo)
    Yg, Tg, nbad = _run(h, st)
    assert nbad == 3
    for c in (3, 9, 20):
        np.testing.assert_array_equal(Yg[:, c], st.Y[:, c])
    assert np.isnan(Tg[3])
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    good = ~ref["bad"]
    assert rel_err(Yg[:, good], ref["Y_new"][:, good]) <= 1e-5


def test_zero_and_tiny_mass_fractions():
    """Y = 0 and Y far below FLT_MIN take the exponent-split path."""
    _note("case tiny Y")
    net = synth.make_net(1)
    st = synth.make_state(1, 128)
    st.Y[0, :32] = 0.0
    st.Y[1, 32:64] = 1e-300
    st.Y[2, 64:96] = 1e-45
    st.Y /= st.Y.sum(axis=0)
    h = make_handle(net, "fp32")
    Yg, _, nbad = _run(h, st)
    ref = chem.step(st.T, st.P, st.Y, net)
    assert nbad == 0
    assert rel_err(Yg, ref["Y_new"]) <= 1e-5


def test_empty_batch_is_noop():
    net = synth.make_net(1)
    h = make_handle(net, "fp32")
    T = torch.zeros(0, dtype=torch.float64, device="cuda")
    Y = torch.zeros((17, 0), dtype=torch.float64, device="cuda")
    h.step(T, T, Y)
    torch.cuda.synchronize()
