"""GPU parity with non-zero biases in every layer and drawn output
statistics (mu_out, sigma_out), on every path: the fused kernel in FP32,
BF16, FP16 and FP8 (both network sizes), the tabulated GELU and the
layer-by-layer path.  The default workload nets have zero biases and the
identity output map, which leaves the bias paths (the accumulator start in
FP32/BF16/FP16, the scaled epilogue fma in FP8) and the output affine map
unchecked.  Also: the contract for non-finite network results, the relative
accuracy of trace species, and the binding's argument checks."""
import sys

import numpy as np
import pytest

import synth
from oracle import chem
from tests.helpers import dev_state, make_handle, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BIAS = 0.1


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _net(config, widths=None):
    return synth.make_net(config, widths=widths, bias_scale=BIAS, out_stats=True)


def _run(h, st):
    T, P, Y = dev_state(st)
    nbad = torch.zeros(1, dtype=torch.int32, device="cuda")
    Yn, Tn = h.step(T, P, Y, n_bad=nbad)
    torch.cuda.synchronize()
    return Yn.cpu().numpy(), (Tn.cpu().numpy() if Tn is not None else None), int(nbad.item())


def _rel(a, b, floor=1e-10):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def _narrow_bar(got, emu, ex, k_rms, k_med, k_p99, k_max, what):
    """The statistical bar of the narrow formats (see the fused and
    layer-by-layer parity tests for its derivation): the deviation from the
    emulation is a fraction of the quantisation error (emulation - FP64)."""
    ge, ee = got - emu, emu - ex
    rg, re = _rel(got, emu), _rel(emu, ex)
    rms_g, rms_e = np.sqrt(np.mean(ge ** 2)), np.sqrt(np.mean(ee ** 2))
    _note(f"  {what}: gpu-emu rms {rms_g:.2e} med {np.median(rg):.2e} p99 {np.quantile(rg, .99):.2e} "
          f"max {rg.max():.2e} | emu-fp64 rms {rms_e:.2e} med {np.median(re):.2e} "
          f"p99 {np.quantile(re, .99):.2e} max {re.max():.2e}")
    assert rms_g <= k_rms * rms_e
    assert np.median(rg) <= k_med * np.median(re)
    assert np.quantile(rg, 0.99) <= k_p99 * np.quantile(re, 0.99)
    assert rg.max() <= k_max * re.max()


def _with_trace_species(st, seed, n_trace=512):
    """The first n_trace cells get one trace species each (species c mod S),
    Y = 10^-u with u ~ U(10, 26), the columns renormalised."""
    rng = np.random.default_rng(seed)
    Y = st.Y.copy()
    c = np.arange(min(n_trace, st.n))
    Y[c % st.S, c] = 10.0 ** -rng.uniform(10.0, 26.0, size=c.size)
    Y /= Y.sum(axis=0)
    return synth.State(st.T.copy(), st.P.copy(), Y)


def _post_bar(Y, o, net, y_post):
    """Relative error bound of the FP32 inverse transform given the network
    output o: the base Y^lam + lam delta of the power 1/lam carries a few
    ulp of its two terms, and the power multiplies the relative error of
    the base by 1/lam = 10; log2 and exp2 (at most one ulp each on gfx950)
    add about |log2 Y_new| ulp; the renormalisation sum carries the errors of
    the major species (the same bound at ratio 1).  So 1e-5 (1 + r) +
    (|log2 Y_new| + 8) 2^-22, r = (Y^lam + |lam delta|) / Y_new^lam."""
    lam = net.lam
    delta = o * net.out_std[:, None] + net.out_mean[:, None]
    yl = np.where(Y > 0, np.power(np.maximum(Y, 0.0), lam), 0.0)
    yn = np.maximum(y_post, 1e-300)
    r = (yl + np.abs(lam * delta)) / np.power(yn, lam)
    return 1e-5 * (1.0 + r) + (np.abs(np.log2(yn)) + 8.0) * 2.0 ** -22


def _fp32_decomposed(h, net, st, thermo, n_trace):
    """FP32 operands against the oracle, error by error: (a) the network
    output, per cell |o - o_ref|_inf <= 1e-5 max(1, |o_ref|_inf); (b) the
    post-processing given the GPU's own o, against the oracle's FP64
    post-processing of it, within the FP32 inverse transform's bound
    (_post_bar); (c) T_new and, on the cells without trace species, Y_new end
    to end within 1e-5 relative (floor 1e-10).  On trace species the inverse
    transform amplifies the error of o by about sigma_out / Y_new^lam, which
    the end-to-end figure shows."""
    T, P, Y = dev_state(st)
    nb = torch.zeros(1, dtype=torch.int32, device="cuda")
    Yn, Tn = h.step(T, P, Y, n_bad=nb)
    _, acc = h.debug_layers(T, P, Y)
    torch.cuda.synchronize()
    Yg, Tg = Yn.cpu().numpy(), Tn.cpu().numpy()
    o = acc[-1].cpu().numpy().astype(np.float64)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    assert int(nb.item()) == int(ref["bad"].sum()) == 0
    # (a)
    d = np.abs(o - ref["o"]).max(axis=0) / np.maximum(1.0, np.abs(ref["o"]).max(axis=0))
    # (b)
    y_post, t_post, _ = chem.post(o, st.T, st.Y, net.out_mean, net.out_std, net.lam, thermo)
    bar = _post_bar(st.Y, o, net, y_post)
    # (below FP32's normal range the kernel's Y* is subnormal or zero: an
    # absolute 2^-126 there)
    ap = np.abs(Yg - y_post)
    rp = ap / np.maximum(y_post, 1e-300)
    sel = y_post > 2.0 ** -126
    # (c)
    e2e = np.abs(Yg - ref["Y_new"]) / np.maximum(np.abs(ref["Y_new"]), 1e-10)
    e_t = rel_err(Tg, ref["T_new"], floor=1.0)
    i = np.unravel_index(np.argmax(e2e), e2e.shape)
    _note(f"  (a) network output: max per-cell error {d.max():.3e}")
    _note(f"  (b) post given o: max rel err / bar {np.max(rp[sel] / bar[sel]):.3f}, max rel err "
          f"{rp[sel].max():.2e}; below 2^-126 max |diff| {np.max(ap[~sel], initial=0):.1e}")
    _note(f"  (c) end to end: Y max {e2e.max():.3e} (cells without trace species "
          f"{e2e[:, n_trace:].max():.3e}), T {e_t:.3e}; worst entry species {i[0]} cell {i[1]}: "
          f"Y {st.Y[i]:.3e} Y_new ref {ref['Y_new'][i]:.6e} gpu {Yg[i]:.6e} post(o_gpu) {y_post[i]:.6e} "
          f"o ref {ref['o'][i]:.8e} gpu {o[i]:.8e}")
    assert np.all(d <= 1e-5)
    assert np.all(rp[sel] <= bar[sel])
    assert np.all(ap[~sel] <= 2.0 ** -126)
    assert e_t <= 1e-5
    assert e2e[:, n_trace:].max() <= 1e-5


# ------------------------------------------------------------------ fused, FP32 vs FP64
@pytest.mark.parametrize("config,n", [(1, 4096 - 37), (2, 2048 + 5)])
def test_fp32_biases_and_output_stats_match_oracle(config, n):
    """FP32 operands, random biases (U(+-0.1)) in all four layers, drawn
    output statistics and 512 cells with a trace species each: the error
    decomposition of _fp32_decomposed."""
    _note(f"case fused fp32 biases+stats config={config} n={n}")
    net = _net(config)
    S = net.widths[-1]
    thermo = synth.make_thermo(config, S)
    st = _with_trace_species(synth.make_state(config, n), 100 + config)
    h = make_handle(net, "fp32", thermo=thermo)
    _fp32_decomposed(h, net, st, thermo, 512)


def test_fp32_gelu_table_biases_and_output_stats_match_oracle():
    """The tabulated GELU with biases and output statistics (FP32 operands)
    against the oracle evaluating the same table: 1e-5 relative."""
    _note("case fused fp32 table biases+stats")
    net = _net(2)
    thermo = synth.make_thermo(2, 29)
    st = synth.make_state(2, 2048 + 5)
    h = make_handle(net, "fp32", thermo=thermo, gelu="table")
    Yg, Tg, nbad = _run(h, st)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo, act=chem.gelu_table)
    e_y, e_t = rel_err(Yg, ref["Y_new"]), rel_err(Tg, ref["T_new"], floor=1.0)
    _note(f"  rel err Y {e_y:.3e}  T {e_t:.3e}")
    assert nbad == 0 and e_y <= 1e-5 and e_t <= 1e-5


# ------------------------------------------------------------------ fused, narrow formats
@pytest.mark.parametrize("config,prec,fmt", [(2, "bf16", "bf16"), (2, "fp16", "f16"),
                                             (1, "bf16", "bf16"), (1, "fp16", "f16")])
def test_narrow_biases_and_output_stats_match_emulation(config, prec, fmt):
    """BF16 / FP16 operands with biases and output statistics against the
    oracle that rounds the same operands; the fused path's bar."""
    n = 4096 + 11
    _note(f"case fused {prec} biases+stats config={config} n={n}")
    net = _net(config)
    S = net.widths[-1]
    thermo = synth.make_thermo(config, S)
    st = synth.make_state(config, n)
    h = make_handle(net, prec, thermo=thermo)
    Yg, Tg, nbad = _run(h, st)
    emu = chem.step(st.T, st.P, st.Y, net, fmt=fmt, thermo=thermo)
    ex = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    assert nbad == 0
    _narrow_bar(Yg, emu["Y_new"], ex["Y_new"], 0.25, 0.05, 0.5, 0.5, "Y")
    tg, te = Tg - emu["T_new"], emu["T_new"] - ex["T_new"]
    assert np.sqrt(np.mean(tg ** 2)) <= 0.25 * np.sqrt(np.mean(te ** 2))
    assert np.abs(tg).max() <= np.abs(te).max()


@pytest.mark.parametrize("config,n", [(1, 4096 - 5), (2, 4096 + 11)])
def test_fp8_biases_and_output_stats_match_emulation(config, n):
    """FP8 e4m3 with per-layer power-of-two scales: the biases enter after
    the accumulator is scaled back (a separate code path from the 16-bit
    formats, whose accumulators start at the bias).  Scales from the oracle's
    calibration of this biased net; the library reproduces them bit for bit;
    the fused path's bar against the emulation."""
    _note(f"case fused fp8 biases+stats config={config} n={n}")
    net = _net(config)
    S = net.widths[-1]
    cal = synth.make_state(config, 1 << 14, stream="calibration")
    amax = chem.layer_input_amax(cal.T, cal.P, cal.Y, net).astype(np.float32)
    act_s = chem.pow2_scale(amax.astype(np.float64))
    w_s = chem.pow2_scale(chem.weight_amax(net))
    thermo = synth.make_thermo(config, S)
    st = synth.make_state(config, n)
    h = make_handle(net, "fp8", thermo=thermo, act_amax=amax)
    a, w = h.scales()
    np.testing.assert_array_equal(a.astype(np.float64), act_s)
    np.testing.assert_array_equal(w.astype(np.float64), w_s)
    Yg, Tg, nbad = _run(h, st)
    emu = chem.step(st.T, st.P, st.Y, net, fmt="e4m3", act_scale=act_s, w_scale=w_s, thermo=thermo)
    ex = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    assert nbad == 0
    _narrow_bar(Yg, emu["Y_new"], ex["Y_new"], 0.25, 0.05, 0.5, 0.5, "Y")
    tg, te = Tg - emu["T_new"], emu["T_new"] - ex["T_new"]
    assert np.sqrt(np.mean(tg ** 2)) <= 0.25 * np.sqrt(np.mean(te ** 2))
    assert np.abs(tg).max() <= np.abs(te).max()
    np.testing.assert_allclose(Yg.sum(axis=0), 1.0, atol=1e-13)


# ------------------------------------------------------------------ layer by layer
@pytest.fixture(scope="module")
def odenet():
    return _net(6)


def test_layered_fp32_biases_and_output_stats_match_oracle(odenet):
    """The paper-size ODENet (19-2048-4096-2048-1024-512-17) on the
    layer-by-layer path with biases in all six layers, output statistics
    and trace species: the error decomposition of _fp32_decomposed."""
    n = 1000 + 7
    _note(f"case layered fp32 biases+stats n={n}")
    thermo = synth.make_thermo(6, 17)
    st = _with_trace_species(synth.make_state(6, n), 106)
    h = make_handle(odenet, "fp32", thermo=thermo)
    _fp32_decomposed(h, odenet, st, thermo, 512)


U32 = 2.0 ** -24


def _gelu_err(z):
    """Relative error bound of the kernels' FP32 GELU (see test_gpu_layers)."""
    xp = np.abs(2.0 * chem.SQRT_2_OVER_PI * (z + chem.GELU_CUBIC * z ** 3) / np.log(2.0))
    return (3.0 * xp + 16.0) * U32


@pytest.mark.parametrize("prec,fmt", [("bf16", "bf16"), ("fp16", "f16")])
def test_layered_narrow_biases_and_output_stats_match_emulation(odenet, prec, fmt):
    """BF16 / FP16 on the layer-by-layer path with biases and output
    statistics, against the emulation, cell by cell.  In a deep network a
    single operand that rounds to the other side of a rounding boundary (the
    FP32 accumulation or GELU lands it there, the FP64 emulation not)
    perturbs every later layer, and such a cell follows its own rounding
    trajectory from then on; in this 6-layer net with K up to 4096 most
    cells get one in BF16 and all do in FP16.  The parity criterion is therefore per cell and exact:
    - a cell whose operands equal the emulation's in every layer matches it
      at FP32 level (network output within 1e-5 max(1, |o|_inf), Y_new within
      1e-5 relative, floor 1e-10);
    - in every other cell, at the first layer where its operands differ,
      each differing operand is the emulation's value's neighbour and the
      exact value lies within the FP32 error bound (Higham's gamma_K of the
      products, through the GELU slope, plus the GELU's own FP32 error; for
      the first layer the preprocessing's 2e-6 max(1, |z|)) of the rounding
      midpoint.
    (After its first divergence a cell's later layers are checked by the
    layer-isolated test of the same network, which holds every layer to the
    exact product of its own operands.)  The end-to-end statistics against
    the quantisation error are printed."""
    n = 1024 + 3
    _note(f"case layered {prec} biases+stats n={n}")
    thermo = synth.make_thermo(6, 17)
    st = synth.make_state(6, n)
    h = make_handle(odenet, prec, thermo=thermo)
    T, P, Y = dev_state(st)
    Yn, Tn = h.step(T, P, Y)
    qin, acc = h.debug_layers(T, P, Y)
    torch.cuda.synchronize()
    Yg, Tg = Yn.cpu().numpy(), Tn.cpu().numpy()
    qin = [q.cpu().numpy().astype(np.float64) for q in qin]
    o = acc[-1].cpu().numpy().astype(np.float64)
    emu = chem.step(st.T, st.P, st.Y, odenet, fmt=fmt, thermo=thermo)
    ex = chem.step(st.T, st.P, st.Y, odenet, thermo=thermo)
    # the emulation's operands layer by layer (the arithmetic of chem.mlp)
    L = len(odenet.W)
    Wq = [chem.round_to(np.asarray(W, np.float64), fmt) for W in odenet.W]
    b64 = [np.asarray(b, np.float64) for b in odenet.b]
    z0 = chem.features(st.T, st.P, st.Y, odenet.in_mean, odenet.in_std, odenet.lam)
    x_pre = [z0]                                  # exact values before each rounding
    tol = [2e-6 * np.maximum(1.0, np.abs(z0))]
    a_emu = [chem.round_to(z0, fmt)]
    for l in range(L - 1):
        z = Wq[l] @ a_emu[l] + b64[l][:, None]
        bound = (odenet.widths[l] + 1) * U32 * 1.01 * (np.abs(Wq[l]) @ np.abs(a_emu[l]) + np.abs(b64[l])[:, None])
        g = chem.gelu(z)
        x_pre.append(g)
        tol.append(np.abs(chem.gelu_grad(z)) * bound + _gelu_err(z) * np.abs(g) + 1e-30)
        a_emu.append(chem.round_to(g, fmt))
    first = np.full(n, -1)
    for l in range(L):
        d = np.any(qin[l] != a_emu[l], axis=0) & (first < 0)
        first[d] = l
    div = first >= 0
    _note(f"  {div.sum()} of {n} cells leave the emulation's rounding trajectory "
          f"(first at layers {np.bincount(first[div], minlength=L).tolist()})")
    for l in range(L):
        cells = first == l
        if not cells.any():
            continue
        qg, qe, xp, tl = qin[l][:, cells], a_emu[l][:, cells], x_pre[l][:, cells], tol[l][:, cells]
        m = qg != qe
        lo = chem.round_to(xp[m] - tl[m], fmt)
        hi = chem.round_to(xp[m] + tl[m], fmt)
        ok = (qg[m] >= lo) & (qg[m] <= hi)
        _note(f"    layer {l + 1}: {m.sum()} differing operands in {cells.sum()} cells, all within the "
              f"FP32 error of a rounding boundary: {ok.all()}")
        assert ok.all(), f"layer {l + 1}"
    keep = ~div
    if keep.any():
        do = np.abs(o - emu["o"])[:, keep].max(axis=0) / np.maximum(1.0, np.abs(emu["o"][:, keep]).max(axis=0))
        ey = _rel(Yg[:, keep], emu["Y_new"][:, keep]).max()
        _note(f"  cells on the emulation's trajectory: network output {do.max():.2e}, Y_new {ey:.2e}")
        assert do.max() <= 1e-5 and ey <= 1e-5
    for got, e, x, name in ((Yg, emu["Y_new"], ex["Y_new"], "Y"), (Tg, emu["T_new"], ex["T_new"], "T")):
        rg, re = _rel(got, e), _rel(e, x)
        _note(f"  {name}: gpu-emu rms {np.sqrt(np.mean((got - e) ** 2)):.2e} med {np.median(rg):.2e} "
              f"max {rg.max():.2e} | emu-fp64 rms {np.sqrt(np.mean((e - x) ** 2)):.2e} "
              f"med {np.median(re):.2e} max {re.max():.2e}")


# ------------------------------------------------------------------ non-finite results
@pytest.mark.parametrize("widths,prec", [(synth.NET_SMALL, "fp32"), (synth.NET_SMALL, "bf16"),
                                         ((19, 256, 256, 17), "fp32")])
def test_non_finite_network_output_flags_the_cell(widths, prec):
    """A cell whose network result is not finite is passed through and
    counted, as the oracle does.  Two cases: (1) finite but extreme inputs
    (T = 1e300 K: its Z-score overflows FP32 and the network output turns
    NaN on the GPU; the FP64 oracle's update overflows too) - the flags of
    both sides agree cell by cell; (2) a NaN output bias of one species: that
    output is NaN in every cell, and every cell must be flagged - not
    renormalised without the species.  Fused nets (FP32, BF16) and a
    layer-by-layer net."""
    _note(f"case non-finite outputs widths={widths} {prec}")
    net = _net(1, widths=widths)
    thermo = synth.make_thermo(1, 17)
    st = synth.make_state(1, 200)
    st.T[[5, 77, 150]] = 1e300
    st.T[33] = -1e300
    h = make_handle(net, prec, thermo=thermo)
    Yg, Tg, nbad = _run(h, st)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    gbad = np.all(Yg == st.Y, axis=0) & (Tg == st.T)
    _note(f"  extreme T: oracle flags {np.nonzero(ref['bad'])[0].tolist()}, gpu n_bad {nbad}")
    assert ref["bad"][[5, 33, 77, 150]].all()
    assert nbad == int(ref["bad"].sum())
    assert np.array_equal(gbad, ref["bad"])
    # (2) NaN output bias of species 4
    net.b[-1] = net.b[-1].copy()
    net.b[-1][4] = np.nan
    st2 = synth.make_state(1, 100)
    h2 = make_handle(net, prec, thermo=thermo)
    Yg2, Tg2, nbad2 = _run(h2, st2)
    ref2 = chem.step(st2.T, st2.P, st2.Y, net, thermo=thermo)
    assert ref2["bad"].all()
    assert nbad2 == 100
    np.testing.assert_array_equal(Yg2, st2.Y)
    np.testing.assert_array_equal(Tg2, st2.T)


# ------------------------------------------------------------------ binding checks
def test_autograd_with_padded_leading_dimension():
    """The autograd function on an input x that is a column slice of a wider
    buffer (leading dimension > batch): the saved pre-activations and the
    incoming gradient are given x's leading dimension, and the results equal
    those of a contiguous x bit for bit."""
    _note("case autograd ld > B")
    from paper_2508_18969_amd import autograd_function
    net = _net(1)
    B, ld = 1000, 1024
    h = make_handle(net, "fp32", max_batch=B)
    F = autograd_function()
    rng = np.random.default_rng(5)
    xw = torch.tensor(rng.standard_normal((19, ld)), dtype=torch.float32, device="cuda")
    xc = xw[:, :B].contiguous()
    tgt = torch.tensor(rng.standard_normal((17, B)), dtype=torch.float32, device="cuda")
    res = []
    for base in (xw, xc):
        p = h._params.clone().requires_grad_(True)
        leaf = base.clone().requires_grad_(True)
        xx = leaf[:, :B]                       # leading dimension 1024, then 1000
        assert xx.stride(0) == base.shape[1]
        out = F.apply(xx, p, h, False)
        loss = ((out - tgt) ** 2).mean()
        loss.backward()
        torch.cuda.synchronize()
        res.append((out.detach().cpu(), p.grad.detach().cpu(), leaf.grad[:, :B].detach().cpu()))
    for a, b in zip(res[0], res[1]):
        assert torch.equal(a, b)


def test_binding_rejects_bad_counter_and_saved_before_launch():
    """n_bad on the host or of 64-bit type, and saved pre-activations of the
    wrong shape or stride, are rejected by the binding (ValueError) before
    anything is enqueued."""
    net = synth.make_net(1)
    h = make_handle(net, "fp32", max_batch=64)
    st = synth.make_state(1, 64)
    T, P, Y = dev_state(st)
    for bad in (torch.zeros(1, dtype=torch.int32), torch.zeros(1, dtype=torch.int64, device="cuda"),
                torch.zeros(0, dtype=torch.int32, device="cuda")):
        with pytest.raises(ValueError):
            h.step(T, P, Y, n_bad=bad)
    x = torch.zeros((19, 64), dtype=torch.float32, device="cuda")
    for saved in (torch.zeros((700, 32), dtype=torch.float32, device="cuda"),
                  torch.zeros((64, 700), dtype=torch.float32, device="cuda").t(),
                  torch.zeros((700, 64), dtype=torch.float64, device="cuda")):
        with pytest.raises(ValueError):
            h.mlp_forward(x, h._params, saved)
    with pytest.raises(ValueError):
        h.mlp_forward(x, h._params[:-1])
