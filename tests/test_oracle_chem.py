"""Pins of the FP64 oracle's chemistry update against independent facts:
library routines (scipy, torch), closed forms, invariants and 50-digit values.
CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps
import torch

import synth
from oracle import chem

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LAM = 0.1


# ---------------------------------------------------------------- Box-Cox
def test_boxcox_matches_scipy_and_round_trips():
    y = np.concatenate([[1.0], np.logspace(-300, 0, 601), np.random.default_rng(1).random(1000)])
    u = chem.boxcox(y, LAM)
    ref = sps.boxcox(y, LAM)
    np.testing.assert_allclose(u, ref, rtol=1e-13, atol=1e-13)
    back = chem.boxcox_inv(u, LAM)
    # u = (y^lam - 1)/lam keeps y^lam = 1 + lam u only to an absolute error of
    # a few ulp of 1: the round trip is exact to that level in the y^lam domain
    assert np.all(np.abs(back ** LAM - y ** LAM) <= 4 * 2.0 ** -52)
    big = y > 1e-30
    np.testing.assert_allclose(back[big], y[big], rtol=1e-12)
    np.testing.assert_allclose(back, sps.inv_boxcox(u, LAM), rtol=1e-12)
    assert chem.boxcox(np.array([1.0]), LAM)[0] == 0.0
    assert chem.boxcox(np.array([0.0]), LAM)[0] == -10.0
    assert chem.boxcox(np.array([-1e-20]), LAM)[0] == -10.0      # non-positive taken as 0


def test_boxcox_inverse_clamps_below_domain():
    # 1 + lam u < 0 would be turned positive by the even power 1/lam = 10
    assert chem.boxcox_inv(np.array([-10.0, -11.0, -1e3]), LAM).tolist() == [0.0, 0.0, 0.0]


# ---------------------------------------------------------------- GELU
def _golden_gelu():
    rows = [l.split() for l in open(os.path.join(GOLD, "gelu_tanh_mp50.txt")) if not l.startswith("#")]
    return [(float(r[0]), float(r[1]), float(r[2]), float(r[3])) for r in rows]


def test_gelu_50_digit_values_and_derivative():
    for x, g, d, _ in _golden_gelu():
        assert abs(chem.gelu(np.array([x]))[0] - g) <= 2e-16 * max(1.0, abs(g))
        assert abs(chem.gelu_grad(np.array([x]))[0] - d) <= 1e-15 * max(1.0, abs(d))


def test_gelu_identities_and_erf_form():
    x = np.linspace(-12, 12, 20001)
    g = chem.gelu(x)
    assert chem.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(g - chem.gelu(-x), x, atol=4e-15)   # tanh is odd
    erf_form = x * sps.ndtr(x)
    err = np.abs(g - erf_form)
    assert err.max() <= 4.8e-4 and err.max() >= 4.5e-4            # the two forms differ
    xt = torch.tensor(x, dtype=torch.float64)
    tg = torch.nn.functional.gelu(xt, approximate="tanh").numpy()
    np.testing.assert_allclose(g, tg, rtol=1e-14, atol=1e-15)


def test_gelu_constants_are_the_papers():
    c = json.load(open(os.path.join(GOLD, "paper_constants.json")))["gelu_tanh_form"]
    assert chem.GELU_CUBIC == c["cubic"]
    assert abs(chem.SQRT_2_OVER_PI - c["sqrt_2_over_pi"]) < 1e-16


# ---------------------------------------------------------------- narrow formats
def test_round_bf16_matches_torch():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 3.0e38, 1e-40]])
    x32 = x.astype(np.float32).astype(np.float64)      # torch rounds from fp32
    ref = torch.tensor(x32, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(chem.round_to(x32, "bf16"), ref)


def test_round_f16_matches_numpy():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 6, 20000)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(chem.round_to(x, "f16"), ref)


def _e4m3_table():
    rows = [l.split() for l in open(os.path.join(GOLD, "e4m3_codes.txt")) if not l.startswith("#")]
    return np.array([float(r[1]) for r in rows])


def test_round_e4m3_against_code_table():
    vals = _e4m3_table()
    fin = np.isfinite(vals)
    grid = np.unique(vals[fin])
    # every representable value maps to itself
    np.testing.assert_array_equal(chem.round_to(grid, "e4m3"), grid)
    # brute force: nearest grid point, ties to the even code (lowest mantissa bit 0)
    pos = np.unique(vals[fin & (vals >= 0)])
    codes = {v: c for c, v in enumerate(vals) if np.isfinite(v) and (v > 0 or c == 0)}
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(0, 448, 5000), rng.uniform(0, 0.03, 5000),
                        (pos[1:] + pos[:-1]) / 2])                 # all midpoints
    got = chem.round_to(x, "e4m3")
    for xi, gi in zip(x, got):
        d = np.abs(pos - xi)
        best = pos[d == d.min()]
        if best.size == 1:
            assert gi == best[0]
        else:
            even = [b for b in best if codes[b] % 2 == 0]
            assert gi == even[0]
    np.testing.assert_array_equal(chem.round_to(-x, "e4m3"), -got)
    # torch agrees inside the range (it does not saturate)
    t = torch.tensor(x, dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, t)
    # saturation instead of NaN/inf
    assert chem.round_to(np.array([500.0, -1e9, np.inf]), "e4m3").tolist() == [448.0, -448.0, 448.0]


def test_pow2_scale():
    amax = np.array([1e-30, 0.01, 1.0, 447.9, 448.0, 448.1, 896.0, 1e6])
    s = chem.pow2_scale(amax)
    assert np.all(np.log2(s) == np.round(np.log2(s)))              # powers of two
    r = amax / s
    assert np.all(r <= 448.0) and np.all(r > 224.0)
    assert chem.pow2_scale(np.array([0.0]))[0] == 1.0


# ---------------------------------------------------------------- normalisation
def test_zscore_features_have_unit_moments():
    """The analytic input moments of the generator and the oracle's (x-mu)/sigma
    together give mean 0 and std 1 on a large draw (statistical bound)."""
    S = 29
    st = synth.draw_uniform_state(np.random.default_rng(5), S, 1 << 18)
    mu, sd = synth.uniform_state_input_moments(S)
    z = chem.features(st.T, st.P, st.Y, mu, sd, LAM)
    n = z.shape[1]
    assert np.all(np.abs(z.mean(axis=1)) < 6.0 / math.sqrt(n))
    assert np.all(np.abs(z.std(axis=1) - 1.0) < 0.02)
    assert np.all(np.abs(chem.features(st.T[:1] * 0 + mu[0], st.P[:1] * 0 + mu[1],
                                       st.Y[:, :1], mu, sd, LAM)[:2]) < 1e-15)


# ---------------------------------------------------------------- MLP
def _torch_mlp(z, W, b):
    a = torch.tensor(z.T, dtype=torch.float64)
    for l, (w, v) in enumerate(zip(W, b)):
        a = torch.nn.functional.linear(a, torch.tensor(np.asarray(w, np.float64)),
                                       torch.tensor(np.asarray(v, np.float64)))
        if l < len(W) - 1:
            a = torch.nn.functional.gelu(a, approximate="tanh")
    return a.numpy().T


@pytest.mark.parametrize("widths", [(5, 7), (19, 40, 20, 10, 17), (31, 64, 32, 16, 29)])
def test_mlp_matches_torch(widths):
    rng = np.random.default_rng(6)
    W, b = synth.xavier_weights(rng, widths, bias_scale=0.3)
    z = rng.standard_normal((widths[0], 333))
    np.testing.assert_allclose(chem.mlp(z, W, b), _torch_mlp(z, W, b), rtol=1e-12, atol=1e-13)


def test_mlp_cells_independent_and_padding_invariant():
    rng = np.random.default_rng(7)
    widths = (19, 40, 20, 10, 17)
    W, b = synth.xavier_weights(rng, widths, bias_scale=0.3)
    z = rng.standard_normal((19, 50))
    full = chem.mlp(z, W, b)
    one = chem.mlp(z[:, 17:18], W, b)
    # the library matmul may block differently for one column: equal to rounding
    np.testing.assert_allclose(full[:, 17:18], one, rtol=1e-14, atol=1e-15)
    # zero-padded hidden units (zero weights in and out, zero bias) change nothing
    Wp = [np.vstack([W[0], np.zeros((8, 19))]), np.hstack([W[1], np.zeros((20, 8))]), W[2], W[3]]
    bp = [np.concatenate([b[0], np.zeros(8)]), b[1], b[2], b[3]]
    np.testing.assert_allclose(chem.mlp(z, Wp, bp), full, rtol=0, atol=1e-15)


def test_emulated_mlp_matches_torch_quantisation():
    rng = np.random.default_rng(8)
    widths = (19, 40, 20, 10, 17)
    W, b = synth.xavier_weights(rng, widths, bias_scale=0.1)
    z = rng.standard_normal((19, 64))
    for fmt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16), ("e4m3", torch.float8_e4m3fn)):
        sa = np.array([2.0 ** -5, 2.0 ** -7, 2.0 ** -8, 2.0 ** -8]) if fmt == "e4m3" else None
        sw = np.array([2.0 ** -9] * 4) if fmt == "e4m3" else None
        got = chem.mlp(z, W, b, fmt=fmt, act_scale=sa, w_scale=sw)
        a = torch.tensor(z, dtype=torch.float64)
        for l in range(4):
            s_a = 1.0 if sa is None else sa[l]
            s_w = 1.0 if sw is None else sw[l]
            lim = 448.0 if fmt == "e4m3" else float("inf")      # saturating cast
            aq = (a / s_a).clamp(-lim, lim).to(torch.float32).to(tdt).to(torch.float64)
            wq = (torch.tensor(np.asarray(W[l], np.float64) / s_w).clamp(-lim, lim)
                  .to(torch.float32).to(tdt).to(torch.float64))
            a = (wq @ aq) * (s_a * s_w) + torch.tensor(np.asarray(b[l], np.float64))[:, None]
            if l < 3:
                a = torch.nn.functional.gelu(a, approximate="tanh")
        np.testing.assert_allclose(got, a.numpy(), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- post / step
def _state(n=500, S=17, seed=9):
    return synth.draw_uniform_state(np.random.default_rng(seed), S, n)


def test_post_inverse_transform_matches_scipy():
    st = _state()
    rng = np.random.default_rng(10)
    o = 0.05 * rng.standard_normal(st.Y.shape)
    ynew, _, bad = chem.post(o, st.T, st.Y, np.zeros(17), np.ones(17), LAM)
    ystar = sps.inv_boxcox(sps.boxcox(st.Y, LAM) + o, LAM)
    ystar = np.where(1 + LAM * (sps.boxcox(st.Y, LAM) + o) < 0, 0.0, ystar)
    np.testing.assert_allclose(ynew, ystar / ystar.sum(axis=0), rtol=1e-12, atol=1e-300)
    assert not bad.any()
    np.testing.assert_allclose(ynew.sum(axis=0), 1.0, atol=17 * 2.0 ** -52)
    assert (ynew >= 0).all()


def test_post_zero_increment_is_identity_and_keeps_enthalpy():
    st = _state()
    hf, cp, tref = synth.make_thermo(1, 17)
    ynew, tnew, bad = chem.post(np.zeros_like(st.Y), st.T, st.Y, np.zeros(17), np.ones(17), LAM,
                                (hf, cp, tref))
    np.testing.assert_allclose(ynew, st.Y, rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(tnew, st.T, rtol=1e-13)
    o = 0.1 * np.random.default_rng(11).standard_normal(st.Y.shape)
    ynew, tnew, bad = chem.post(o, st.T, st.Y, np.zeros(17), np.ones(17), LAM, (hf, cp, tref))
    h0 = (st.Y * (hf[:, None] + cp[:, None] * (st.T - tref))).sum(axis=0)
    h1 = (ynew * (hf[:, None] + cp[:, None] * (tnew - tref))).sum(axis=0)
    np.testing.assert_allclose(h1, h0, rtol=1e-12, atol=1e-6)


def test_output_statistics_are_applied():
    st = _state(n=50)
    o = np.ones_like(st.Y)
    mu, sd = np.full(17, 0.02), np.full(17, 3.0)
    y1, _, _ = chem.post(o, st.T, st.Y, mu, sd, LAM)
    y2, _, _ = chem.post(o * 3.0 + 0.02, st.T, st.Y, np.zeros(17), np.ones(17), LAM)
    np.testing.assert_allclose(y1, y2, rtol=1e-15)


def test_step_flags_and_passes_through_bad_cells():
    net = synth.make_net(1)
    st = _state(n=8)
    T, Y = st.T.copy(), st.Y.copy()
    T[1] = np.nan
    Y[3, 2] = np.inf
    Y[:, 5] = 0.0                       # all-zero composition is legal input
    hf, cp, tref = synth.make_thermo(1, 17)
    r = chem.step(T, st.P, Y, net, thermo=(hf, cp, tref))
    assert r["bad"][1] and r["bad"][2]
    assert np.isnan(r["T_new"][1])
    np.testing.assert_array_equal(r["Y_new"][:, 2], Y[:, 2])
    good = ~r["bad"]
    np.testing.assert_allclose(r["Y_new"][:, good].sum(axis=0), 1.0, atol=1e-14)


def test_step_with_zero_output_layer_returns_input():
    net = synth.make_net(1)
    net.W[-1] = np.zeros_like(net.W[-1])
    st = _state(n=64)
    r = chem.step(st.T, st.P, st.Y, net)
    np.testing.assert_allclose(r["Y_new"], st.Y / st.Y.sum(axis=0), rtol=1e-13, atol=1e-300)


# ------------------------------------------------------------------ tabulated GELU (Sec. 3.3.2)
def test_gelu_second_derivative_central_differences():
    x = np.linspace(-5.0, 5.0, 2001)
    h = 1e-5
    fd = (chem.gelu_grad(x + h) - chem.gelu_grad(x - h)) / (2 * h)
    assert np.max(np.abs(fd - chem.gelu_second(x))) <= 1e-8


def test_gelu_table_is_exact_at_midpoints_and_within_taylor_bound():
    """Second-order Taylor expansion about each midpoint: exact there, and off
    by at most (h/2)^3/6 max|GELU'''| inside [-3, 3]."""
    m = -3.0 + (np.arange(600) + 0.5) * 0.01
    np.testing.assert_array_equal(chem.gelu_table(m), chem.gelu(m))
    x = np.linspace(-3.0, 3.0, 600001)
    err = np.max(np.abs(chem.gelu_table(x) - chem.gelu(x)))
    xs = np.linspace(-3.0, 3.0, 60001)
    h = 1e-4
    f3 = np.max(np.abs((chem.gelu_second(xs + h) - chem.gelu_second(xs - h)) / (2 * h)))
    bound = 0.005 ** 3 / 6.0 * f3
    assert err <= 1.001 * bound, (err, bound)
    assert err >= 0.5 * bound          # the bound is attained: the expansion is second order


def test_gelu_table_outside_and_jump():
    """Zero below -3 and the identity above 3 (the paper's statement); the jump
    at the ends is the GELU's own value there."""
    x = np.array([-50.0, -3.5, -3.000001, 3.000001, 4.0, 60.0])
    np.testing.assert_array_equal(chem.gelu_table(x), np.where(x < 0, 0.0, x))
    jump = abs(chem.gelu_table(-2.9999999) - chem.gelu_table(-3.0000001))
    assert abs(jump - abs(chem.gelu(-3.0))) <= 1e-6


def test_gelu_table16_coefficients_and_error():
    """FP16 tabulation (Sec. 3.3.2): the coefficients are the FP32 table's
    FP64 values rounded once to FP16 - numpy's own FP16 conversion (round to
    nearest even) gives the same values; against the FP64 table the error is
    at most the coefficient rounding, |dc0| + |dc1| h/2 + |dc2| (h/2)^2 with
    each |dc_k| <= 2^-11 |c_k|; against the tanh form that plus the table's
    own Taylor error (<= 1.6e-8)."""
    c64 = chem.gelu_table_coeffs()
    c16 = chem.gelu_table16_coeffs()
    np.testing.assert_array_equal(c16, c64.astype(np.float16).astype(np.float64))
    dc = np.abs(c16 - c64)
    assert np.all(dc <= 2.0 ** -11 * np.abs(c64))
    x = np.linspace(-3.0, 3.0, 600001)
    i = np.clip(np.floor((x + 3.0) / 0.01), 0, 599).astype(int)
    d = np.abs(x - (-3.0 + (i + 0.5) * 0.01))
    bound = dc[i, 0] + dc[i, 1] * d + dc[i, 2] * d * d
    e16 = np.abs(chem.gelu_table16(x) - chem.gelu_table(x))
    assert np.all(e16 <= bound * (1 + 1e-9) + 1e-15)
    err = np.max(np.abs(chem.gelu_table16(x) - chem.gelu(x)))
    assert err <= np.max(bound) + 1.6e-8
    assert 1e-4 <= err <= 1.6e-3          # FP16's 11 bits on values up to 3


# ------------------------------------------------------------------ source terms
def test_density_of_a_single_species_is_the_ideal_gas_law():
    """One species: rho = P W / (R T); nitrogen at 300 K and 1 atm is
    1.138 kg/m^3 (W = 28.0134 g/mol)."""
    W = np.array([0.0280134, 0.0319988])
    Y = np.array([[1.0], [0.0]])
    rho = chem.mixture_density(np.array([300.0]), np.array([101325.0]), Y, W)
    assert abs(rho[0] - 101325.0 * 0.0280134 / (8.31446261815324 * 300.0)) < 1e-12
    assert abs(rho[0] - 1.138) < 5e-4


def test_density_matches_the_mole_fraction_form():
    """rho = P Wbar / (R T) with Wbar = sum_s x_s W_s and x_s the mole
    fractions: another route to the same number."""
    S, n = 9, 50
    rng = np.random.default_rng(3)
    W = rng.uniform(0.002, 0.2, S)
    Y = rng.dirichlet(np.full(S, 0.5), n).T
    T = rng.uniform(300, 3000, n)
    P = rng.uniform(1e5, 2e7, n)
    moles = Y / W[:, None]
    x = moles / moles.sum(axis=0)
    wbar = (x * W[:, None]).sum(axis=0)
    np.testing.assert_allclose(chem.mixture_density(T, P, Y, W), P * wbar / (chem.R_GAS * T),
                               rtol=1e-13)


def test_source_terms_conserve_mass_and_scale_with_dt():
    """sum_s omega_s = 0 when both states sum to one; omega is linear in the
    change and inversely proportional to dt; a passed-through cell has none."""
    net = synth.make_net(1)
    st = synth.make_state(1, 300)
    W = synth.make_molar_masses(1, 17)
    out = chem.step(st.T, st.P, st.Y, net)
    om = chem.source_terms(st.T, st.P, st.Y, out["Y_new"], W, 1e-6)
    rho = chem.mixture_density(st.T, st.P, st.Y, W)
    scale = rho / 1e-6
    assert np.max(np.abs(om.sum(axis=0)) / scale) < 1e-14
    om2 = chem.source_terms(st.T, st.P, st.Y, out["Y_new"], W, 2e-6)
    np.testing.assert_allclose(om2, om / 2, rtol=1e-14, atol=0)
    np.testing.assert_allclose(om * 1e-6 / rho, out["Y_new"] - st.Y, rtol=1e-12, atol=1e-18)
    assert not np.any(chem.source_terms(st.T, st.P, st.Y, st.Y, W, 1e-6))
