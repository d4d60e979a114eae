"""FP64 oracle of the chemistry update (test infrastructure; see package doc).

Every function follows one passage of the paper or one stated reading of a
point the paper leaves open; the readings are listed in the design notes.

Layout: features or species first, cells second (``x[j][i]``), like the
solver's structure-of-arrays fields.
"""
from __future__ import annotations

import math

import numpy as np

SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)
GELU_CUBIC = 0.044715

# Narrow operand formats: (precision bits incl. the hidden bit, minimum normal
# exponent, largest finite value, saturate on overflow).
FORMATS = {
    "bf16": (8, -126, float.fromhex("0x1.fep127"), False),
    "f16": (11, -14, 65504.0, False),
    "e4m3": (4, -6, 448.0, True),      # OCP FP8 E4M3 ("fn": no infinities)
}


# --------------------------------------------------------------------------- transforms
def boxcox(y, lam):
    """Power (Box-Cox) transform of mass fractions, (y^lam - 1)/lam.

    Not described in the paper; it is the input transform of the chemistry
    net here.  Non-positive y are taken as 0, so BC(0) = -1/lam.
    """
    y = np.asarray(y, dtype=np.float64)
    yl = np.where(y > 0, np.power(np.maximum(y, 0.0), lam), 0.0)
    return (yl - 1.0) / lam


def boxcox_inv(u, lam):
    """Inverse transform (max(0, 1 + lam u))^(1/lam); the clamp keeps an even
    power 1/lam from turning a negative base positive."""
    base = np.maximum(1.0 + lam * np.asarray(u, dtype=np.float64), 0.0)
    return np.power(base, 1.0 / lam)


def gelu(x):
    """GELU in the tanh form the paper implements (Sec. 3.3.2):
    0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + np.tanh(SQRT_2_OVER_PI * (x + GELU_CUBIC * x ** 3)))


# Tabulated GELU of Sec. 3.3.2: zero below -3, the identity above 3, and a
# second-order table with interval 0.01 on [-3, 3].  The paper gives no more
# detail; reading: 600 intervals, each with the second-order Taylor expansion
# of the tanh-form GELU about the interval's midpoint.
GELU_TAB_LO, GELU_TAB_HI, GELU_TAB_H = -3.0, 3.0, 0.01
GELU_TAB_N = 600


def gelu_second(x):
    """d2/dx2 of the tanh-form GELU."""
    x = np.asarray(x, dtype=np.float64)
    v = SQRT_2_OVER_PI * (x + GELU_CUBIC * x ** 3)
    t = np.tanh(v)
    s2 = 1.0 - t * t                                   # sech^2 v
    dv = SQRT_2_OVER_PI * (1.0 + 3.0 * GELU_CUBIC * x * x)
    d2v = SQRT_2_OVER_PI * 6.0 * GELU_CUBIC * x
    # GELU = x (1 + t)/2:  G'' = t' + x t''/2,  t' = s2 v',  t'' = s2 (v'' - 2 t v'^2)
    return s2 * dv + 0.5 * x * s2 * (d2v - 2.0 * t * dv * dv)


def gelu_table_coeffs():
    """[600][3] FP64: value, first derivative and half the second derivative
    of the GELU at the midpoints -3 + (i + 1/2) 0.01."""
    m = GELU_TAB_LO + (np.arange(GELU_TAB_N) + 0.5) * GELU_TAB_H
    return np.stack([gelu(m), gelu_grad(m), 0.5 * gelu_second(m)], axis=1)


def gelu_table(x, coeffs=None):
    """The tabulated GELU: c0 + c1 d + c2 d^2 with d the offset from the
    midpoint of x's interval; 0 below -3, x above 3."""
    x = np.asarray(x, dtype=np.float64)
    c = gelu_table_coeffs() if coeffs is None else coeffs
    i = np.clip(np.floor((x - GELU_TAB_LO) / GELU_TAB_H), 0, GELU_TAB_N - 1).astype(np.int64)
    d = x - (GELU_TAB_LO + (i + 0.5) * GELU_TAB_H)
    y = c[i, 0] + d * (c[i, 1] + d * c[i, 2])
    return np.where(x < GELU_TAB_LO, 0.0, np.where(x > GELU_TAB_HI, x, y))


def gelu_table16_coeffs():
    """The same coefficients rounded once to FP16 (round to nearest even):
    the paper implements both FP32- and FP16-precision tabulation of the
    GELU (Sec. 3.3.2)."""
    return round_to(gelu_table_coeffs(), "f16")


def gelu_table16(x):
    """The tabulated GELU with FP16 coefficients, evaluated exactly (FP64)."""
    return gelu_table(x, gelu_table16_coeffs())


def gelu_grad(x):
    """d/dx of the tanh-form GELU."""
    x = np.asarray(x, dtype=np.float64)
    v = SQRT_2_OVER_PI * (x + GELU_CUBIC * x ** 3)
    t = np.tanh(v)
    dv = SQRT_2_OVER_PI * (1.0 + 3.0 * GELU_CUBIC * x * x)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * dv


# --------------------------------------------------------------------------- narrow formats
def round_to(x, fmt):
    """Round-to-nearest-even of FP64 values to a narrow format, returned as FP64.

    With p precision bits and minimum normal exponent emin, a value whose
    leading bit has exponent e (clamped below at emin for subnormals) lies on
    the grid of spacing 2^(max(e, emin) - p + 1); rounding to that grid with
    ties to even is exact in FP64 because the scaling is by a power of two.
    Overflow goes to +-inf, or to +-max for the saturating FP8 format.
    """
    p, emin, vmax, sat = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, copy=True)
    fin = np.isfinite(x) & (x != 0)
    xv = x[fin]
    _, E = np.frexp(xv)                      # |x| = m 2^E, m in [0.5, 1)
    e = np.maximum(E - 1, emin)
    q = np.ldexp(1.0, e - (p - 1))
    r = np.rint(xv / q) * q                  # np.rint rounds half to even
    big = np.abs(r) > vmax
    r = np.where(big, np.copysign(vmax if sat else np.inf, r), r)
    out[fin] = r
    if sat:
        out = np.where(np.isinf(x), np.copysign(vmax, x), out)
    return out


def pow2_scale(amax, fmt="e4m3"):
    """Smallest power of two s with amax / s <= largest finite value of fmt.

    Reading of the per-layer amax scaling: a power of two makes the scaling
    and the later unscaling of the FP32 accumulator exact.
    """
    vmax = FORMATS[fmt][2]
    amax = np.asarray(amax, dtype=np.float64)
    out = np.ones_like(amax)
    pos = amax > 0
    m, E = np.frexp(amax[pos] / vmax)        # ratio = m 2^E, m in [0.5, 1)
    k = np.where(m == 0.5, E - 1, E)         # ceil(log2(ratio))
    out[pos] = np.ldexp(1.0, k)
    return out


# --------------------------------------------------------------------------- forward
def features(T, P, Y, in_mean, in_std, lam):
    """Network input: x = [T, P, BC(Y_1..Y_S)], Z-score normalised (Sec. 3.3.1)."""
    T = np.asarray(T, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    x = np.vstack([T[None, :], P[None, :], boxcox(Y, lam)])
    return (x - np.asarray(in_mean)[:, None]) / np.asarray(in_std)[:, None]


def mlp(z, W, b, fmt=None, act_scale=None, w_scale=None, amax=None, act=gelu):
    """Fully connected net: hidden layers a_l = GELU(W_l a_(l-1) + b_l), linear
    output layer.  W[l] is [out][in], z is [in][cells].

    fmt=None is exact FP64.  With fmt in FORMATS, each layer's operands are
    the narrow-format values round(a / s_A) and round(W / s_W) (the paper runs
    weights and activations in FP16, Sec. 3.3.1); their products are summed in
    FP64 and scaled back by s_A s_W before the bias is added.  Scales default
    to 1.  ``amax`` (a list) receives each layer's input max |a|.  ``act`` is
    the activation (the tanh-form GELU, or gelu_table).
    """
    a = np.asarray(z, dtype=np.float64)
    L = len(W)
    for l in range(L):
        Wl = np.asarray(W[l], dtype=np.float64)
        bl = np.asarray(b[l], dtype=np.float64)
        if amax is not None:
            amax.append(float(np.max(np.abs(a))) if a.size else 0.0)
        if fmt is None:
            zl = Wl @ a + bl[:, None]
        else:
            sa = 1.0 if act_scale is None else float(act_scale[l])
            sw = 1.0 if w_scale is None else float(w_scale[l])
            zl = (round_to(Wl / sw, fmt) @ round_to(a / sa, fmt)) * (sa * sw) + bl[:, None]
        a = act(zl) if l < L - 1 else zl
    return a


def post(o, T, Y, out_mean, out_std, lam, thermo=None):
    """Inverse transform, FP64 update and renormalisation of one step.

    delta = o * sigma_out + mu_out is the predicted increment of BC(Y);
    Y* = BC^-1(BC(Y) + delta) = (max(0, Y^lam + lam delta))^(1/lam);
    dY = Y* - Y;  Yhat = Y + dY;  Y_new = Yhat / sum(Yhat).
    With thermo = (h_f, c_p, T_ref), the new temperature keeps the mixture
    enthalpy sum_i Y_i (h_f,i + c_p,i (T - T_ref)) unchanged.  Cells with a
    non-finite input or result, or sum(Yhat) <= 0, are passed through
    unchanged and flagged.
    """
    o = np.asarray(o, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    delta = o * np.asarray(out_std)[:, None] + np.asarray(out_mean)[:, None]
    yl = np.where(Y > 0, np.power(np.maximum(Y, 0.0), lam), 0.0)
    ystar = np.power(np.maximum(yl + lam * delta, 0.0), 1.0 / lam)
    dY = ystar - Y
    yhat = Y + dY
    s = yhat.sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        ynew = yhat / s
    T_new = None
    if thermo is not None:
        hf, cp, t_ref = thermo
        hf = np.asarray(hf)[:, None]
        cp = np.asarray(cp)[:, None]
        h0 = (Y * (hf + cp * (T[None, :] - t_ref))).sum(axis=0)
        with np.errstate(invalid="ignore", divide="ignore"):
            T_new = t_ref + (h0 - (ynew * hf).sum(axis=0)) / (ynew * cp).sum(axis=0)
    bad = ~(s > 0) | ~np.isfinite(s) | ~np.all(np.isfinite(ynew), axis=0)
    if T_new is not None:
        bad |= ~np.isfinite(T_new)
    ynew = np.where(bad[None, :], Y, ynew)
    if T_new is not None:
        T_new = np.where(bad, T, T_new)
    return ynew, T_new, bad


def step(T, P, Y, net, fmt=None, act_scale=None, w_scale=None, thermo=None, act=gelu):
    """One chemistry update of every cell.  ``net`` has the attributes of
    ``synth.Net`` (widths, W, b, in/out statistics, lam).

    Returns dict(Y_new, T_new, o, bad).  Cells with a non-finite T, P or Y
    are flagged and passed through.
    """
    T = np.asarray(T, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    fin_in = np.isfinite(T) & np.isfinite(P) & np.all(np.isfinite(Y), axis=0)
    Ts = np.where(fin_in, T, 1000.0)
    Ps = np.where(fin_in, P, 1.0e7)
    Ys = np.where(fin_in[None, :], Y, 0.0)
    z = features(Ts, Ps, Ys, net.in_mean, net.in_std, net.lam)
    W64 = [np.asarray(w, dtype=np.float64) for w in net.W]
    b64 = [np.asarray(v, dtype=np.float64) for v in net.b]
    o = mlp(z, W64, b64, fmt, act_scale, w_scale, act=act)
    ynew, tnew, bad = post(o, Ts, Ys, net.out_mean, net.out_std, net.lam, thermo)
    bad = bad | ~fin_in
    ynew = np.where(bad[None, :], Y, ynew)
    if tnew is not None:
        tnew = np.where(bad, T, tnew)
    return {"Y_new": ynew, "T_new": tnew, "o": o, "bad": bad}


# Molar gas constant, J/(mol K) (exact in the SI since 2019: N_A k_B).
R_GAS = 8.31446261815324


def mixture_density(T, P, Y, W):
    """Ideal-gas density (kg/m^3) of cells at T (K) and P (Pa) with mass
    fractions Y [S][n] and species molar masses W [S] (kg/mol):
    rho = P / (R T sum_s Y_s / W_s).  (The flame of the paper is
    supercritical and takes rho from a property network; the ideal-gas law
    is the reading used here.)"""
    T = np.asarray(T, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    return P / (R_GAS * T * np.sum(Y / W[:, None], axis=0))


def source_terms(T, P, Y, Y_new, W, dt):
    """Chemical source terms of the species transport equations, the
    quantity the network's result stands for (Sec. 2, DeepFlame workflow):
    omega_s = rho (Y_new,s - Y_s) / dt in kg/(m^3 s), rho the ideal-gas
    density of the state before the step.  Cells passed through by the step
    (Y_new = Y) get 0."""
    rho = mixture_density(T, P, Y, W)
    return rho[None, :] * (np.asarray(Y_new, np.float64) - np.asarray(Y, np.float64)) / float(dt)


def layer_input_amax(T, P, Y, net):
    """Per-layer max |input| of the exact FP64 forward over a calibration set."""
    z = features(T, P, Y, net.in_mean, net.in_std, net.lam)
    am = []
    mlp(z, [np.asarray(w, np.float64) for w in net.W],
        [np.asarray(v, np.float64) for v in net.b], amax=am)
    return np.array(am)


def weight_amax(net):
    return np.array([float(np.max(np.abs(np.asarray(w, np.float64)))) for w in net.W])


def fp8_scales(T, P, Y, net):
    """(act_scale, w_scale): power-of-two per-layer scales for OCP e4m3 from
    the calibration set's activation amax and the weights' amax."""
    return pow2_scale(layer_input_amax(T, P, Y, net)), pow2_scale(weight_amax(net))
