"""Seeded synthetic inputs for the per-cell DNN chemistry update.

This module only draws random numbers and states the moments of the
distributions it draws from.  It holds none of the update's arithmetic
(no Box-Cox transform, no network, no renormalisation): both the FP64
oracle and the HIP path receive the arrays made here as inputs.

The paper's workloads (supercritical LOX/CH4 Taylor-Green vortex and a
rocket combustor, Sec. 4.1) need meshes, a 17-species mechanism and trained
ODENet weights that are not published; the draws below stand in for them:

* states (T, P, Y): the paper's ODENet input is the thermochemical state
  (T, p, Y_i) (Sec. 2, DeepFlame workflow); pressures around 10 MPa and
  temperatures of 150-3000+ K follow Sec. 4.1;
* weights: Xavier-uniform in FP64, rounded to FP32 (the paper trains its
  nets; trained weights are unavailable);
* Z-score statistics: the exact mean and population standard deviation of
  each input feature under the state distribution (the paper normalises
  inputs to mean 0, std 1, Sec. 3.3.1);
* a synthetic element-conserving reaction mechanism for training labels.

Every array is generated in FP64 (FP32 for network parameters) from
``numpy.random.SeedSequence(18969 + 1000 * config)`` spawned into named
streams, so the same seed always gives bitwise-identical arrays.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np
from scipy import special

SEED_BASE = 18969
# (new names go at the end: a spawned child depends only on its index, so the
# earlier streams keep their draws)
STREAMS = ("weights", "inputs", "calibration", "mechanism", "subsample", "extra", "stats")

# Network shapes of the five workloads.  D = S + 2 inputs (T, P, S species),
# S outputs, three GELU hidden layers.
NET_SMALL = (19, 400, 200, 100, 17)     # 17 species
NET_LARGE = (31, 1600, 800, 400, 29)    # 29 species
# the ODENet size of the paper's runs (20-2048-4096-2048-1024-512-17) with
# S + 2 = 19 inputs for 17 species
NET_ODENET = (19, 2048, 4096, 2048, 1024, 512, 17)
BOXCOX_LAMBDA = 0.1

# Property networks of the supercritical flame (the paper's PRNet, Sec. 4
# network sizes): three inputs -> density, and three inputs -> temperature and
# three transport properties.  Workloads 7 and 8.
NET_PRNET_RHO = (3, 1024, 512, 256, 1)
NET_PRNET_TRANS = (3, 2048, 1024, 512, 4)
PROP_NETS = {7: NET_PRNET_RHO, 8: NET_PRNET_TRANS}
# Output scales (mean, std) of the properties: density kg/m^3; temperature K,
# viscosity Pa s, thermal diffusivity m^2/s, thermal conductivity W/(m K).
PROP_OUT = {7: ([600.0], [350.0]),
            8: ([1500.0, 4.0e-5, 1.0e-6, 0.1], [900.0, 3.0e-5, 8.0e-7, 0.06])}

T_UNIFORM = (300.0, 3000.0)        # K
P_MEDIAN, P_SIGMA = 1.0e7, 0.3     # Pa, lognormal
DIRICHLET_ALPHA = 0.5


def streams(config: int) -> dict:
    """Named independent generators for workload ``config`` (1..5; 6 is the
    paper-size ODENet over the states of workload 1; 7 and 8 the property
    networks)."""
    ss = np.random.SeedSequence(SEED_BASE + 1000 * int(config))
    kids = ss.spawn(len(STREAMS))
    return {name: np.random.Generator(np.random.PCG64(k)) for name, k in zip(STREAMS, kids)}


# --------------------------------------------------------------------------- states
@dataclass
class State:
    T: np.ndarray          # [n] K, float64
    P: np.ndarray          # [n] Pa, float64
    Y: np.ndarray          # [S][n] mass fractions, float64, each column sums to 1

    @property
    def n(self) -> int:
        return int(self.T.shape[0])

    @property
    def S(self) -> int:
        return int(self.Y.shape[0])


def _dirichlet(rng, S, n, alpha=DIRICHLET_ALPHA):
    # Gamma(alpha) draws normalised per column: a Dirichlet(alpha * 1_S) sample.
    g = rng.standard_gamma(alpha, size=(S, n))
    s = g.sum(axis=0)
    bad = s <= 0
    if bad.any():                      # astronomically rare; redraw those columns
        g[:, bad] = rng.standard_gamma(alpha, size=(S, int(bad.sum()))) + 1e-300
        s = g.sum(axis=0)
    return g / s


def draw_uniform_state(rng, S: int, n: int) -> State:
    """T ~ U(300, 3000) K, P = 10 MPa * exp(0.3 N(0,1)), Y ~ Dirichlet(0.5)."""
    T = rng.uniform(*T_UNIFORM, size=n)
    P = P_MEDIAN * np.exp(P_SIGMA * rng.standard_normal(n))
    Y = _dirichlet(rng, S, n)
    return State(T, P, Y)


def draw_bimodal_state(rng, S: int, n: int) -> State:
    """T from a 50/50 mixture of N(800, 100) and N(2800, 150) K; P and Y as above."""
    hot = rng.random(n) < 0.5
    T = np.where(hot, rng.normal(2800.0, 150.0, n), rng.normal(800.0, 100.0, n))
    P = P_MEDIAN * np.exp(P_SIGMA * rng.standard_normal(n))
    Y = _dirichlet(rng, S, n)
    return State(T, P, Y)


def draw_block_state(rng, S: int, edge: int, coarse: int = 64, smooth: float = 2.0) -> State:
    """Smooth 3-D block of edge^3 cells (x fastest), CPU version for small edges.

    Three fields xi, c, p in [0, 1]: white noise on a coarse^3 grid, Gaussian
    smoothing (sigma = ``smooth`` coarse cells, via FFT), standardisation, the
    normal CDF, then trilinear upsampling to edge^3.
    T = 300 + 2900 c K, P = 5 + 15 p MPa,
    Y = (1 - c) [(1 - xi) Y_lox + xi Y_ch4] + c D_cell with Y_lox / Y_ch4
    dominated by species 0 / 1 and D_cell ~ Dirichlet(0.5).
    """
    fields = [_smooth_field(rng, coarse, smooth) for _ in range(3)]
    xi, c, p = (_upsample(f, edge).reshape(-1) for f in fields)
    n = edge ** 3
    T = 300.0 + 2900.0 * c
    P = 5.0e6 + 15.0e6 * p
    y_lox = 0.05 * _dirichlet(rng, S, 1)[:, 0]
    y_lox[0] += 0.95
    y_ch4 = 0.05 * _dirichlet(rng, S, 1)[:, 0]
    y_ch4[1] += 0.95
    D = _dirichlet(rng, S, n)
    Y = (1.0 - c) * ((1.0 - xi) * y_lox[:, None] + xi * y_ch4[:, None]) + c * D
    Y /= Y.sum(axis=0)
    return State(T, P, Y)



def make_block_state_device(config: int, edge: int, S: int = 29, device="cuda",
                            coarse: int = 64, smooth: float = 2.0, slab_cells: int = 1 << 22):
    """The block workload drawn on a torch device, for blocks too large for the
    host generator (512^3 cells hold 33 GB of FP64 state).

    Same construction as draw_block_state: the three coarse smooth fields and
    the two reference compositions come from this workload's "inputs" stream
    on the host; the trilinear upsampling runs on the device; the per-cell
    Dirichlet(0.5) draws come from a torch generator seeded from the same
    stream, slab by slab.  Returns (T [n], P [n], Y [S][n]) FP64 tensors.
    """
    import torch
    rng = streams(config)["inputs"]
    fields = [_smooth_field(rng, coarse, smooth) for _ in range(3)]
    y_lox = 0.05 * _dirichlet(rng, S, 1)[:, 0]
    y_lox[0] += 0.95
    y_ch4 = 0.05 * _dirichlet(rng, S, 1)[:, 0]
    y_ch4[1] += 0.95
    gen = torch.Generator(device=device)
    gen.manual_seed(int(rng.integers(1 << 62)))
    n = edge ** 3
    f64 = dict(dtype=torch.float64, device=device)
    m = coarse
    x = (torch.arange(edge, **f64) + 0.5) * (m / edge) - 0.5
    i0 = torch.clamp(torch.floor(x).long(), 0, m - 1)
    i1 = torch.clamp(i0 + 1, 0, m - 1)
    t = torch.clamp(x - i0, 0.0, 1.0)

    def upsample(f):                   # [z][y][x] like _upsample
        f = torch.as_tensor(f, **f64)
        g = f[i0] * (1 - t)[:, None, None] + f[i1] * t[:, None, None]
        g = g[:, i0] * (1 - t)[None, :, None] + g[:, i1] * t[None, :, None]
        g = g[:, :, i0] * (1 - t)[None, None, :] + g[:, :, i1] * t[None, None, :]
        return g.reshape(-1)

    xi, c, p = (upsample(f) for f in fields)
    T = 300.0 + 2900.0 * c
    P = 5.0e6 + 15.0e6 * p
    Y = torch.empty((S, n), **f64)
    ylox = torch.as_tensor(y_lox, **f64)[:, None]
    ych4 = torch.as_tensor(y_ch4, **f64)[:, None]
    alpha = torch.full((S, min(slab_cells, n)), DIRICHLET_ALPHA, **f64)
    for a in range(0, n, slab_cells):
        b = min(n, a + slab_cells)
        g = torch._standard_gamma(alpha[:, : b - a], generator=gen)
        g = g / g.sum(dim=0, keepdim=True).clamp_min(1e-300)
        cs, xs = c[a:b][None, :], xi[a:b][None, :]
        y = (1.0 - cs) * ((1.0 - xs) * ylox + xs * ych4) + cs * g
        Y[:, a:b] = y / y.sum(dim=0, keepdim=True)
    del xi, c, p
    return T, P, Y

def _smooth_field(rng, m, sigma):
    w = rng.standard_normal((m, m, m))
    k = np.fft.fftfreq(m)
    kk = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    f = np.real(np.fft.ifftn(np.fft.fftn(w) * np.exp(-2.0 * (math.pi * sigma) ** 2 * kk)))
    f = (f - f.mean()) / f.std()
    return special.ndtr(f)


def _upsample(f, edge):
    m = f.shape[0]
    x = (np.arange(edge) + 0.5) * (m / edge) - 0.5
    i0 = np.clip(np.floor(x).astype(int), 0, m - 1)
    i1 = np.clip(i0 + 1, 0, m - 1)
    t = np.clip(x - i0, 0.0, 1.0)
    g = f[i0] * (1 - t)[:, None, None] + f[i1] * t[:, None, None]
    g = g[:, i0] * (1 - t)[None, :, None] + g[:, i1] * t[None, :, None]
    g = g[:, :, i0] * (1 - t)[None, None, :] + g[:, :, i1] * t[None, None, :]
    return g  # indexed [z][y][x]


# --------------------------------------------------------------------------- networks
@dataclass
class Net:
    widths: tuple                      # (D, H1, ..., S)
    W: list                            # W[l]: float32 [widths[l+1]][widths[l]]
    b: list                            # b[l]: float32 [widths[l+1]]
    in_mean: np.ndarray                # float64 [D]
    in_std: np.ndarray                 # float64 [D]
    out_mean: np.ndarray               # float64 [S]
    out_std: np.ndarray                # float64 [S]
    lam: float = BOXCOX_LAMBDA

    @property
    def n_layers(self) -> int:
        return len(self.widths) - 1

    def flat_params(self) -> np.ndarray:
        """FP32 flat vector [W1 (out x in, row-major), b1, W2, b2, ...]."""
        parts = []
        for W, b in zip(self.W, self.b):
            parts += [W.reshape(-1), b.reshape(-1)]
        return np.concatenate(parts).astype(np.float32)


def n_params(widths) -> int:
    return sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1))


def xavier_weights(rng, widths, bias_scale: float = 0.0):
    """W ~ U(+-sqrt(6/(fan_in+fan_out))) drawn in FP64 then rounded to FP32.

    Biases are 0 unless ``bias_scale`` > 0, then U(+-bias_scale).
    """
    Ws, bs = [], []
    for i in range(len(widths) - 1):
        fi, fo = widths[i], widths[i + 1]
        a = math.sqrt(6.0 / (fi + fo))
        Ws.append(rng.uniform(-a, a, size=(fo, fi)).astype(np.float32))
        if bias_scale > 0:
            bs.append(rng.uniform(-bias_scale, bias_scale, size=fo).astype(np.float32))
        else:
            bs.append(np.zeros(fo, dtype=np.float32))
    return Ws, bs


def uniform_state_input_moments(S: int, lam: float = BOXCOX_LAMBDA):
    """Exact mean and population std of each input feature of the ODENet input.

    Features: T ~ U(300, 3000); P lognormal (median 10 MPa, sigma 0.3); and,
    for each species, the power-family coordinate (Y^lam - 1)/lam of a
    Dirichlet(0.5) marginal Y ~ Beta(a, b), a = 0.5, b = 0.5 (S - 1), whose raw
    moments are E[Y^k] = B(a + k, b) / B(a, b).
    """
    lo, hi = T_UNIFORM
    mean = [0.5 * (lo + hi)]
    std = [(hi - lo) / math.sqrt(12.0)]
    s2 = P_SIGMA ** 2
    pm = P_MEDIAN * math.exp(0.5 * s2)
    mean.append(pm)
    std.append(pm * math.sqrt(math.expm1(s2)))
    a, b = DIRICHLET_ALPHA, DIRICHLET_ALPHA * (S - 1)
    m1 = math.exp(special.betaln(a + lam, b) - special.betaln(a, b))
    m2 = math.exp(special.betaln(a + 2 * lam, b) - special.betaln(a, b))
    for _ in range(S):
        mean.append((m1 - 1.0) / lam)
        std.append(math.sqrt(m2 - m1 * m1) / lam)
    return np.array(mean), np.array(std)


def make_net(config: int, widths=None, bias_scale: float = 0.0, out_stats: bool = False) -> Net:
    """Random-init network of a workload with exact input Z-score statistics.

    Output statistics are the identity (mean 0, std 1): an untrained net's
    raw output is taken as the normalised Box-Cox increment.  With
    ``out_stats`` they are drawn instead (a trained net's label statistics
    stand-in): mean ~ U(-0.2, 0.2), std ~ U(0.5, 2), from the "stats" stream.
    ``bias_scale`` > 0 draws every layer's biases from U(+-bias_scale).
    """
    if widths is None:
        widths = NET_SMALL if config in (1, 4) else NET_ODENET if config == 6 else NET_LARGE
    rng = streams(config)["weights"]
    W, b = xavier_weights(rng, widths, bias_scale)
    S = widths[-1]
    mu, sd = uniform_state_input_moments(S)
    om, osd = np.zeros(S), np.ones(S)
    if out_stats:
        r = streams(config)["stats"]
        om = r.uniform(-0.2, 0.2, size=S)
        osd = r.uniform(0.5, 2.0, size=S)
    return Net(tuple(widths), W, b, mu, sd, om, osd)


def make_state(config: int, n: int, stream: str = "inputs", S: int | None = None) -> State:
    """Seeded input states of a workload (n cells)."""
    if S is None:
        S = 17 if config in (1, 4, 6) else 29
    rng = streams(config)[stream]
    if config == 3:
        return draw_bimodal_state(rng, S, n)
    if config == 5:
        edge = round(n ** (1.0 / 3.0))
        if edge ** 3 != n:
            raise ValueError("config 5 needs a cube cell count")
        return draw_block_state(rng, S, edge)
    return draw_uniform_state(rng, S, n)


def draw_prop_inputs(rng, n: int) -> np.ndarray:
    """Inputs of the property networks, [3][n] float64: specific internal
    energy E (J/kg), pressure p (Pa) and mixture fraction xi of a LOX/CH4
    mixing layer.  xi ~ Beta(0.5, 0.5) (most cells near one of the two
    streams), a reaction progress c ~ U(0, 1), E = -3.5e6 (1 - xi) - 1.0e6 xi
    + 2.5e6 c, and p lognormal around 10 MPa (sigma 0.3) as for the chemistry
    states."""
    xi = rng.beta(0.5, 0.5, size=n)
    c = rng.uniform(0.0, 1.0, size=n)
    E = -3.5e6 * (1.0 - xi) - 1.0e6 * xi + 2.5e6 * c
    p = P_MEDIAN * np.exp(P_SIGMA * rng.standard_normal(n))
    return np.vstack([E, p, xi])


def make_prop_inputs(config: int, n: int, stream: str = "inputs") -> np.ndarray:
    """Seeded property-network inputs of workload 7 or 8 (n cells)."""
    if config not in PROP_NETS:
        raise ValueError("property workloads are 7 and 8")
    return draw_prop_inputs(streams(config)[stream], n)


def make_prop_net(config: int, widths=None, bias_scale: float = 0.0) -> Net:
    """Random-init property network of workload 7 (density) or 8 (temperature
    and transport properties): Xavier weights, input Z-score statistics (FP64
    mean, population std) of a 65,536-cell calibration draw, and the stated
    output scales."""
    if widths is None:
        widths = PROP_NETS[config]
    rng = streams(config)["weights"]
    W, b = xavier_weights(rng, widths, bias_scale)
    cal = make_prop_inputs(config, 65536, stream="calibration")
    om, osd = PROP_OUT[config]
    K = widths[-1]
    om = np.resize(np.asarray(om, np.float64), K)
    osd = np.resize(np.asarray(osd, np.float64), K)
    return Net(tuple(widths), W, b, cal.mean(axis=1), cal.std(axis=1), om, osd)


def make_thermo(config: int, S: int):
    """Per-species formation enthalpy h_f [J/kg] ~ U(-0.5, 0.5) MJ/kg and constant
    c_p [J/(kg K)] ~ U(1000, 2500); reference temperature 298.15 K."""
    rng = streams(config)["extra"]
    hf = rng.uniform(-0.5e6, 0.5e6, size=S)
    cp = rng.uniform(1000.0, 2500.0, size=S)
    return hf, cp, 298.15


def make_molar_masses(config: int, S: int) -> np.ndarray:
    """Species molar masses [S] in kg/mol, log-uniform on [2e-3, 2e-1] (from
    hydrogen to heavy hydrocarbons); drawn after make_thermo's values on the
    same stream."""
    rng = streams(config)["extra"]
    rng.uniform(size=2 * S)                      # the thermo table's draws
    return np.exp(rng.uniform(np.log(2e-3), np.log(2e-1), size=S))


# --------------------------------------------------------------------------- mechanism
ATOMIC_MASS = np.array([12.011, 1.008, 15.999, 14.007]) * 1e-3   # kg/mol: C, H, O, N


@dataclass
class Mechanism:
    comp: np.ndarray        # int [S][4] element counts
    W: np.ndarray           # [S] molar mass kg/mol
    nu_f: np.ndarray        # int [R][S] reactant coefficients
    nu_r: np.ndarray        # int [R][S] product coefficients
    A: np.ndarray           # [R] pre-exponential, SI units (m^3/mol)^(order-1)/s
    b: np.ndarray           # [R] temperature exponent
    Ea: np.ndarray          # [R] activation energy J/mol
    hf: np.ndarray          # [S] J/kg
    cp: np.ndarray          # [S] J/(kg K)
    t_ref: float = 298.15
    A_cgs: np.ndarray = field(default=None)   # [R] pre-exponential as drawn, cm-mol-s

    @property
    def S(self):
        return self.comp.shape[0]

    @property
    def R(self):
        return self.nu_f.shape[0]


def make_mechanism(config: int = 4, S: int = 17, R: int = 40, n_base: int = 6) -> Mechanism:
    """Seeded element-conserving mechanism.

    ``n_base`` base species get random element counts in {0..3}^4 (not all 0);
    the other S - n_base species are sums of two base species, so balanced
    reactions exist by construction.  All element-balanced pairs (reactants,
    products) with one or two species per side are enumerated and R distinct
    ones drawn; the draw is repeated until every species takes part.
    Arrhenius parameters: log10 A ~ U(8, 14) (cm-mol-s), b ~ U(-1, 1),
    Ea ~ U(0, 200) kJ/mol.
    """
    rng = streams(config)["mechanism"]
    while True:
        base = rng.integers(0, 4, size=(n_base, 4))
        if (base.sum(axis=1) == 0).any():
            continue
        pairs = list(itertools.combinations_with_replacement(range(n_base), 2))
        pick = rng.choice(len(pairs), size=S - n_base, replace=False)
        comp = np.vstack([base] + [base[pairs[k][0]] + base[pairs[k][1]] for k in pick])
        sides = [(i,) for i in range(S)] + list(itertools.combinations_with_replacement(range(S), 2))
        vec = [comp[list(s)].sum(axis=0) for s in sides]
        cand = []
        for i, j in itertools.permutations(range(len(sides)), 2):
            if np.array_equal(vec[i], vec[j]):
                cand.append((sides[i], sides[j]))
        if len(cand) < R:
            continue
        for _ in range(50):
            sel = rng.choice(len(cand), size=R, replace=False)
            used = set()
            for k in sel:
                used.update(cand[k][0])
                used.update(cand[k][1])
            if len(used) == S:
                break
        else:
            continue
        break
    nu_f = np.zeros((R, S), dtype=np.int64)
    nu_r = np.zeros((R, S), dtype=np.int64)
    for r, k in enumerate(sel):
        for s in cand[k][0]:
            nu_f[r, s] += 1
        for s in cand[k][1]:
            nu_r[r, s] += 1
    W = comp @ ATOMIC_MASS
    A_cgs = 10.0 ** rng.uniform(8.0, 14.0, size=R)
    order = nu_f.sum(axis=1)
    A = A_cgs * (1e-6) ** (order - 1)         # (cm^3/mol)^(o-1)/s -> (m^3/mol)^(o-1)/s
    b = rng.uniform(-1.0, 1.0, size=R)
    Ea = rng.uniform(0.0, 200.0e3, size=R)
    hf = rng.uniform(-0.5e6, 0.5e6, size=S)
    cp = rng.uniform(1000.0, 2500.0, size=S)
    return Mechanism(comp, W, nu_f, nu_r, A, b, Ea, hf, cp, 298.15, A_cgs)


def subsample_indices(config: int, n: int, k: int) -> np.ndarray:
    """Seeded sorted sample of k distinct cell indices out of n."""
    rng = streams(config)["subsample"]
    if k >= n:
        return np.arange(n)
    return np.sort(rng.choice(n, size=k, replace=False))
