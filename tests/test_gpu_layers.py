"""Layer-isolated parity of the matrix-core paths (chem_dnn_debug_layers).

End-to-end comparison of a narrow-format network with its emulation can
only be statistical: the two sides accumulate in different precisions, so an
activation near a rounding boundary may round one ulp apart and the flip
propagates.  Layer by layer the check is exact.  The library's debug build of
the same kernels dumps, for a small batch, every layer's input operand values
(as the matrix cores received them) and its FP32 accumulators.  Per layer:

1. Products.  The accumulators are compared with the exact FP64 product of
   the very same operands (the GPU's inputs, the oracle's rounding of the
   FP32 master weights): |acc - ref| <= gamma_K sum |q(w) q(a)| + 1 ulp(acc),
   gamma_K = K u / (1 - K u), u = 2^-24, K the number of terms (fan-in, plus
   one when the accumulator starts at the bias) - Higham's bound for any
   order of FP32 summation (Accuracy and Stability of Numerical Algorithms,
   2nd ed., Sec. 3.1).  The FP8 instruction accumulates each 128-product
   k-step on a narrower grid (see the FP8 bound below).
2. Activation and rounding.  The next layer's operands are compared with the
   FP64 value q(GELU(z)) computed from the GPU's own accumulators z: equal,
   except where the FP64 value lies within the FP32 evaluation error of the
   GELU of a rounding boundary of the operand format (then one ulp apart is
   allowed).  FP32 operands: within that evaluation error.
3. Layer 1's operands against the oracle's Z-scored input, the same way.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import chem
from tests.helpers import dev_state, make_handle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U = 2.0 ** -24
FMT = {"fp32": None, "bf16": "bf16", "fp16": "f16", "fp8": "e4m3"}


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gamma(k):
    return k * U / (1.0 - k * U)


def _ulp32(x):
    return np.spacing(np.abs(np.asarray(x, np.float32))).astype(np.float64)


def _gelu_err(z):
    """Bound on the relative error of the FP32 GELU x / (1 + 2^(x p)), p =
    -2 sqrt(2/pi) log2(e) (1 + 0.044715 x^2): the exponent x p carries a
    few roundings of its own size (|x p| u each), which 2^(.) turns into a
    relative error of ln 2 |x p| u; the exp2, the add, the reciprocal and
    the product add a few ulp.  Taken as (3 |x p| + 16) u."""
    z = np.asarray(z, np.float64)
    xp = np.abs(2.0 * chem.SQRT_2_OVER_PI * (z + chem.GELU_CUBIC * z ** 3) / np.log(2.0))
    return (3.0 * xp + 16.0) * U


def _neighbours(q, fmt):
    """The representable values of fmt next to q (below, above)."""
    p, emin, vmax, _ = chem.FORMATS[fmt]
    q = np.asarray(q, np.float64)
    _, E = np.frexp(q)
    e = np.where(q == 0, emin, np.maximum(E - 1, emin))
    step = np.ldexp(1.0, e - (p - 1))
    # just below a power of two the spacing halves
    lo_step = np.where((np.abs(q) == np.ldexp(1.0, e)) & (e > emin), step / 2, step)
    return q - np.where(q > 0, lo_step, step), q + np.where(q < 0, lo_step, step)


def _round(x, fmt):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64) if fmt is None \
        else chem.round_to(x, fmt)


def _check_rounding(q_gpu, x, fmt, rel_err, what):
    """q_gpu = the GPU's operand values for exact values x (FP64), rounded to
    fmt (None: FP32).  The GPU computes x with a relative error of at most
    rel_err (array or scalar; plus 1e-30 absolute), so q_gpu must be the
    rounding of some value within that distance of x: round(x - tol) <=
    q_gpu <= round(x + tol) (rounding is monotone).  Where the interval holds
    one representable value the GPU must match the reference rounding
    exactly; near a rounding boundary it may be the neighbour."""
    x = np.asarray(x, np.float64)
    tol = rel_err * np.abs(x) + 1e-30
    lo, hi = _round(x - tol, fmt), _round(x + tol, fmt)
    ok = (q_gpu >= lo) & (q_gpu <= hi)
    q_ref = _round(x, fmt)
    mism = q_gpu != q_ref
    frac = float(mism.mean())
    _note(f"    {what}: {mism.sum()} of {mism.size} operands differ from the reference rounding "
          f"({100 * frac:.4f} %), all within the error interval: {ok.all()}")
    assert ok.all(), what
    return frac


def _weights(net, fmt, w_scale):
    out = []
    for l, W in enumerate(net.W):
        W64 = np.asarray(W, np.float64)
        if fmt is None:
            out.append(W64)
        else:
            out.append(chem.round_to(W64 / (w_scale[l] if fmt == "e4m3" else 1.0), fmt))
    return out


def _layer_checks(h, net, st, prec, act_s=None, w_s=None):
    fmt = FMT[prec]
    fp8 = prec == "fp8"
    T, P, Y = dev_state(st)
    qin, acc = h.debug_layers(T, P, Y)
    torch.cuda.synchronize()
    qin = [q.cpu().numpy().astype(np.float64) for q in qin]
    acc = [a.cpu().numpy().astype(np.float64) for a in acc]
    L = len(net.W)
    assert all(np.isfinite(q).all() for q in qin) and all(np.isfinite(a).all() for a in acc)
    Wq = _weights(net, fmt, w_s)
    b64 = [np.asarray(b, np.float64) for b in net.b]
    sa = np.ones(L) if act_s is None else np.asarray(act_s, np.float64)
    sw = np.ones(L) if w_s is None else np.asarray(w_s, np.float64)
    # 3. layer 1's operands: the Z-scored input; the FP32 preprocessing is
    # within 2e-6 max(1, |z|) of the FP64 value (Box-Cox power and affine map)
    z0 = chem.features(st.T, st.P, st.Y, net.in_mean, net.in_std, net.lam) / sa[0]
    _check_rounding(qin[0], z0, fmt, 2e-6 * np.maximum(1.0, np.abs(z0)) / np.maximum(np.abs(z0), 1e-30),
                    "layer 1 input")
    worst = 0.0
    for l in range(L):
        K = net.widths[l]
        # 1. products from the GPU's own operands
        ref = Wq[l] @ qin[l]
        mag = np.abs(Wq[l]) @ np.abs(qin[l])
        if not fp8:
            ref = ref + b64[l][:, None]
            mag = mag + np.abs(b64[l])[:, None]
        bound = _gamma(K + (0 if fp8 else 1)) * mag + _ulp32(acc[l])
        r = np.abs(acc[l] - ref) / bound
        worst = max(worst, float(r.max()))
        _note(f"  layer {l + 1} ({K} -> {net.widths[l + 1]}): max |acc - ref| / bound = {r.max():.3f} "
              f"(mean {r.mean():.3f})")
        if fp8:
            # The FP8 matrix instruction sums the 128 products of a k-step on
            # a fixed-point grid aligned to the largest of them: measured on
            # gfx950, 1 + 2^-13 survives and 1 + 2^-14 is lost, while the FP32
            # accumulator it adds to is exact.  Each product thus loses less
            # than 2^-13 max|ab| of its k-step: the bound is, per k-step q,
            # n_q 2^-13 max_q |ab| (n_q nonzero terms), plus FP32 rounding of
            # the running sum over the k-steps (gamma of their count).
            nq = (K + 127) // 128
            fx = np.zeros_like(acc[l])
            for q in range(nq):
                sl = slice(128 * q, min(K, 128 * (q + 1)))
                blk = np.abs(Wq[l][:, sl])[:, :, None] * np.abs(qin[l][sl])[None, :, :]
                fx += (blk > 0).sum(axis=1) * 2.0 ** -13 * blk.max(axis=1)
            bound = fx + _gamma(nq + 1) * mag + _ulp32(acc[l])
            e = np.abs(acc[l] - ref)
            _note(f"    fp8 accumulation: max err / bound = {np.max(e / bound):.3e}, "
                  f"max err / sum|ab| = {np.max(e / np.maximum(mag, 1e-300)):.3e}")
        assert np.all(np.abs(acc[l] - ref) <= bound), f"layer {l + 1} products"
        if l == L - 1:
            break
        # 2. activation and rounding of the next layer's operands
        z = acc[l] * (sa[l] * sw[l]) + b64[l][:, None] if fp8 else acc[l]
        a = chem.gelu(z) / sa[l + 1]
        err = _gelu_err(z)
        if fp8:   # (the FP32 fma that scales the accumulator and adds the bias)
            err = err + U * np.abs(z * chem.gelu_grad(z)) / np.maximum(np.abs(chem.gelu(z)), 1e-300)
        _check_rounding(qin[l + 1], a, fmt, err, f"layer {l + 2} input")
    return worst, acc


@pytest.mark.parametrize("config,prec", [(1, "fp32"), (1, "bf16"), (1, "fp16"), (1, "fp8"),
                                         (2, "fp32"), (2, "bf16"), (2, "fp16"), (2, "fp8")])
def test_fused_layers(config, prec):
    """Both fused networks in every operand format, with random biases and
    output statistics; 200 cells (several tiles and a ragged tail)."""
    _note(f"case fused layers config={config} {prec}")
    net = synth.make_net(config, bias_scale=0.1, out_stats=True)
    act_s = w_s = amax = None
    if prec == "fp8":
        cal = synth.make_state(config, 1 << 14, stream="calibration")
        amax = chem.layer_input_amax(cal.T, cal.P, cal.Y, net).astype(np.float32)
        act_s = chem.pow2_scale(amax.astype(np.float64))
        w_s = chem.pow2_scale(chem.weight_amax(net))
    h = make_handle(net, prec, act_amax=amax)
    st = synth.make_state(config, 200)
    _layer_checks(h, net, st, prec, act_s, w_s)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_layered_layers(prec):
    """The paper-size ODENet (19-2048-4096-2048-1024-512-17) on the
    layer-by-layer path, biases and output statistics, 300 cells."""
    _note(f"case layered layers {prec}")
    net = synth.make_net(6, bias_scale=0.1, out_stats=True)
    h = make_handle(net, prec)
    st = synth.make_state(6, 300)
    _layer_checks(h, net, st, prec)


@pytest.mark.parametrize("config", [1, 2])
def test_dump_is_the_step_network(config):
    """The dump runs the network of chem_dnn_step: for FP32 operands, the
    output accumulators (o, started at the bias) put through the FP64
    post-processing of the oracle reproduce the step's Y_new to the FP32
    post-processing's own error; and o itself is within 1e-5 max(1, |o|_inf)
    of the oracle's FP64 network output, per cell."""
    _note(f"case dump vs step config={config}")
    net = synth.make_net(config, bias_scale=0.1, out_stats=True)
    thermo = synth.make_thermo(config, net.widths[-1])
    h = make_handle(net, "fp32", thermo=thermo)
    st = synth.make_state(config, 333)
    T, P, Y = dev_state(st)
    _, acc = h.debug_layers(T, P, Y)
    Yn, Tn = h.step(T, P, Y)
    torch.cuda.synchronize()
    o = acc[-1].cpu().numpy().astype(np.float64)
    ref = chem.step(st.T, st.P, st.Y, net, thermo=thermo)
    d = np.abs(o - ref["o"]).max(axis=0) / np.maximum(1.0, np.abs(ref["o"]).max(axis=0))
    _note(f"  network output: max per-cell |o - o_ref|_inf / max(1, |o_ref|_inf) = {d.max():.3e}")
    assert np.all(d <= 1e-5)
    y_post, _, _ = chem.post(o, st.T, st.Y, net.out_mean, net.out_std, net.lam, thermo)
    yg = Yn.cpu().numpy()
    rel = np.abs(yg - y_post) / np.maximum(np.abs(y_post), 1e-10)
    _note(f"  Y_new vs FP64 post of the GPU's o: max rel (floor 1e-10) {rel.max():.3e}")
    assert rel.max() <= 1e-5
