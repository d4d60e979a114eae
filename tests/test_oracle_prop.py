"""Pins of the property-network oracle (oracle/prop.py) against facts that do
not come from the oracle itself: an identity of the GELU, brute force on a
tiny net, exact special cases, and invariants of the normalisation."""
import math

import numpy as np

import synth
from oracle import prop


class _Net:
    def __init__(self, W, b, in_mean, in_std, out_mean, out_std):
        self.W, self.b = W, b
        self.in_mean, self.in_std = np.asarray(in_mean, float), np.asarray(in_std, float)
        self.out_mean, self.out_std = np.asarray(out_mean, float), np.asarray(out_std, float)


def test_gelu_pair_network_is_the_identity():
    """GELU(z) - GELU(-z) = z for the tanh form (tanh is odd), so a two-layer
    net with hidden weights [I; -I] and output weights [I, -I] returns z; with
    the output scaling equal to the input normalisation the whole map returns
    the inputs.  A transposed operand, a sign error, a dropped normalisation or
    a swapped output mean/scale breaks this."""
    x = synth.make_prop_inputs(7, 257)
    mu, sd = x.mean(axis=1) * 0.9, x.std(axis=1) * 1.3
    I = np.eye(3)
    net = _Net([np.vstack([I, -I]), np.hstack([I, -I])], [np.zeros(6), np.zeros(3)],
               mu, sd, mu, sd)
    y = prop.evaluate(x, net)["y"]
    np.testing.assert_allclose(y, x, rtol=1e-13, atol=1e-15 * np.abs(x).max())


def test_brute_force_tiny_net():
    """A 3-5-4-2 net evaluated by scalar loops from the definitions."""
    rng = np.random.default_rng(7)
    widths = (3, 5, 4, 2)
    W = [rng.normal(size=(widths[l + 1], widths[l])) for l in range(3)]
    b = [rng.normal(size=widths[l + 1]) for l in range(3)]
    mu, sd = rng.normal(size=3), rng.uniform(0.5, 2.0, size=3)
    om, osd = rng.normal(size=2), rng.uniform(0.5, 2.0, size=2)
    x = rng.normal(size=(3, 6))
    net = _Net(W, b, mu, sd, om, osd)
    y = prop.evaluate(x, net)["y"]

    def gelu(v):
        return 0.5 * v * (1.0 + math.tanh(math.sqrt(2.0 / math.pi) * (v + 0.044715 * v ** 3)))

    for c in range(x.shape[1]):
        a = [(x[f, c] - mu[f]) / sd[f] for f in range(3)]
        for l in range(3):
            z = [sum(W[l][j][k] * a[k] for k in range(len(a))) + b[l][j] for j in range(widths[l + 1])]
            a = [gelu(v) for v in z] if l < 2 else z
        for k in range(2):
            assert abs(y[k, c] - (a[k] * osd[k] + om[k])) <= 1e-12 * max(1.0, abs(y[k, c]))


def test_zero_output_weights_give_the_scaled_bias():
    """With W_L = 0 the output is b_L sigma_out + mu_out exactly, whatever the
    inputs."""
    net = synth.make_prop_net(8)
    W = list(net.W)
    W[-1] = np.zeros_like(W[-1])
    b = [np.zeros_like(v) for v in net.b]
    b[-1] = np.array([0.5, -1.0, 2.0, 0.25], dtype=np.float32)
    n2 = _Net(W, b, net.in_mean, net.in_std, net.out_mean, net.out_std)
    y = prop.evaluate(synth.make_prop_inputs(8, 33), n2)["y"]
    want = b[-1].astype(np.float64) * net.out_std + net.out_mean
    assert np.array_equal(y, np.repeat(want[:, None], 33, axis=1))


def test_normalisation_divides_by_the_scale():
    """Scaling an input's sigma by 2 and its first-layer weights by 2 leaves
    the output unchanged (exactly, up to rounding)."""
    net = synth.make_prop_net(7, widths=(3, 16, 8, 1))
    x = synth.make_prop_inputs(7, 64)
    y0 = prop.evaluate(x, net)["y"]
    W = [w.astype(np.float64) for w in net.W]
    W[0] = W[0] * 2.0
    n2 = _Net(W, net.b, net.in_mean, net.in_std * 2.0, net.out_mean, net.out_std)
    np.testing.assert_allclose(prop.evaluate(x, n2)["y"], y0, rtol=1e-14, atol=0)


def test_cells_are_independent():
    net = synth.make_prop_net(7, widths=(3, 32, 16, 1))
    x = synth.make_prop_inputs(7, 50)
    perm = np.random.default_rng(3).permutation(50)
    np.testing.assert_array_equal(prop.evaluate(x[:, perm], net)["y"], prop.evaluate(x, net)["y"][:, perm])


def test_input_statistics_normalise_the_calibration_draw():
    """The stored statistics are the FP64 mean and population std of the
    calibration draw: its features have mean 0 and std 1."""
    for cfg in (7, 8):
        net = synth.make_prop_net(cfg)
        z = prop.features(synth.make_prop_inputs(cfg, 65536, stream="calibration"), net.in_mean, net.in_std)
        assert np.abs(z.mean(axis=1)).max() < 1e-12
        assert np.abs(z.std(axis=1) - 1.0).max() < 1e-12


def test_input_recipe():
    """E, p and xi stay in their stated ranges; xi is bimodal."""
    x = synth.make_prop_inputs(7, 100000)
    E, p, xi = x
    assert (xi >= 0).all() and (xi <= 1).all()
    assert E.min() >= -3.5e6 and E.max() <= 1.5e6
    assert abs(np.median(p) / 1e7 - 1) < 0.01
    assert np.mean(xi < 0.1) > 0.19 and np.mean(xi > 0.9) > 0.19    # Beta(1/2, 1/2): 0.205 each
