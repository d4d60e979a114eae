"""Training at the benchmark batch on labels from the stiff integrator: the
19-400-200-100-17 network, batch 65,536, Adam lr 1e-3, several hundred steps
(the differentiation pattern of the chemistry update, trained on samples
from the FP64 integrator of the synthetic 17-species, 40-reaction mechanism
with dt = 1e-6 s).  Label generation is timed on its own; the loss curve,
the training time per step and a held-out loss are printed."""
import time

import numpy as np
import pytest

import synth
from oracle import kinetics, train
from tests.helpers import dev_state, make_handle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

B = 65536
STEPS = 300
DT = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _labels(mech, st, chunk=8192):
    """Integrator labels in chunks (progress printed per chunk); returns the
    training_set dict of the whole batch."""
    from oracle.chem import boxcox
    lam = synth.BOXCOX_LAMBDA
    M = kinetics.Mech(mech)
    n = st.T.size
    Y1 = np.empty_like(st.Y)
    ns = np.empty(n, np.int32)
    t0 = time.perf_counter()
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        _, Y1[:, a:b], ns[a:b] = kinetics.integrate(M, st.T[a:b], st.P[a:b],
                                                     np.ascontiguousarray(st.Y[:, a:b]), DT)
        print(f"  labels {b}/{n} ({time.perf_counter() - t0:.1f} s)", flush=True)
    x = np.vstack([st.T[None], st.P[None], boxcox(st.Y, lam)])
    d = boxcox(Y1, lam) - boxcox(st.Y, lam)
    return x, d, ns, time.perf_counter() - t0


@pytest.mark.timeout(900)
def test_training_at_batch_65536_on_integrator_labels():
    """65,536 integrator labels; 300 Adam steps over the whole batch on the
    GPU.  The first step's loss matches the FP64 oracle's (1e-5 relative);
    the training loss falls below 0.35 of its start and the loss on 4,096
    held-out states (labels from the same integrator, normalised with the
    training statistics) below 0.5 of its start."""
    print(f"case train on {B} integrator labels, {STEPS} Adam steps", flush=True)
    mech = synth.make_mechanism(4)
    st = synth.make_state(4, B)
    x, d, ns, t_lab = _labels(mech, st)
    assert (ns > 0).all(), "integrator failed on some states"
    in_mean, in_std = x.mean(axis=1), x.std(axis=1)
    out_mean, out_std = d.mean(axis=1), d.std(axis=1)
    out_std = np.where(out_std > 0, out_std, 1.0)
    tgt = np.ascontiguousarray((d - out_mean[:, None]) / out_std[:, None])
    print(f"  label generation: {B} states in {t_lab:.1f} s ({B / t_lab:.0f} states/s, "
          f"{ns.mean():.0f} integrator steps per state on average)", flush=True)

    net = synth.make_net(4)
    net.in_mean, net.in_std = in_mean, in_std
    h = make_handle(net, "fp32", max_batch=B)
    T, P, Y = dev_state(st)
    td = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    p = torch.tensor(net.flat_params(), device="cuda")
    m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.empty_like(p)
    q0 = net.flat_params().astype(np.float64)
    # the oracle's first step on the same features (FP32 inputs, as the GPU sees them)
    xz = ((x - in_mean[:, None]) / in_std[:, None]).astype(np.float32).astype(np.float64)
    r = train.train_step(xz, tgt.astype(np.float32).astype(np.float64), q0, np.zeros_like(q0),
                         np.zeros_like(q0), 1, list(net.widths))

    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, STEPS + 1):
        lt = h.train_step(T, P, Y, td, p, g, m, v, k, lr=1e-3)
        losses.append(lt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / STEPS * 1e3
    losses = [float(l.item()) for l in losses]
    assert abs(losses[0] - r["loss"]) <= 1e-5 * r["loss"], (losses[0], r["loss"])
    curve = ", ".join(f"{k}: {losses[k - 1]:.4f}" for k in (1, 10, 25, 50, 100, 150, 200, 250, 300))
    print(f"  loss curve (step: loss) {curve}", flush=True)
    print(f"  training: {ms:.3f} ms per Adam step at batch {B} (wall clock, {STEPS} steps)", flush=True)
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.35 * losses[0]

    # held-out states of the same distribution
    sh = synth.make_state(4, 4096, stream="calibration")
    xh, dh, nsh, _ = _labels(mech, sh, chunk=4096)
    assert (nsh > 0).all()
    zh = (xh - in_mean[:, None]) / in_std[:, None]
    th = (dh - out_mean[:, None]) / out_std[:, None]
    o0, _ = train.forward(zh, q0, list(net.widths))
    o1, _ = train.forward(zh, p.cpu().numpy().astype(np.float64), list(net.widths))
    l0, _ = train.mse(o0, th)
    l1, _ = train.mse(o1, th)
    print(f"  held-out loss (4096 states): {l0:.4f} before, {l1:.4f} after training", flush=True)
    assert l1 < 0.5 * l0
