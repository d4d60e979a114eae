"""GPU parity of the training path (chem_dnn_mlp_forward / _mlp_backward /
_train_step and the autograd Function) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import chem, train
from tests.helpers import dev_state, make_handle, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WIDTHS = synth.NET_SMALL


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _tensor_rel(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30))


def _per_tensor(g, widths):
    W, b = train.unflatten(g, widths)
    return W + b


def _setup(B, seed=0):
    net = synth.make_net(4)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((WIDTHS[0], B))
    t = 0.5 * rng.standard_normal((WIDTHS[-1], B))
    return net, x, t


@pytest.mark.parametrize("B", [4096, 1000, 65536])
def test_forward_backward_match_fp64(B):
    """Forward, every gradient tensor and grad_x against the FP64 oracle
    (1e-4 relative per tensor), recomputed pre-activations bitwise equal to
    saved ones; 65,536 is the benchmark's batch, whose weight gradients use
    the per-layer batch splits of that size (32 to 256 splits)."""
    print(f"case train fwd/bwd B={B}", flush=True)
    net, x, t = _setup(B)
    h = make_handle(net, "fp32", max_batch=B)
    p = torch.tensor(net.flat_params(), device="cuda")
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    saved = torch.empty((sum(WIDTHS[1:-1]), B), dtype=torch.float32, device="cuda")
    out = h.mlp_forward(xd, p, saved)
    p64 = net.flat_params().astype(np.float64)
    x32 = x.astype(np.float32).astype(np.float64)
    o_ref, zs = train.forward(x32, p64, WIDTHS)
    np.testing.assert_allclose(out.cpu().numpy(), o_ref, rtol=1e-4, atol=1e-5)
    _, go = train.mse(o_ref, t)
    god = torch.tensor(go, dtype=torch.float32, device="cuda")
    gp, gx = h.mlp_backward(xd, p, saved, god, want_grad_x=True)
    g_ref, gx_ref = train.backward(x32, p64, WIDTHS, zs, go.astype(np.float32).astype(np.float64))
    torch.cuda.synchronize()
    gpn = gp.cpu().numpy().astype(np.float64)
    for a, r in zip(_per_tensor(gpn, WIDTHS), _per_tensor(g_ref, WIDTHS)):
        assert _tensor_rel(a, r) <= 1e-4
    assert _tensor_rel(gx.cpu().numpy(), gx_ref) <= 1e-4
    # recomputation of the pre-activations gives bitwise the same gradient
    gp2, _ = h.mlp_backward(xd, p, None, god)
    gp3, _ = h.mlp_backward(xd, p, saved, god)
    torch.cuda.synchronize()
    assert torch.equal(gp2, gp) and torch.equal(gp3, gp)


def test_train_step_matches_fp64_and_is_reproducible():
    B = 2048 + 7
    print(f"case train_step B={B}", flush=True)
    net = synth.make_net(4)
    st = synth.make_state(4, B)
    rng = np.random.default_rng(3)
    tgt = 0.3 * rng.standard_normal((17, B))
    h = make_handle(net, "fp32", max_batch=4096)
    T, P, Y = dev_state(st)
    td = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    res = []
    for recompute in (False, True):
        p = torch.tensor(net.flat_params(), device="cuda")
        m = torch.zeros_like(p)
        v = torch.zeros_like(p)
        g = torch.empty_like(p)
        losses = []
        for k in (1, 2, 3):
            loss = h.train_step(T, P, Y, td, p, g, m, v, k, lr=1e-3, recompute=recompute)
            losses.append(float(loss.item()))
        torch.cuda.synchronize()
        res.append((p.cpu().numpy(), g.cpu().numpy(), losses))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    # oracle: features in FP64 from the same statistics, three Adam steps
    x = chem.features(st.T, st.P, st.Y, net.in_mean, net.in_std, net.lam)
    q = net.flat_params().astype(np.float64)
    mm = np.zeros_like(q)
    vv = np.zeros_like(q)
    for k in (1, 2, 3):
        r = train.train_step(x, tgt.astype(np.float32).astype(np.float64), q, mm, vv, k, WIDTHS)
        assert abs(r["loss"] - res[0][2][k - 1]) <= 1e-5 * r["loss"]
        last_g = r["grads"]
        q, mm, vv = r["params"], r["m"], r["v"]
    for a, b in zip(_per_tensor(res[0][1].astype(np.float64), WIDTHS), _per_tensor(last_g, WIDTHS)):
        assert _tensor_rel(a, b) <= 1e-3
    # Adam moves every parameter by about lr per step whatever |g| is, so a
    # gradient at rounding level may flip one step; nearly all agree closely
    d = np.abs(res[0][0] - q)
    assert np.mean(d > 1e-5) < 1e-3 and d.max() <= 6.1e-3


def test_train_step_at_benchmark_batch():
    """One Adam step at the benchmark's batch of 65,536 states: the loss (its
    partial sums reduced by one wave) against the FP64 oracle's forward and
    MSE to 1e-5, and two runs from the same parameters bitwise equal (the
    split reductions have a fixed order)."""
    B = 65536
    print(f"case train_step full batch B={B}", flush=True)
    net = synth.make_net(4)
    st = synth.make_state(4, B)
    tgt = 0.3 * np.random.default_rng(5).standard_normal((17, B))
    h = make_handle(net, "fp32", max_batch=B)
    T, P, Y = dev_state(st)
    td = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    runs = []
    for _ in range(2):
        p = torch.tensor(net.flat_params(), device="cuda")
        m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.empty_like(p)
        loss = h.train_step(T, P, Y, td, p, g, m, v, 1, lr=1e-3)
        torch.cuda.synchronize()
        runs.append((float(loss.item()), p.cpu().numpy(), g.cpu().numpy()))
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])
    x = chem.features(st.T, st.P, st.Y, net.in_mean, net.in_std, net.lam)
    o_ref, _ = train.forward(x, net.flat_params().astype(np.float64), WIDTHS)
    l_ref, _ = train.mse(o_ref, tgt.astype(np.float32).astype(np.float64))
    assert abs(runs[0][0] - l_ref) <= 1e-5 * l_ref


def test_autograd_function_matches_finite_differences():
    print("case autograd", flush=True)
    from paper_2508_18969_amd import autograd_function
    F = autograd_function()
    net, x, t = _setup(512, seed=5)
    h = make_handle(net, "fp32", max_batch=512)
    p = torch.tensor(net.flat_params(), device="cuda", requires_grad=True)
    xd = torch.tensor(x, dtype=torch.float32, device="cuda", requires_grad=True)
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    for recompute in (False, True):
        out = F.apply(xd, p, h, recompute)
        loss = ((out - td) ** 2).mean()
        gp, gx = torch.autograd.grad(loss, (p, xd))
        p64 = net.flat_params().astype(np.float64)
        o, zs = train.forward(x.astype(np.float32).astype(np.float64), p64, WIDTHS)
        _, go = train.mse(o, t)
        g_ref, gx_ref = train.backward(x.astype(np.float32).astype(np.float64), p64, WIDTHS, zs, go)
        assert _tensor_rel(gp.cpu().numpy(), g_ref) <= 1e-4
        assert _tensor_rel(gx.cpu().numpy(), gx_ref) <= 1e-4
    # directional finite difference through the GPU forward
    d = torch.randn_like(p) * 1e-3
    with torch.no_grad():
        lp = ((F.apply(xd, p + d, h, False) - td) ** 2).mean().double()
        lm = ((F.apply(xd, p - d, h, False) - td) ** 2).mean().double()
    fd = float((lp - lm) / 2)
    an = float((gp.double() * d.double()).sum())
    assert abs(fd - an) <= 1e-2 * abs(an) + 1e-9


def test_calibration_amax_matches_oracle():
    print("case calibrate", flush=True)
    for cfg in (1, 2):
        net = synth.make_net(cfg)
        st = synth.make_state(cfg, 3000, stream="calibration")
        h = make_handle(net, "fp32")
        T, P, Y = dev_state(st)
        am = h.calibrate(T, P, Y).cpu().numpy().astype(np.float64)
        ref = chem.layer_input_amax(st.T, st.P, st.Y, net)
        np.testing.assert_allclose(am, ref, rtol=2e-5)


def test_training_on_integrator_samples():
    """Training the 19-400-200-100-17 net on labels from the FP64 stiff
    integrator (synthetic 17-species, 40-reaction mechanism, dt = 1e-6 s):
    the first Adam steps match the FP64 oracle's, and the loss falls."""
    from oracle import kinetics
    print("case train on integrator labels", flush=True)
    B = 2048
    mech = synth.make_mechanism(4)
    st = synth.make_state(4, B)
    ts = kinetics.training_set(mech, st, 1e-6, synth.BOXCOX_LAMBDA)
    ok = ts["ok"]
    assert ok.mean() > 0.99
    idx = np.nonzero(ok)[0]
    sub = synth.State(st.T[idx], st.P[idx], np.ascontiguousarray(st.Y[:, idx]))
    # (column selection gives a Fortran-ordered array; the ABI wants rows)
    tgt = np.ascontiguousarray(ts["t"][:, idx])
    # the net normalises its input with the training set's statistics
    net = synth.make_net(4)
    net.in_mean, net.in_std = ts["in_mean"], ts["in_std"]
    h = make_handle(net, "fp32", max_batch=B)
    T, P, Y = dev_state(sub)
    td = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    p = torch.tensor(net.flat_params(), device="cuda")
    m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.empty_like(p)
    x = ts["x"][:, idx]
    q = net.flat_params().astype(np.float64)
    mm, vv = np.zeros_like(q), np.zeros_like(q)
    losses = []
    for k in range(1, 41):
        loss = float(h.train_step(T, P, Y, td, p, g, m, v, k, lr=1e-3).item())
        losses.append(loss)
        if k <= 3:
            r = train.train_step(x, tgt.astype(np.float32).astype(np.float64), q, mm, vv, k, WIDTHS)
            q, mm, vv = r["params"], r["m"], r["v"]
            assert abs(r["loss"] - loss) <= 1e-5 * r["loss"], (k, r["loss"], loss)
    print(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f} after 40 Adam steps", flush=True)
    assert losses[-1] < 0.7 * losses[0]


def test_binding_rejects_wrong_layouts():
    """Field arrays reach the C ABI as [rows][ld] with the cell index fastest;
    the binding refuses a transposed or Fortran-ordered tensor instead of
    passing it with the wrong strides."""
    print("case binding layouts", flush=True)
    net = synth.make_net(4)
    st = synth.make_state(4, 256)
    h = make_handle(net, "fp32", max_batch=256)
    T, P, Y = dev_state(st)
    p = torch.tensor(net.flat_params(), device="cuda")
    m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.empty_like(p)
    tgt_f = torch.tensor(np.asfortranarray(np.zeros((17, 256))), dtype=torch.float32, device="cuda")
    assert tgt_f.stride() == (1, 17)
    with pytest.raises(ValueError):
        h.train_step(T, P, Y, tgt_f, p, g, m, v, 1)
    with pytest.raises(ValueError):
        h.step(T, P, Y.t().contiguous().t())
    with pytest.raises(ValueError):
        h.step(T.float(), P, Y)
    # the same data in row layout is accepted
    h.train_step(T, P, Y, tgt_f.contiguous(), p, g, m, v, 1)
    torch.cuda.synchronize()


def test_set_params_after_training():
    """Train a few Adam steps on an FP32 handle, load the trained parameters
    into separate inference handles with chem_dnn_set_params (FP32 and BF16;
    FP8 re-derives its weight scales), and compare their updates with the
    oracle evaluating the trained parameters."""
    import dataclasses
    print("case set_params after training", flush=True)
    B = 2048
    net = synth.make_net(4)
    st = synth.make_state(4, B)
    rng = np.random.default_rng(11)
    tgt = torch.tensor(0.3 * rng.standard_normal((17, B)), dtype=torch.float32, device="cuda")
    ht = make_handle(net, "fp32", max_batch=B)
    T, P, Y = dev_state(st)
    p = torch.tensor(net.flat_params(), device="cuda")
    m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.empty_like(p)
    for k in range(1, 6):
        ht.train_step(T, P, Y, tgt, p, g, m, v, k, lr=1e-2)
    torch.cuda.synchronize()
    pt = p.cpu().numpy()
    W, b = train.unflatten(pt, WIDTHS)
    trained = dataclasses.replace(net, W=[w.astype(np.float32) for w in W],
                                  b=[x.astype(np.float32) for x in b])
    assert np.max(np.abs(pt - net.flat_params())) > 1e-3        # the weights did move
    thermo = synth.make_thermo(4, 17)
    ref = chem.step(st.T, st.P, st.Y, trained, thermo=thermo)
    h32 = make_handle(net, "fp32", thermo=thermo)               # packed from the initial weights
    h32.set_params(p)
    Y32, T32 = h32.step(T, P, Y)
    hb = make_handle(net, "bf16", thermo=thermo)
    hb.set_params(p)
    Yb, Tb = hb.step(T, P, Y)
    torch.cuda.synchronize()
    assert rel_err(Y32.cpu().numpy(), ref["Y_new"]) <= 1e-5
    assert rel_err(T32.cpu().numpy(), ref["T_new"], floor=1.0) <= 1e-5
    # BF16 after set_params equals BF16 built from the trained weights
    hb2 = make_handle(trained, "bf16", thermo=thermo)
    Yb2, Tb2 = hb2.step(T, P, Y)
    torch.cuda.synchronize()
    assert torch.equal(Yb, Yb2) and torch.equal(Tb, Tb2)
    # FP8: set_params re-derives the weight scales from the new weights
    amax = chem.layer_input_amax(st.T, st.P, st.Y, trained).astype(np.float32)
    h8 = make_handle(net, "fp8", thermo=thermo, act_amax=amax)
    h8.set_params(p)
    h8b = make_handle(trained, "fp8", thermo=thermo, act_amax=amax)
    Y8, _ = h8.step(T, P, Y)
    Y8b, _ = h8b.step(T, P, Y)
    torch.cuda.synchronize()
    assert torch.equal(Y8, Y8b)
