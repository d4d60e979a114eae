"""Activation recomputation that saves memory: a handle whose description
sets recompute_chunk keeps the activations of one chunk of samples only.
The training step runs chunk by chunk and accumulates the gradient in chunk
order; the MLP backward recomputes pre-activations per chunk when they were
not saved.  Against the FP64 oracle, and bit for bit against itself."""
import numpy as np
import pytest

import synth
from oracle import chem, train
from paper_2508_18969_amd import binding
from tests.helpers import dev_state, make_handle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WIDTHS = synth.NET_SMALL
H = sum(WIDTHS[1:-1])


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _tensor_rel(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30))


def _per_tensor(g):
    W, b = train.unflatten(g, WIDTHS)
    return W + b


def test_step_at_a_batch_whose_activations_do_not_fit():
    """Batch 131,072 on a handle with 16,384-sample chunks: its workspace is
    smaller than the batch's pre-activations alone (131,072 x 700 FP32), yet
    one Adam step gives the loss within 1e-5 and every gradient tensor within
    1e-4 (relative, per tensor) of the FP64 oracle."""
    B, C = 131072, 16384
    print(f"case chunked train step B={B} chunk={C}", flush=True)
    net = synth.make_net(4)
    st = synth.make_state(4, B)
    tgt = 0.3 * np.random.default_rng(11).standard_normal((17, B))
    h = make_handle(net, "fp32", max_batch=B, recompute_chunk=C)
    assert h._ws_bytes < B * H * 4, (h._ws_bytes, B * H * 4)
    T, P, Y = dev_state(st)
    td = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    p = torch.tensor(net.flat_params(), device="cuda")
    m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.empty_like(p)
    loss = h.train_step(T, P, Y, td, p, g, m, v, 1, lr=1e-3, recompute=True)
    torch.cuda.synchronize()
    x = chem.features(st.T, st.P, st.Y, net.in_mean, net.in_std, net.lam)
    q = net.flat_params().astype(np.float64)
    r = train.train_step(x, tgt.astype(np.float32).astype(np.float64), q, np.zeros_like(q),
                         np.zeros_like(q), 1, WIDTHS)
    lg = float(loss.item())
    print(f"  workspace {h._ws_bytes / 2**20:.1f} MiB vs saved pre-activations "
          f"{B * H * 4 / 2**20:.1f} MiB; loss {lg:.6e} ref {r['loss']:.6e}", flush=True)
    assert abs(lg - r["loss"]) <= 1e-5 * r["loss"]
    gg = g.cpu().numpy().astype(np.float64)
    errs = [_tensor_rel(a, b) for a, b in zip(_per_tensor(gg), _per_tensor(r["grads"]))]
    print(f"  per-tensor gradient errors {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= 1e-4


def test_recomputed_equals_saved_bit_for_bit():
    """On a chunked handle (4 chunks of the 65,536 batch, padded leading
    dimension), the backward with the pre-activations saved by the forward
    and the backward that recomputes them per chunk give the same weight,
    bias and input gradients bit for bit, and those match the FP64 oracle
    (1e-4 per tensor).  The training step too: the same bits with and
    without the recompute flag."""
    B, C, ld = 65536, 16384, 65536 + 64
    print(f"case chunked saved vs recomputed B={B} chunk={C}", flush=True)
    net = synth.make_net(4)
    h = make_handle(net, "fp32", max_batch=B, recompute_chunk=C)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((WIDTHS[0], B))
    tg = 0.5 * rng.standard_normal((WIDTHS[-1], B))
    xd = torch.zeros((WIDTHS[0], ld), dtype=torch.float32, device="cuda")[:, :B]
    xd.copy_(torch.tensor(x, dtype=torch.float32))
    p = torch.tensor(net.flat_params(), device="cuda")
    saved = torch.empty((H, ld), dtype=torch.float32, device="cuda")[:, :B]
    out = h.mlp_forward(xd, p, saved)
    out2 = h.mlp_forward(xd, p)               # chunk by chunk through the scratch
    x32 = x.astype(np.float32).astype(np.float64)
    o_ref, zs = train.forward(x32, net.flat_params().astype(np.float64), WIDTHS)
    _, go = train.mse(o_ref, tg)
    god = torch.zeros((WIDTHS[-1], ld), dtype=torch.float32, device="cuda")[:, :B]
    god.copy_(torch.tensor(go, dtype=torch.float32))
    gp_s, gx_s = h.mlp_backward(xd, p, saved, god, want_grad_x=True)
    gp_r, gx_r = h.mlp_backward(xd, p, None, god, want_grad_x=True)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    assert torch.equal(gp_s, gp_r) and torch.equal(gx_s, gx_r)
    g_ref, gx_ref = train.backward(x32, net.flat_params().astype(np.float64), WIDTHS, zs,
                                   go.astype(np.float32).astype(np.float64))
    gpn = gp_s.cpu().numpy().astype(np.float64)
    errs = [_tensor_rel(a, b) for a, b in zip(_per_tensor(gpn), _per_tensor(g_ref))]
    print(f"  per-tensor gradient errors {['%.1e' % e for e in errs]}", flush=True)
    assert max(errs) <= 1e-4
    assert _tensor_rel(gx_s.cpu().numpy(), gx_ref) <= 1e-4
    # the training step: the flag does not change the schedule of a chunked handle
    st = synth.make_state(4, B)
    T, P, Y = dev_state(st)
    td = torch.tensor(0.3 * rng.standard_normal((17, B)), dtype=torch.float32, device="cuda")
    res = []
    for rc in (False, True):
        q = torch.tensor(net.flat_params(), device="cuda")
        m, v, g = torch.zeros_like(q), torch.zeros_like(q), torch.empty_like(q)
        l = h.train_step(T, P, Y, td, q, g, m, v, 1, recompute=rc)
        torch.cuda.synchronize()
        res.append((float(l.item()), q.cpu(), g.cpu()))
    assert res[0][0] == res[1][0] and torch.equal(res[0][1], res[1][1]) and torch.equal(res[0][2], res[1][2])


def test_chunked_and_whole_batch_agree_with_the_oracle():
    """The same step on a whole-batch handle and on a chunked one (different
    reduction trees, so not bit for bit): both within 1e-4 per gradient
    tensor of the FP64 oracle, and within 2e-4 of each other."""
    B = 4096 + 48
    print(f"case chunked vs whole batch B={B}", flush=True)
    net = synth.make_net(4)
    st = synth.make_state(4, B)
    tgt = 0.3 * np.random.default_rng(12).standard_normal((17, B))
    T, P, Y = dev_state(st)
    td = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    x = chem.features(st.T, st.P, st.Y, net.in_mean, net.in_std, net.lam)
    q = net.flat_params().astype(np.float64)
    r = train.train_step(x, tgt.astype(np.float32).astype(np.float64), q, np.zeros_like(q),
                         np.zeros_like(q), 1, WIDTHS)
    grads = []
    for C in (0, 1024):
        h = make_handle(net, "fp32", max_batch=B, recompute_chunk=C)
        p = torch.tensor(net.flat_params(), device="cuda")
        m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.empty_like(p)
        loss = h.train_step(T, P, Y, td, p, g, m, v, 1)
        torch.cuda.synchronize()
        assert abs(float(loss.item()) - r["loss"]) <= 1e-5 * r["loss"]
        gg = g.cpu().numpy().astype(np.float64)
        errs = [_tensor_rel(a, b) for a, b in zip(_per_tensor(gg), _per_tensor(r["grads"]))]
        print(f"  chunk {C}: per-tensor errors max {max(errs):.1e}", flush=True)
        assert max(errs) <= 1e-4
        grads.append(gg)
    for a, b in zip(_per_tensor(grads[0]), _per_tensor(grads[1])):
        assert _tensor_rel(a, b) <= 2e-4
