"""The allocation-free training step (chem_dnn_train_step_noalloc) against
chem_dnn_train_step: two calls in a row, the second on a smaller batch, equal
bit for bit (the same kernels and schedule; only where the scratch lives
differs), and a batch beyond the static scratch rejected."""
import numpy as np
import pytest

import synth
from paper_2508_18969_amd import binding
from tests.helpers import dev_state, make_handle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _state(B, seed):
    net = synth.make_net(4, bias_scale=0.05)
    st = synth.make_state(4, B)
    tgt = 0.3 * np.random.default_rng(seed).standard_normal((17, B))
    return net, st, tgt


def _one_step(h, st, tgt, p0, step, noalloc):
    T, P, Y = dev_state(st)
    td = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    p = p0.clone()
    g = torch.full_like(p, float("nan"))
    m = torch.full_like(p, 1e-3)
    v = torch.full_like(p, 2e-6)
    f = h.train_step_noalloc if noalloc else h.train_step
    loss = f(T, P, Y, td, p, g, m, v, step)
    torch.cuda.synchronize()
    return [loss.cpu(), p.cpu(), g.cpu(), m.cpu(), v.cpu()]


@pytest.mark.parametrize("chunk", [0, 1024])
def test_noalloc_step_equals_workspace_step(chunk):
    """Batches of 4,096 and then 1,000 samples (the second call finds the
    first call's contents in the shared scratch): loss, gradient, parameters
    and both Adam moments equal those of chem_dnn_train_step bit for bit, for
    a whole-batch and a chunked schedule."""
    print(f"case noalloc train step chunk={chunk}", flush=True)
    net, _, _ = _state(16, 0)
    ref = make_handle(net, "fp32", max_batch=4096, recompute_chunk=chunk)
    na = make_handle(net, "fp32", max_batch=0, recompute_chunk=chunk)
    p0 = ref._params
    for B, step, seed, stream in ((4096, 1, 1, "inputs"), (1000, 3, 2, "calibration")):
        st = synth.make_state(4, B, stream=stream)
        tgt = 0.3 * np.random.default_rng(seed).standard_normal((17, B))
        a = _one_step(ref, st, tgt, p0, step, False)
        b = _one_step(na, st, tgt, p0, step, True)
        print(f"  B={B}: loss {float(a[0]):.6e} / {float(b[0]):.6e}", flush=True)
        assert np.isfinite(float(b[0]))
        for x, y in zip(a, b):
            assert torch.equal(x, y)


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    """A batch whose per-sample buffers exceed the static scratch is refused
    with ETOOLARGE before anything is enqueued; a chunked handle takes it."""
    net, _, _ = _state(16, 0)
    h = make_handle(net, "fp32")
    B = 1 << 16
    st = synth.make_state(4, B)
    T, P, Y = dev_state(st)
    td = torch.zeros((17, B), dtype=torch.float32, device="cuda")
    p = h._params.clone()
    g, m, v = torch.empty_like(p), torch.zeros_like(p), torch.zeros_like(p)
    with pytest.raises(binding.ChemDNNError) as e:
        h.train_step_noalloc(T, P, Y, td, p, g, m, v, 1)
    assert e.value.status == binding.ETOOLARGE
    hc = make_handle(net, "fp32", recompute_chunk=4096)
    loss = hc.train_step_noalloc(T, P, Y, td, p, g, m, v, 1)
    torch.cuda.synchronize()
    assert np.isfinite(float(loss.item()))
