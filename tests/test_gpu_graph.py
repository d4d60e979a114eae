"""The library's entry points under HIP graph capture: chem_dnn_step (fused
and layer-by-layer paths), chem_dnn_step_source and chem_prop_eval enqueue
only kernel launches, so a captured graph replays them; every replay, with
eager work and synchronisations between the replays, must equal the eager
result bit for bit (and the eager result is the oracle-checked one of the
other tests)."""
import sys

import numpy as np
import pytest

import synth
from tests.helpers import dev_state, make_handle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _capture_and_replay(fn, outs, replays=3):
    """Runs fn eagerly, captures it in a graph, then replays it with the
    outputs cleared (eagerly) before each replay; returns (eager, replays)."""
    fn()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()                                    # warm-up on a side stream, as torch asks
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    got = []
    for _ in range(replays):
        for o in outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got.append([o.clone() for o in outs])
    return eager, got


@pytest.mark.parametrize("case", ["fused_bf16", "fused_source_fp8", "layered_bf16"])
def test_step_graph_replays_equal_eager(case):
    cfg = {"fused_bf16": 2, "fused_source_fp8": 1, "layered_bf16": 6}[case]
    n = 4099 if cfg != 6 else 1031
    _note(f"case graph {case} n={n}")
    net = synth.make_net(cfg)
    S = net.widths[-1]
    thermo = synth.make_thermo(cfg, S)
    st = synth.make_state(cfg, n)
    T, P, Y = dev_state(st)
    Yo, To = torch.empty_like(Y), torch.empty_like(T)
    if case == "fused_source_fp8":
        cal = synth.make_state(cfg, 4096, stream="calibration")
        h32 = make_handle(net, "fp32", thermo=thermo)
        amax = h32.calibrate(*dev_state(cal)).cpu().numpy()
        W = synth.make_molar_masses(cfg, S)
        h = make_handle(net, "fp8", thermo=thermo, act_amax=amax, molar_mass=W)
        om = torch.empty_like(Y)
        outs = [Yo, To, om]
        fn = lambda: h.step_source(T, P, Y, 1e-6, Y_out=Yo, T_out=To, omega=om)
    else:
        h = make_handle(net, "bf16", thermo=thermo)
        outs = [Yo, To]
        fn = lambda: h.step(T, P, Y, Y_out=Yo, T_out=To)
    eager, got = _capture_and_replay(fn, outs)
    for r, rep in enumerate(got):
        for e, o in zip(eager, rep):
            assert torch.equal(e, o), (case, r)
    assert torch.isfinite(eager[0]).all()


@pytest.mark.parametrize("cfg", [7, 8])
def test_prop_graph_replays_equal_eager(cfg):
    from paper_2508_18969_amd import PropNet
    n = 40000
    _note(f"case graph prop cfg={cfg} n={n}")
    net = synth.make_prop_net(cfg)
    x = torch.tensor(synth.make_prop_inputs(cfg, n), device="cuda")
    y = torch.empty((net.widths[-1], n), dtype=torch.float64, device="cuda")
    h = PropNet(net.widths, "bf16", torch.tensor(net.flat_params(), device="cuda"), net.in_mean,
                net.in_std, net.out_mean, net.out_std)
    eager, got = _capture_and_replay(lambda: h.eval(x, y), [y])
    for r, rep in enumerate(got):
        assert torch.equal(eager[0], rep[0]), (cfg, r)
    assert torch.isfinite(eager[0]).all()


def test_handles_on_concurrent_streams():
    """Two handles (the fused chemistry step and the layer-by-layer property
    network) enqueued on two streams at once give the results they give one
    after the other (bit for bit): each handle's state is its own workspace."""
    from paper_2508_18969_amd import PropNet
    _note("case concurrent streams")
    net = synth.make_net(2)
    thermo = synth.make_thermo(2, 29)
    st = synth.make_state(2, 65536 + 3)
    h = make_handle(net, "bf16", thermo=thermo)
    T, P, Y = dev_state(st)
    pnet = synth.make_prop_net(8)
    x = torch.tensor(synth.make_prop_inputs(8, 70000), device="cuda")
    hp = PropNet(pnet.widths, "bf16", torch.tensor(pnet.flat_params(), device="cuda"), pnet.in_mean,
                 pnet.in_std, pnet.out_mean, pnet.out_std)
    Yo, To = torch.empty_like(Y), torch.empty_like(T)
    y = torch.empty((4, 70000), dtype=torch.float64, device="cuda")
    h.step(T, P, Y, Y_out=Yo, T_out=To)
    hp.eval(x, y)
    torch.cuda.synchronize()
    ref = [Yo.clone(), To.clone(), y.clone()]
    for o in (Yo, To, y):
        o.fill_(-1.0)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        with torch.cuda.stream(s1):
            h.step(T, P, Y, Y_out=Yo, T_out=To)
        with torch.cuda.stream(s2):
            hp.eval(x, y)
    torch.cuda.synchronize()
    assert torch.equal(Yo, ref[0]) and torch.equal(To, ref[1]) and torch.equal(y, ref[2])
