"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chem_dnn.h")


@pytest.fixture(scope="module")
def L():
    from paper_2508_18969_amd import binding
    if not os.path.exists(binding.LIB):
        pytest.skip("library not built")
    return binding


def test_header_declares_what_the_library_exports(L):
    decl = set(re.findall(r"\b(chem_(?:dnn|prop)_[a-z_]+)\s*\(", open(HEADER).read()))
    assert decl == set(L.EXPORTS)
    assert {"chem_prop_init", "chem_prop_eval"} <= decl
    lib = L.lib()
    for name in decl:
        assert hasattr(lib, name), name
    assert lib.chem_dnn_abi_version() == 5
    for st in (0, -1, -2, -3, -4, -5):
        assert L.strerror(st) and L.strerror(st) != "unknown status"


def _desc(L, **kw):
    net = synth.make_net(1)
    args = dict(widths=net.widths, precision="fp32", in_mean=net.in_mean, in_std=net.in_std)
    args.update(kw)
    return L.make_desc(**args)


def test_workspace_bytes_and_validation(L):
    d, keep = _desc(L)
    n = L.workspace_bytes(d)
    assert n > 4 * 110017          # at least the packed FP32 weights
    d2, k2 = _desc(L, max_batch=65536)
    assert L.workspace_bytes(d2) > n + 65536 * 700 * 4
    # activation recomputation: the training scratch holds one chunk, so the
    # workspace drops by at least the pre-activations of the other samples
    d3, k3 = _desc(L, max_batch=65536, recompute_chunk=4096)
    assert L.workspace_bytes(d2) - L.workspace_bytes(d3) >= (65536 - 4096) * 700 * 4
    d4, k4 = _desc(L, max_batch=1 << 20, recompute_chunk=4096)
    assert L.workspace_bytes(d4) < L.workspace_bytes(d2)        # 16x the batch, less memory
    for bad_chunk in (-16, 100):                                 # negative, not a multiple of 16
        d5, k5 = _desc(L, max_batch=65536, recompute_chunk=bad_chunk)
        with pytest.raises(L.ChemDNNError):
            L.workspace_bytes(d5)
    bad = [dict(widths=(19, 400, 200, 100, 16)),           # S mismatch
           dict(widths=(19, 400, 200, 17)),                # 3 layers: unsupported
           dict(widths=(19, 0, 200, 100, 17)),
           dict(precision=7),
           dict(in_std=np.zeros(19)),
           dict(precision="fp8"),                          # FP8 needs act_amax
           dict(gelu=3),                                   # no such activation form
           dict(molar_mass=-np.ones(17))]                  # molar masses must be positive
    for kw in bad:
        d3, k3 = _desc(L, **kw)
        with pytest.raises(L.ChemDNNError) as e:
            L.workspace_bytes(d3)
        assert e.value.status in (L.EINVAL, L.EUNSUPPORTED)
    d4, k4 = _desc(L, widths=(19, 64, 64, 64, 17))          # valid but not compiled
    with pytest.raises(L.ChemDNNError) as e:
        L.workspace_bytes(d4)
    assert e.value.status == L.EUNSUPPORTED


def test_entry_points_reject_null_handles(L):
    lib = L.lib()
    assert lib.chem_dnn_step(None, 10, 10, None, None, None, None, None, None, None) == L.EINVAL
    assert lib.chem_dnn_step_source(None, 10, 10, None, None, None, None, None, None, 1e-6, None,
                                    None) == L.EINVAL
    assert lib.chem_dnn_destroy(None) == L.EINVAL
    assert lib.chem_dnn_set_params(None, None, None) == L.EINVAL
    assert lib.chem_dnn_train_step(None, 1, 1, None, None, None, None, None, None, None, None, 1,
                                   C.c_float(1e-3), 0, None, None) == L.EINVAL
    d, keep = _desc(L)
    out = C.c_void_p()
    # no workspace: caught before any device call
    assert lib.chem_dnn_init(C.byref(d), C.c_void_p(1), None, 0, None, C.byref(out)) == L.EWORKSPACE
    assert lib.chem_dnn_workspace_bytes(C.byref(d), None) == L.EINVAL


def test_init_without_device_reports_enodev(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    d, keep = _desc(L)
    n = L.workspace_bytes(d)
    buf = (C.c_uint8 * (n + 256))()
    addr = (C.addressof(buf) + 255) // 256 * 256
    out = C.c_void_p()
    st = L.lib().chem_dnn_init(C.byref(d), C.c_void_p(16), C.c_void_p(addr), n, None, C.byref(out))
    assert st == L.ENODEV and not out.value


def test_layered_shapes_workspace_and_limits(L):
    """Networks outside the fused shapes run layer by layer when their hidden
    widths are multiples of 256 (FP32/BF16/FP16, tanh GELU, no training): the
    workspace then also holds two chunk-sized activation buffers."""
    net = synth.make_net(6)
    assert net.widths == (19, 2048, 4096, 2048, 1024, 512, 17)
    d, keep = L.make_desc(net.widths, "bf16", net.in_mean, net.in_std)
    n = L.workspace_bytes(d)
    weights = 2 * sum(a * b for a, b in zip((32,) + net.widths[1:-1], net.widths[1:-1] + (32,)))
    assert n >= weights + 2 * 4096 * 32768 * 2 + 32 * 32768 * 4
    d32, k32 = L.make_desc(net.widths, "fp32", net.in_mean, net.in_std)
    assert L.workspace_bytes(d32) > n
    for kw in (dict(precision="fp8", act_amax=np.ones(6, np.float32)),   # no FP8 there
               dict(max_batch=1024),                                     # no training there
               dict(gelu="table"),                                       # tanh form only
               dict(widths=(19, 2048, 4000, 2048, 1024, 512, 17))):      # not a multiple of 256
        args = dict(widths=net.widths, precision="bf16", in_mean=net.in_mean, in_std=net.in_std)
        args.update(kw)
        d2, k2 = L.make_desc(**args)
        with pytest.raises(L.ChemDNNError) as e:
            L.workspace_bytes(d2)
        assert e.value.status == L.EUNSUPPORTED, kw


def test_property_networks_workspace_and_validation(L):
    """The property networks: the density net 3-1024-512-256-1 runs in the
    fused kernel (workspace: packed weights and constants only), the transport
    net 3-2048-1024-512-4 and a five-layer variant of the density net layer by
    layer (also two chunk-sized activation buffers and the FP32 output
    buffer); bad descriptions are EINVAL, shapes and formats the library lacks
    EUNSUPPORTED; null handles are rejected."""
    lib = L.lib()
    for widths, chunk_bf16 in (((3, 2048, 1024, 512, 4), 65536), ((3, 1024, 512, 256, 256, 1), 131072),
                               ((3, 1024, 512, 256, 1), 0)):
        net = synth.make_prop_net(7, widths=widths)
        d, keep = L.make_prop_desc(net.widths, "bf16", net.in_mean, net.in_std, net.out_mean, net.out_std)
        n = L.prop_workspace_bytes(d)
        hmax = max(net.widths[1:-1])
        weights = 2 * sum(a * b for a, b in zip((32,) + net.widths[1:-1], net.widths[1:-1] + (32,)))
        assert n >= weights + 2 * hmax * chunk_bf16 * 2 + 32 * chunk_bf16 * 4
        if chunk_bf16:
            assert n < weights + 2 * hmax * 2 * chunk_bf16 * 2 + 32 * 2 * chunk_bf16 * 4   # not larger
        else:
            assert n < weights + (1 << 20)                          # fused: no activation buffers
        d32, k32 = L.make_prop_desc(net.widths, "fp32", net.in_mean, net.in_std)
        assert L.prop_workspace_bytes(d32) >= 2 * weights + (2 * hmax * 32768 * 4 if chunk_bf16 else 0)
    net = synth.make_prop_net(7)
    base = dict(widths=net.widths, precision="bf16", in_mean=net.in_mean, in_std=net.in_std)
    for kw, want in ((dict(widths=(3, 1)), L.EINVAL),                       # no hidden layer
                     (dict(widths=(0, 1024, 1)), L.EINVAL),
                     (dict(widths=(33, 1024, 1)), L.EINVAL),                # > 32 inputs
                     (dict(widths=(3, 1024, 33)), L.EINVAL),                # > 32 outputs
                     (dict(in_std=np.array([1.0, 0.0, 1.0])), L.EINVAL),
                     (dict(out_mean=np.array([np.nan])), L.EINVAL),
                     (dict(precision=9), L.EINVAL),
                     (dict(precision="fp8"), L.EUNSUPPORTED),
                     (dict(widths=(3, 1000, 512, 256, 1)), L.EUNSUPPORTED)):  # not a multiple of 256
        args = dict(base)
        args.update(kw)
        d2, k2 = L.make_prop_desc(**args)
        with pytest.raises(L.ChemDNNError) as e:
            L.prop_workspace_bytes(d2)
        assert e.value.status == want, kw
    assert lib.chem_prop_eval(None, 10, 10, None, None, None) == L.EINVAL
    assert lib.chem_prop_set_params(None, None, None) == L.EINVAL
    assert lib.chem_prop_destroy(None) == L.EINVAL
    d, keep = L.make_prop_desc(**base)
    out = C.c_void_p()
    assert lib.chem_prop_init(C.byref(d), C.c_void_p(1), None, 0, None, C.byref(out)) == L.EWORKSPACE
    assert lib.chem_prop_workspace_bytes(C.byref(d), None) == L.EINVAL
    import torch
    if not torch.cuda.is_available():
        # a valid description and workspace: the missing device is reported
        n = L.prop_workspace_bytes(d)
        buf = (C.c_uint8 * (n + 256))()
        addr = (C.addressof(buf) + 255) // 256 * 256
        st = lib.chem_prop_init(C.byref(d), C.c_void_p(16), C.c_void_p(addr), n, None, C.byref(out))
        assert st == L.ENODEV and not out.value
