"""ctypes binding of ``libchemdnn.so`` (declared in ``include/chem_dnn.h``).

Argument marshalling only: every step of the chemistry update and of the
training step runs in the library's HIP kernels.  PyTorch provides device
memory (CUDA tensors on ROCm) and the current stream.  Importing this module
does not need a GPU; creating a handle does, and fails loudly when the
library is missing or the device is not gfx950.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libchemdnn.so")

OK, EINVAL, ENODEV, EWORKSPACE, EUNSUPPORTED, EHIP, ETOOLARGE = 0, -1, -2, -3, -4, -5, -6
FP32, BF16, FP16, FP8E4M3 = 0, 1, 2, 3
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16, "fp8": FP8E4M3}
EXPORTS = ("chem_dnn_workspace_bytes", "chem_dnn_init", "chem_dnn_set_params", "chem_dnn_step",
           "chem_dnn_step_source", "chem_dnn_calibrate", "chem_dnn_get_scales", "chem_dnn_mlp_forward",
           "chem_dnn_mlp_backward", "chem_dnn_train_step", "chem_dnn_destroy",
           "chem_dnn_strerror", "chem_dnn_abi_version", "chem_prop_workspace_bytes",
           "chem_prop_init", "chem_prop_set_params", "chem_prop_eval", "chem_prop_destroy",
           "chem_dnn_debug_layers", "chem_dnn_train_step_noalloc")
DEBUG_MAX_CELLS = 4096

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)


class Desc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_layers", C.c_int32), ("widths", C.c_int32 * 9),
                ("precision", C.c_int32), ("gelu_form", C.c_int32), ("boxcox_lambda", C.c_double),
                ("in_mean", _dp), ("in_std", _dp), ("out_mean", _dp), ("out_std", _dp),
                ("act_amax", _fp), ("thermo_hf", _dp), ("thermo_cp", _dp), ("t_ref", C.c_double),
                ("max_batch", C.c_int64), ("molar_mass", _dp), ("recompute_chunk", C.c_int64)]


class PropDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("widths", C.c_int32 * 9), ("precision", C.c_int32),
                ("in_mean", _dp), ("in_std", _dp), ("out_mean", _dp), ("out_std", _dp)]


class ChemDNNError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with "
                               "`python -m paper_2508_18969_amd.build`")
        L = C.CDLL(LIB)
        vp = C.c_void_p
        i64 = C.c_int64
        L.chem_dnn_workspace_bytes.argtypes = [C.POINTER(Desc), C.POINTER(C.c_size_t)]
        L.chem_dnn_init.argtypes = [C.POINTER(Desc), vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.chem_dnn_set_params.argtypes = [vp, vp, vp]
        L.chem_dnn_step.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp]
        L.chem_dnn_step_source.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, C.c_double, vp, vp]
        L.chem_dnn_calibrate.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp]
        L.chem_dnn_get_scales.argtypes = [vp, _fp, _fp, vp]
        L.chem_dnn_mlp_forward.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp]
        L.chem_dnn_mlp_backward.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp]
        L.chem_dnn_train_step.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, i64,
                                          C.c_float, C.c_int32, vp, vp]
        L.chem_dnn_destroy.argtypes = [vp]
        L.chem_dnn_debug_layers.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp]
        L.chem_dnn_train_step_noalloc.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp,
                                                  i64, C.c_float, vp, vp]
        L.chem_prop_workspace_bytes.argtypes = [C.POINTER(PropDesc), C.POINTER(C.c_size_t)]
        L.chem_prop_init.argtypes = [C.POINTER(PropDesc), vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.chem_prop_set_params.argtypes = [vp, vp, vp]
        L.chem_prop_eval.argtypes = [vp, i64, i64, vp, vp, vp]
        L.chem_prop_destroy.argtypes = [vp]
        L.chem_dnn_strerror.argtypes = [C.c_int32]
        L.chem_dnn_strerror.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("chem_dnn_strerror",):
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def strerror(status: int) -> str:
    try:
        return lib().chem_dnn_strerror(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


def _check(status, what):
    if status != OK:
        raise ChemDNNError(status, what)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_field(t, name, rows, n, ld, dtype):
    """The C ABI takes field arrays as [rows][ld] with the cell index fastest
    (element (j, i) at j * ld + i).  Tensors of another layout (a transposed
    or Fortran-ordered copy, a column slice) are rejected here instead of
    being read with the wrong strides."""
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype:
        raise ValueError(f"{name}: expected a CUDA {dtype} tensor")
    if rows == 1 and t.dim() == 1:
        if t.shape[0] != n or (n > 1 and t.stride(0) != 1):
            raise ValueError(f"{name}: expected a contiguous [{n}] tensor")
        return
    if t.dim() != 2 or tuple(t.shape) != (rows, n):
        raise ValueError(f"{name}: expected shape ({rows}, {n}), got {tuple(t.shape)}")
    if n > 1 and t.stride(1) != 1:
        raise ValueError(f"{name}: the cell index must be the fastest (stride 1), got strides {t.stride()}")
    if rows > 1 and t.stride(0) != ld:
        raise ValueError(f"{name}: leading dimension {t.stride(0)}, expected {ld} (that of the state)")


def _check_counter(t, name="n_bad"):
    """The bad-cell counter: a CUDA 32-bit integer tensor with at least one
    element (the kernels add to its first element with a device atomic)."""
    import torch
    if t is None:
        return
    if (not isinstance(t, torch.Tensor) or not t.is_cuda
            or t.dtype not in (torch.int32, torch.uint32) or t.numel() < 1):
        raise ValueError(f"{name}: expected a CUDA int32 tensor with at least one element")


def _check_params(t, count, name="params"):
    """A flat FP32 parameter vector on the device, contiguous, `count` long."""
    import torch
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32
            or not t.is_contiguous() or t.numel() != count):
        raise ValueError(f"{name}: expected a contiguous CUDA float32 tensor of {count} elements")


def n_params(widths):
    return sum(int(widths[i]) * int(widths[i + 1]) + int(widths[i + 1])
               for i in range(len(widths) - 1))


def _check_saved(t, rows, B, ld):
    """Saved pre-activations of the training forward: CUDA float32 [rows][B]
    with the batch index fastest and leading dimension ld (that of x)."""
    if t is None:
        return
    _check_field(t, "saved", rows, B, ld, __import__("torch").float32)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _arr(a, ctype):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64 if ctype is C.c_double else np.float32)
    return a, a.ctypes.data_as(C.POINTER(ctype))


GELU_FORMS = {"tanh": 0, "table": 1, "table16": 2}


def make_desc(widths, precision, in_mean, in_std, out_mean=None, out_std=None, act_amax=None,
              thermo=None, max_batch=0, lam=0.1, gelu="tanh", molar_mass=None, recompute_chunk=0):
    """Fills a Desc; returns (desc, keepalive) - keep the second alive while the
    desc is in use."""
    d = Desc()
    widths = [int(w) for w in widths]
    d.n_species = widths[-1]
    d.n_layers = len(widths) - 1
    for i, w in enumerate(widths):
        d.widths[i] = w
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.gelu_form = GELU_FORMS[gelu] if isinstance(gelu, str) else int(gelu)
    d.boxcox_lambda = float(lam)
    keep = []
    for name, val, ct in (("in_mean", in_mean, C.c_double), ("in_std", in_std, C.c_double),
                          ("out_mean", out_mean, C.c_double), ("out_std", out_std, C.c_double),
                          ("act_amax", act_amax, C.c_float)):
        a, p = _arr(val, ct)
        keep.append(a)
        setattr(d, name, p)
    if thermo is not None:
        hf, cp, tref = thermo
        a, p = _arr(hf, C.c_double)
        b, q = _arr(cp, C.c_double)
        keep += [a, b]
        d.thermo_hf, d.thermo_cp, d.t_ref = p, q, float(tref)
    d.max_batch = int(max_batch)
    d.recompute_chunk = int(recompute_chunk)
    if molar_mass is not None:
        a, p = _arr(molar_mass, C.c_double)
        keep.append(a)
        d.molar_mass = p
    return d, keep


def workspace_bytes(desc) -> int:
    n = C.c_size_t(0)
    _check(lib().chem_dnn_workspace_bytes(C.byref(desc), C.byref(n)), "chem_dnn_workspace_bytes")
    return int(n.value)


class ChemDNN:
    """A chemistry-update handle on the current device.

    params: CUDA float32 tensor, flat [W1 (out x in), b1, ..., W4, b4].
    The workspace is a torch uint8 tensor owned by this object.
    """

    def __init__(self, widths, precision, params, in_mean, in_std, out_mean=None, out_std=None,
                 act_amax=None, thermo=None, max_batch=0, lam=0.1, gelu="tanh", molar_mass=None,
                 recompute_chunk=0):
        import torch
        self.widths = tuple(int(w) for w in widths)
        self.S = self.widths[-1]
        self.L = len(self.widths) - 1
        self.precision = precision
        self.thermo = thermo is not None
        desc, keep = make_desc(self.widths, precision, in_mean, in_std, out_mean, out_std,
                               act_amax, thermo, max_batch, lam, gelu, molar_mass, recompute_chunk)
        _check_params(params, n_params(self.widths))
        nbytes = workspace_bytes(desc)
        dev = params.device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self._ws_bytes = nbytes
        h = C.c_void_p()
        _check(lib().chem_dnn_init(C.byref(desc), _ptr(params), C.c_void_p(self._ws_ptr),
                                   C.c_size_t(nbytes), _stream(), C.byref(h)), "chem_dnn_init")
        self._h = h
        del keep

    # -- inference --------------------------------------------------------
    def step(self, T, P, Y, Y_out=None, T_out=None, n_bad=None):
        """Chemistry update of n cells (T, P: float64 [n]; Y: float64 [S][ld])."""
        import torch
        n = int(T.shape[0])
        ld = int(Y.stride(0)) if Y.dim() == 2 else n
        if Y_out is None:
            Y_out = torch.empty_like(Y)
        if T_out is None and self.thermo:
            T_out = torch.empty_like(T)
        f64 = torch.float64
        for t, nm, r in ((T, "T", 1), (P, "P", 1), (Y, "Y", self.S), (Y_out, "Y_out", self.S),
                         (T_out, "T_out", 1)):
            _check_field(t, nm, r, n, ld, f64)
        _check_counter(n_bad)
        _check(lib().chem_dnn_step(self._h, n, ld, _ptr(T), _ptr(P), _ptr(Y), _ptr(Y_out),
                                   _ptr(T_out), _ptr(n_bad), _stream()), "chem_dnn_step")
        return Y_out, T_out

    def step_source(self, T, P, Y, dt, Y_out=None, T_out=None, omega=None, n_bad=None):
        """chem_dnn_step plus the species source terms omega [S][ld] (float64,
        kg/(m^3 s)) of a step of dt seconds; needs molar_mass at construction."""
        import torch
        n = int(T.shape[0])
        ld = int(Y.stride(0)) if Y.dim() == 2 else n
        if Y_out is None:
            Y_out = torch.empty_like(Y)
        if T_out is None and self.thermo:
            T_out = torch.empty_like(T)
        if omega is None:
            omega = torch.empty_like(Y)
        f64 = torch.float64
        for t, nm, r in ((T, "T", 1), (P, "P", 1), (Y, "Y", self.S), (Y_out, "Y_out", self.S),
                         (T_out, "T_out", 1), (omega, "omega", self.S)):
            _check_field(t, nm, r, n, ld, f64)
        _check_counter(n_bad)
        _check(lib().chem_dnn_step_source(self._h, n, ld, _ptr(T), _ptr(P), _ptr(Y), _ptr(Y_out),
                                          _ptr(T_out), _ptr(omega), float(dt), _ptr(n_bad),
                                          _stream()), "chem_dnn_step_source")
        return Y_out, T_out, omega

    def calibrate(self, T, P, Y):
        """Per-layer input max |a| (CUDA float32 [L]) for an FP8 description."""
        import torch
        amax = torch.empty(self.L, dtype=torch.float32, device=T.device)
        n = int(T.shape[0])
        ld = int(Y.stride(0))
        for t, nm, r in ((T, "T", 1), (P, "P", 1), (Y, "Y", self.S)):
            _check_field(t, nm, r, n, ld, torch.float64)
        _check(lib().chem_dnn_calibrate(self._h, n, ld, _ptr(T), _ptr(P), _ptr(Y), _ptr(amax),
                                        _stream()), "chem_dnn_calibrate")
        return amax

    def debug_layers(self, T, P, Y):
        """Layer dump of chem_dnn_debug_layers for n <= DEBUG_MAX_CELLS cells:
        (qin, acc), lists over the layers of CUDA float32 tensors [widths[l]][n]
        (the input operand values of layer l as the matrix cores received
        them) and [widths[l+1]][n] (its FP32 accumulators before the
        activation)."""
        import torch
        n = int(T.shape[0])
        ld = int(Y.stride(0)) if Y.dim() == 2 and self.S > 1 else n
        for t, nm, r in ((T, "T", 1), (P, "P", 1), (Y, "Y", self.S)):
            _check_field(t, nm, r, n, ld, torch.float64)
        if n > DEBUG_MAX_CELLS:
            raise ValueError(f"debug_layers: at most {DEBUG_MAX_CELLS} cells")
        w = self.widths
        qin = torch.full((sum(w[:-1]), n), float("nan"), dtype=torch.float32, device=T.device)
        acc = torch.full((sum(w[1:]), n), float("nan"), dtype=torch.float32, device=T.device)
        _check(lib().chem_dnn_debug_layers(self._h, n, ld, _ptr(T), _ptr(P), _ptr(Y), _ptr(qin),
                                           _ptr(acc), _stream()), "chem_dnn_debug_layers")
        qs, accs, ri, ra = [], [], 0, 0
        for l in range(self.L):
            qs.append(qin[ri:ri + w[l]])
            accs.append(acc[ra:ra + w[l + 1]])
            ri += w[l]
            ra += w[l + 1]
        return qs, accs

    def scales(self):
        a = (C.c_float * self.L)()
        w = (C.c_float * self.L)()
        _check(lib().chem_dnn_get_scales(self._h, a, w, _stream()), "chem_dnn_get_scales")
        return np.array(a[:]), np.array(w[:])

    def set_params(self, params):
        _check_params(params, n_params(self.widths))
        _check(lib().chem_dnn_set_params(self._h, _ptr(params), _stream()), "chem_dnn_set_params")

    # -- training ---------------------------------------------------------
    def mlp_forward(self, x, params, saved=None):
        import torch
        B = int(x.shape[1])
        ld = int(x.stride(0))
        _check_field(x, "x", self.widths[0], B, ld, torch.float32)
        _check_saved(saved, hidden_total(self.widths), B, ld)
        _check_params(params, n_params(self.widths))
        out = torch.empty((self.S, B), dtype=torch.float32, device=x.device)
        if out.stride(0) != ld:
            out = torch.empty((self.S, ld), dtype=torch.float32, device=x.device)[:, :B]
        _check(lib().chem_dnn_mlp_forward(self._h, B, ld, _ptr(x), _ptr(params), _ptr(out),
                                          _ptr(saved), _stream()), "chem_dnn_mlp_forward")
        return out

    def mlp_backward(self, x, params, saved, grad_out, want_grad_x=False):
        import torch
        B = int(x.shape[1])
        ld = int(x.stride(0))
        _check_field(x, "x", self.widths[0], B, ld, torch.float32)
        _check_field(grad_out, "grad_out", self.S, B, ld, torch.float32)
        _check_saved(saved, hidden_total(self.widths), B, ld)
        _check_params(params, n_params(self.widths))
        gp = torch.empty_like(params)
        gx = torch.empty((x.shape[0], ld), dtype=torch.float32, device=x.device)[:, :B] \
            if want_grad_x else None
        _check(lib().chem_dnn_mlp_backward(self._h, B, ld, _ptr(x), _ptr(params), _ptr(saved),
                                           _ptr(grad_out), _ptr(gp), _ptr(gx), _stream()),
               "chem_dnn_mlp_backward")
        return gp, gx

    def train_step(self, T, P, Y, target, params, grads, adam_m, adam_v, step, lr=1e-3,
                   recompute=False, loss=None):
        import torch
        B = int(T.shape[0])
        ld = int(Y.stride(0))
        for t, nm, r in ((T, "T", 1), (P, "P", 1), (Y, "Y", self.S)):
            _check_field(t, nm, r, B, ld, torch.float64)
        _check_field(target, "target", self.S, B, ld, torch.float32)
        np_ = n_params(self.widths)
        for t, nm in ((params, "params"), (grads, "grads"), (adam_m, "adam_m"), (adam_v, "adam_v")):
            _check_params(t, np_, nm)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=T.device)
        elif (not isinstance(loss, torch.Tensor) or not loss.is_cuda or loss.dtype != torch.float32
              or loss.numel() < 1):
            raise ValueError("loss: expected a CUDA float32 tensor with at least one element")
        _check(lib().chem_dnn_train_step(self._h, B, ld, _ptr(T), _ptr(P), _ptr(Y), _ptr(target),
                                         _ptr(params), _ptr(grads), _ptr(adam_m), _ptr(adam_v),
                                         int(step), float(lr), int(bool(recompute)), _ptr(loss),
                                         _stream()), "chem_dnn_train_step")
        return loss

    def train_step_noalloc(self, T, P, Y, target, params, grads, adam_m, adam_v, step, lr=1e-3,
                           loss=None):
        """chem_dnn_train_step_noalloc: the training step with its scratch in
        the library's static device array (no workspace scratch needed)."""
        import torch
        B = int(T.shape[0])
        ld = int(Y.stride(0))
        for t, nm, r in ((T, "T", 1), (P, "P", 1), (Y, "Y", self.S)):
            _check_field(t, nm, r, B, ld, torch.float64)
        _check_field(target, "target", self.S, B, ld, torch.float32)
        np_ = n_params(self.widths)
        for t, nm in ((params, "params"), (grads, "grads"), (adam_m, "adam_m"), (adam_v, "adam_v")):
            _check_params(t, np_, nm)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=T.device)
        _check(lib().chem_dnn_train_step_noalloc(self._h, B, ld, _ptr(T), _ptr(P), _ptr(Y),
                                                 _ptr(target), _ptr(params), _ptr(grads),
                                                 _ptr(adam_m), _ptr(adam_v), int(step), float(lr),
                                                 _ptr(loss), _stream()),
               "chem_dnn_train_step_noalloc")
        return loss

    def close(self):
        if getattr(self, "_h", None):
            lib().chem_dnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_prop_desc(widths, precision, in_mean, in_std, out_mean=None, out_std=None):
    """Fills a PropDesc; returns (desc, keepalive)."""
    d = PropDesc()
    widths = [int(w) for w in widths]
    d.n_layers = len(widths) - 1
    for i, w in enumerate(widths):
        d.widths[i] = w
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    keep = []
    for name, val in (("in_mean", in_mean), ("in_std", in_std), ("out_mean", out_mean),
                      ("out_std", out_std)):
        a, ptr = _arr(val, C.c_double)
        keep.append(a)
        setattr(d, name, ptr)
    return d, keep


def prop_workspace_bytes(desc) -> int:
    n = C.c_size_t(0)
    _check(lib().chem_prop_workspace_bytes(C.byref(desc), C.byref(n)), "chem_prop_workspace_bytes")
    return int(n.value)


class PropNet:
    """A property-network handle (chem_prop_*) on the current device: inputs
    x [n_in][ld] -> outputs y [n_out][ld], both float64.

    params: CUDA float32 tensor, flat [W1 (out x in), b1, ..., WL, bL].
    """

    def __init__(self, widths, precision, params, in_mean, in_std, out_mean=None, out_std=None):
        import torch
        self.widths = tuple(int(w) for w in widths)
        self.n_in, self.n_out = self.widths[0], self.widths[-1]
        self.precision = precision
        desc, keep = make_prop_desc(self.widths, precision, in_mean, in_std, out_mean, out_std)
        _check_params(params, n_params(self.widths))
        nbytes = prop_workspace_bytes(desc)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=params.device)
        base = self.workspace.data_ptr()
        ws = base + (-base) % 256
        h = C.c_void_p()
        _check(lib().chem_prop_init(C.byref(desc), _ptr(params), C.c_void_p(ws), C.c_size_t(nbytes),
                                    _stream(), C.byref(h)), "chem_prop_init")
        self._h = h
        del keep

    def eval(self, x, y=None):
        """Outputs of n cells for inputs x (float64 [n_in][ld])."""
        import torch
        n = int(x.shape[1])
        # the common leading dimension (a one-row field does not fix it)
        if self.n_in > 1:
            ld = int(x.stride(0))
        elif y is not None and self.n_out > 1:
            ld = int(y.stride(0))
        else:
            ld = n
        if y is None:
            y = torch.empty((self.n_out, ld), dtype=torch.float64, device=x.device)[:, :n]
        _check_field(x, "x", self.n_in, n, ld, torch.float64)
        _check_field(y, "y", self.n_out, n, ld, torch.float64)
        _check(lib().chem_prop_eval(self._h, n, ld, _ptr(x), _ptr(y), _stream()), "chem_prop_eval")
        return y

    def set_params(self, params):
        _check_params(params, n_params(self.widths))
        _check(lib().chem_prop_set_params(self._h, _ptr(params), _stream()), "chem_prop_set_params")

    def close(self):
        if getattr(self, "_h", None):
            lib().chem_prop_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hidden_total(widths):
    return sum(widths[1:-1])


def autograd_function():
    """torch.autograd.Function whose forward and backward are the library's
    MLP kernels.  Torch only sequences the calls."""
    import torch

    class ChemMLPFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, params, handle, recompute=False):
            B = x.shape[1]
            # x's leading dimension: the library indexes every [rows][B]
            # operand of one call with it
            ld = int(x.stride(0)) if x.shape[0] > 1 else B
            saved = None
            if not recompute:
                saved = torch.empty((hidden_total(handle.widths), ld), dtype=torch.float32,
                                    device=x.device)[:, :B]
            out = handle.mlp_forward(x, params, saved)
            ctx.handle = handle
            if recompute:
                ctx.save_for_backward(x, params)
            else:
                ctx.save_for_backward(x, params, saved)
            return out

        @staticmethod
        def backward(ctx, grad_out):
            tensors = ctx.saved_tensors
            x, params = tensors[0], tensors[1]
            saved = tensors[2] if len(tensors) > 2 else None
            B = x.shape[1]
            ld = int(x.stride(0)) if x.shape[0] > 1 else B
            go = grad_out
            if go.dim() != 2 or go.stride(1) != 1 or (go.shape[0] > 1 and go.stride(0) != ld):
                go = torch.empty((grad_out.shape[0], ld), dtype=torch.float32,
                                 device=grad_out.device)[:, :B]
                go.copy_(grad_out)
            gp, gx = ctx.handle.mlp_backward(x, params, saved, go, want_grad_x=ctx.needs_input_grad[0])
            return gx, gp, None, None

    return ChemMLPFunction
