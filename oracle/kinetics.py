"""ctypes front end of the FP64 ROS2 reference integrator in ``kinetics.c``
(test infrastructure; see package doc)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kinetics.c")
LIB = os.path.join(HERE, "libkinetics.so")
R_GAS = 8.314462618


def build(verbose: bool = False) -> str:
    """Compile the integrator with gcc (-O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Mech(C.Structure):
    _fields_ = [("S", C.c_int), ("R", C.c_int),
                ("W", C.POINTER(C.c_double)), ("hf", C.POINTER(C.c_double)),
                ("cp", C.POINTER(C.c_double)), ("t_ref", C.c_double),
                ("nu_f", C.POINTER(C.c_int32)), ("nu_r", C.POINTER(C.c_int32)),
                ("A", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)),
                ("Ea", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.kin_rhs.argtypes = [C.POINTER(_Mech), C.c_double, dp, dp]
        L.kin_jac.argtypes = [C.POINTER(_Mech), C.c_double, dp, dp]
        L.kin_integrate.argtypes = [C.POINTER(_Mech), C.c_int64, C.c_int64, dp, dp, dp,
                                    C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                    dp, dp, C.POINTER(C.c_int32), C.c_int]
        L.kin_integrate.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Mech:
    """Holds contiguous copies of a mechanism's arrays and the C struct."""

    def __init__(self, mech):
        self.S, self.R = int(mech.nu_f.shape[1]), int(mech.nu_f.shape[0])
        self._keep = dict(
            W=np.ascontiguousarray(mech.W, np.float64),
            hf=np.ascontiguousarray(mech.hf, np.float64),
            cp=np.ascontiguousarray(mech.cp, np.float64),
            nu_f=np.ascontiguousarray(mech.nu_f, np.int32),
            nu_r=np.ascontiguousarray(mech.nu_r, np.int32),
            A=np.ascontiguousarray(mech.A, np.float64),
            b=np.ascontiguousarray(mech.b, np.float64),
            Ea=np.ascontiguousarray(mech.Ea, np.float64))
        k = self._keep
        self.c = _Mech(self.S, self.R, _dp(k["W"]), _dp(k["hf"]), _dp(k["cp"]), float(mech.t_ref),
                       k["nu_f"].ctypes.data_as(C.POINTER(C.c_int32)),
                       k["nu_r"].ctypes.data_as(C.POINTER(C.c_int32)),
                       _dp(k["A"]), _dp(k["b"]), _dp(k["Ea"]))


def rhs(mech: Mech, P: float, y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, np.float64)
    f = np.zeros_like(y)
    lib().kin_rhs(C.byref(mech.c), float(P), _dp(y), _dp(f))
    return f


def jac(mech: Mech, P: float, y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, np.float64)
    n = y.size
    J = np.zeros((n, n))
    lib().kin_jac(C.byref(mech.c), float(P), _dp(y), _dp(J))
    return J


def integrate(mech: Mech, T, P, Y, dt, rtol=1e-4, atol=1e-10, atol_T=1e-4,
              max_steps=200000, nthreads=0):
    """Advance n states (T[n], P[n], Y[S][n]) by dt.  Returns (T_out, Y_out, nsteps)."""
    T = np.ascontiguousarray(T, np.float64)
    P = np.ascontiguousarray(P, np.float64)
    Y = np.ascontiguousarray(Y, np.float64)
    n = T.size
    T_out = np.zeros_like(T)
    Y_out = np.zeros_like(Y)
    ns = np.zeros(n, np.int32)
    lib().kin_integrate(C.byref(mech.c), n, n, _dp(T), _dp(P), _dp(Y), float(dt), float(rtol),
                        float(atol), float(atol_T), int(max_steps), _dp(T_out), _dp(Y_out),
                        ns.ctypes.data_as(C.POINTER(C.c_int32)), int(nthreads))
    return T_out, Y_out, ns


def training_set(mech, state, dt, lam, rtol=1e-4, atol=1e-10, nthreads=0):
    """Labels for the chemistry net: normalised increments of BC(Y) over dt.

    Returns dict(x, t, in_mean, in_std, out_mean, out_std, T1, Y1, nsteps)
    where x = Z-scored [T, P, BC(Y)] and t = (BC(Y(t+dt)) - BC(Y(t)) - mu)/sigma
    with FP64 mean and population std over the set.
    """
    from .chem import boxcox
    M = mech if isinstance(mech, Mech) else Mech(mech)
    T1, Y1, ns = integrate(M, state.T, state.P, state.Y, dt, rtol, atol, nthreads=nthreads)
    ok = ns >= 0
    x = np.vstack([state.T[None], state.P[None], boxcox(state.Y, lam)])
    d = boxcox(Y1, lam) - boxcox(state.Y, lam)
    in_mean, in_std = x[:, ok].mean(axis=1), x[:, ok].std(axis=1)
    out_mean, out_std = d[:, ok].mean(axis=1), d[:, ok].std(axis=1)
    out_std = np.where(out_std > 0, out_std, 1.0)
    return dict(x=(x - in_mean[:, None]) / in_std[:, None],
                t=(d - out_mean[:, None]) / out_std[:, None],
                in_mean=in_mean, in_std=in_std, out_mean=out_mean, out_std=out_std,
                T1=T1, Y1=Y1, nsteps=ns, ok=ok)
