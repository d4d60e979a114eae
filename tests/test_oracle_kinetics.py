"""Pins of the FP64 stiff integrator: closed-form solutions of two-reaction
systems, element and enthalpy conservation, finite-difference Jacobian,
convergence under tolerance refinement, agreement with a library stiff
solver (scipy's Radau IIA)."""
import math

import numpy as np
import pytest

import synth
from oracle import kinetics as K

R = K.R_GAS


def _mech(comp, W, nu_f, nu_r, A, hf=None, cp=None, b=None, Ea=None):
    S = len(W)
    Rn = len(A)
    return synth.Mechanism(np.array(comp), np.array(W, float), np.array(nu_f), np.array(nu_r),
                           np.array(A, float), np.zeros(Rn) if b is None else np.array(b, float),
                           np.zeros(Rn) if Ea is None else np.array(Ea, float),
                           np.zeros(S) if hf is None else np.array(hf, float),
                           np.full(S, 1500.0) if cp is None else np.array(cp, float), 298.15)


@pytest.fixture(scope="module", autouse=True)
def _built():
    K.build()


def test_isomerisation_pair_exact_solution():
    # A -> B (k1), B -> A (k2); same molar mass, h_f and c_p: isothermal,
    # constant density, linear ODE with an exponential solution.
    k1, k2 = 3.0e5, 1.0e5
    m = K.Mech(_mech([[1, 2, 0, 0], [1, 2, 0, 0]], [0.014, 0.014], [[1, 0], [0, 1]],
                     [[0, 1], [1, 0]], [k1, k2]))
    ya0 = np.array([0.9, 0.2, 0.0])
    Y = np.vstack([ya0, 1 - ya0])
    T = np.full(3, 1200.0)
    P = np.full(3, 1e7)
    dt = 4e-6
    T1, Y1, ns = K.integrate(m, T, P, Y, dt, rtol=1e-8, atol=1e-12, atol_T=1e-8)
    yeq = k2 / (k1 + k2)
    exact = yeq + (ya0 - yeq) * math.exp(-(k1 + k2) * dt)
    assert (ns > 0).all()
    np.testing.assert_allclose(Y1[0], exact, rtol=1e-6)
    np.testing.assert_allclose(Y1.sum(axis=0), 1.0, atol=1e-14)
    np.testing.assert_allclose(T1, T, rtol=1e-14)


def test_arrhenius_temperature_dependence_by_hand():
    """k = A T^b exp(-Ea / (R T)) with b != 0 and Ea != 0, read off the exact
    relaxation of the isomerisation pair A <-> B at two temperatures.  The
    parameters make k computable by hand:
      A -> B: A1 = 1.2, b1 = 2, Ea1 = R (1000 K) ln 4
        T = 1000 K: T^2 = 1e6, exp(-ln 4) = 1/4      -> k1 = 3.0e5 /s
        T =  500 K: T^2 = 2.5e5, exp(-2 ln 4) = 1/16 -> k1 = 1.875e4 /s
      B -> A: A2 = 1e9, b2 = -1, Ea2 = R (1000 K) ln 10
        T = 1000 K: 1e-3 * 1/10                      -> k2 = 1.0e5 /s
        T =  500 K: 2e-3 * 1/100                     -> k2 = 2.0e4 /s
    A dropped or inverted temperature factor, a sign slip in the exponent or
    an activation energy taken in kJ would each move k by a large factor and
    the relaxation far off the exact curve."""
    T_ref = 1000.0
    Ea1, Ea2 = R * T_ref * math.log(4.0), R * T_ref * math.log(10.0)
    m = K.Mech(_mech([[1, 2, 0, 0], [1, 2, 0, 0]], [0.014, 0.014], [[1, 0], [0, 1]],
                     [[0, 1], [1, 0]], [1.2, 1.0e9], b=[2.0, -1.0], Ea=[Ea1, Ea2]))
    k_hand = {1000.0: (3.0e5, 1.0e5), 500.0: (1.875e4, 2.0e4)}
    ya0 = np.array([0.9, 0.1, 0.9, 0.1])
    T = np.array([1000.0, 1000.0, 500.0, 500.0])
    Y = np.vstack([ya0, 1 - ya0])
    dt = 4e-6
    T1, Y1, ns = K.integrate(m, T, np.full(4, 1e7), Y, dt, rtol=1e-9, atol=1e-14, atol_T=1e-9)
    assert (ns > 0).all()
    for c in range(4):
        k1, k2 = k_hand[T[c]]
        yeq = k2 / (k1 + k2)
        exact = yeq + (ya0[c] - yeq) * math.exp(-(k1 + k2) * dt)
        assert abs(Y1[0, c] - exact) <= 1e-7 * abs(ya0[c] - exact), (c, Y1[0, c], exact)
    np.testing.assert_allclose(T1, T, rtol=1e-14)


def test_label_tolerance_reading():
    """Training labels use rtol 1e-4, atol 1e-10 (the default).  Against a
    solution at rtol 1e-7 (16 states of the synthetic mechanism, dt = 1e-6 s)
    the Box-Cox label error stays small next to the spread of the labels: RMS
    below 1e-2 of the per-species label standard deviation (measured 9.5e-4
    on 256 states; at rtol 1e-6 the cost is 10x and at 1e-8 76x)."""
    from oracle.chem import boxcox
    mech = synth.make_mechanism(4)
    st = synth.make_state(4, 16)
    M = K.Mech(mech)
    _, Y4, n4 = K.integrate(M, st.T, st.P, st.Y, 1e-6)
    _, Y7, n7 = K.integrate(M, st.T, st.P, st.Y, 1e-6, rtol=1e-7, atol=1e-13, atol_T=1e-7,
                            max_steps=2000000)
    assert (n4 > 0).all() and (n7 > 0).all()
    lam = synth.BOXCOX_LAMBDA
    d4, d7 = boxcox(Y4, lam) - boxcox(st.Y, lam), boxcox(Y7, lam) - boxcox(st.Y, lam)
    sd = d7.std(axis=1)
    e = (d4 - d7) / sd[:, None]
    assert np.sqrt(np.mean(e ** 2)) < 1e-2
    assert np.abs(e).max() < 0.2


def test_dimerisation_equilibrium_closed_form():
    # A2 -> 2A (k1, first order), 2A -> A2 (k2, second order).  Equal h_f and
    # c_p per unit mass make it thermoneutral, so T stays fixed and the total
    # molar concentration of the equilibrium mixture is c = P/(R T).
    k1, k2 = 2.0e4, 50.0
    WA = 0.016
    m = K.Mech(_mech([[1, 0, 0, 0], [2, 0, 0, 0]], [WA, 2 * WA], [[0, 1], [2, 0]],
                     [[2, 0], [0, 1]], [k1, k2]))
    T0, P0 = 1500.0, 2.0e6
    c = P0 / (R * T0)
    A_eq = (-k1 + math.sqrt(k1 * k1 + 4 * k1 * k2 * c)) / (2 * k2)
    YA_eq = A_eq * WA / (A_eq * WA + (c - A_eq) * 2 * WA)
    Y = np.array([[0.05, 0.7], [0.95, 0.3]])
    T1, Y1, ns = K.integrate(m, np.full(2, T0), np.full(2, P0), Y, 5e-3, rtol=1e-8, atol=1e-12,
                             atol_T=1e-8)
    assert (ns > 0).all()
    np.testing.assert_allclose(Y1[0], YA_eq, rtol=1e-6)
    np.testing.assert_allclose(T1, T0, rtol=1e-14)


@pytest.fixture(scope="module")
def c4_run():
    mech = synth.make_mechanism(4)
    st = synth.make_state(4, 256)
    M = K.Mech(mech)
    T1, Y1, ns = K.integrate(M, st.T, st.P, st.Y, 1e-6)
    return mech, M, st, T1, Y1, ns


def test_generated_mechanism_is_element_balanced(c4_run):
    mech = c4_run[0]
    assert mech.S == 17 and mech.R == 40
    assert np.all(mech.comp.T @ (mech.nu_r - mech.nu_f).T == 0)
    assert set(np.nonzero(mech.nu_f.sum(0) + mech.nu_r.sum(0))[0]) == set(range(17))


def test_element_and_mass_conservation(c4_run):
    mech, _, st, T1, Y1, ns = c4_run
    assert (ns > 0).all()
    E = mech.comp.T / mech.W
    e0, e1 = E @ st.Y, E @ Y1
    assert np.max(np.abs(e1 - e0) / np.abs(e0)) < 1e-12
    np.testing.assert_allclose(Y1.sum(axis=0), 1.0, atol=1e-12)


def test_enthalpy_conservation(c4_run):
    mech, _, st, T1, Y1, _ = c4_run
    h = lambda T, Y: (Y * (mech.hf[:, None] + mech.cp[:, None] * (T - mech.t_ref))).sum(axis=0)
    cpbar = (Y1 * mech.cp[:, None]).sum(axis=0)
    # temperature implied by enthalpy conservation of the final composition
    t_cons = mech.t_ref + (h(st.T, st.Y) - (Y1 * mech.hf[:, None]).sum(axis=0)) / cpbar
    assert np.max(np.abs(t_cons - T1)) < 0.05          # K, at rtol 1e-4
    assert np.max(np.abs(T1 - st.T)) > 10.0            # the step does change T


def test_jacobian_matches_central_differences(c4_run):
    _, M, st, _, _, _ = c4_run
    for c in range(4):
        y = np.concatenate([st.Y[:, c], [st.T[c]]])
        J = K.jac(M, st.P[c], y)
        Jfd = np.zeros_like(J)
        for j in range(y.size):
            h = 1e-6 * max(1e-3, abs(y[j]))
            yp, ym = y.copy(), y.copy()
            yp[j] += h
            ym[j] -= h
            Jfd[:, j] = (K.rhs(M, st.P[c], yp) - K.rhs(M, st.P[c], ym)) / (2 * h)
        assert np.abs(J - Jfd).max() <= 1e-6 * np.abs(J).max()


def test_tolerance_refinement_converges(c4_run):
    mech, M, st, _, _, _ = c4_run
    sl = slice(0, 24)
    res = []
    for rtol in (1e-3, 1e-5, 1e-7):
        T1, Y1, ns = K.integrate(M, st.T[sl], st.P[sl], st.Y[:, sl], 1e-6, rtol=rtol,
                                 atol=rtol * 1e-6, atol_T=rtol)
        assert (ns > 0).all()
        res.append(Y1)
    e1 = np.abs(res[0] - res[2]).max()
    e2 = np.abs(res[1] - res[2]).max()
    assert e2 < 0.2 * e1


def test_matches_library_stiff_solver(c4_run):
    """The ROS2 step against scipy's Radau IIA (an independent implicit
    Runge-Kutta method of order 5) on the same right-hand side and Jacobian,
    both at tight tolerances, for states of the synthetic mechanism: the two
    time integrations agree to the tolerance."""
    from scipy.integrate import solve_ivp
    _, M, st, _, _, _ = c4_run
    sl = slice(0, 6)
    T1, Y1, ns = K.integrate(M, st.T[sl], st.P[sl], st.Y[:, sl], 1e-6, rtol=1e-7, atol=1e-13,
                             atol_T=1e-7)
    assert (ns > 0).all()
    for c in range(6):
        y0 = np.concatenate([st.Y[:, c], [st.T[c]]])
        P = st.P[c]
        sol = solve_ivp(lambda t, y: K.rhs(M, P, y), (0.0, 1e-6), y0, method="Radau",
                        jac=lambda t, y: K.jac(M, P, y), rtol=1e-11, atol=1e-16)
        assert sol.success
        yr = sol.y[:, -1]
        # (measured: at most 3e-8 of the largest change of Y and 4e-6 K)
        assert np.abs(Y1[:, c] - yr[:-1]).max() <= 1e-6 * np.abs(yr[:-1] - y0[:-1]).max()
        assert abs(T1[c] - yr[-1]) <= 1e-4
