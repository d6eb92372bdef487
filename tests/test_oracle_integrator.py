"""Pins of the oracle's adaptive Rosenbrock integrator against independent
solutions: a closed form, brute-force RK4, scipy's Radau, linear invariants,
and the documented failure modes."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import chemgen
import oracle


def test_isomer_closed_form():
    """A <=> B with identical thermo: Y_A(t) = s/2 + (Y_A0 - s/2) e^{-2kt},
    T and rho constant."""
    k = 1e5
    mech = chemgen.isomer_mechanism(k)
    om = oracle.OracleMech(mech)
    Y0 = np.array([[0.2, 0.03], [0.05, 0.17], [0.75, 0.8]])
    T0 = np.array([1500.0, 700.0])
    p = np.full(2, oracle.PREF)
    for dt in (1e-6, 1e-5, 4e-5):
        for rtol in (1e-6, 1e-10):
            out = oracle.chem_step(om, dt, T0, p, Y0, opts=dict(rtol=rtol, atol_Y=1e-16))
            assert np.all(out["stats"][2] == 0)
            s = Y0[0] + Y0[1]
            ya = s / 2 + (Y0[0] - s / 2) * np.exp(-2 * k * dt)
            np.testing.assert_allclose(out["Y"][0], ya, rtol=20 * rtol)
            np.testing.assert_allclose(out["Y"][1], s - ya, rtol=20 * rtol)
            np.testing.assert_array_equal(out["T"], T0)


def _lam_max(om, p, y):
    J = oracle.jacobian(om, p, y)
    return np.abs(np.linalg.eigvals(J)).max()


def test_rk4_brute_force():
    """Mild kinetics so that explicit RK4 is affordable: RK4 at h and h/2
    (Richardson) agrees with the adaptive RODAS3 result to tolerance level at
    default settings and to 1e-8 at rtol = 1e-11."""
    mech = chemgen.make_mechanism("h2_mild")
    om = oracle.OracleMech(mech)
    T, p, Y = chemgen.make_states(mech, "h2", N=16, seed=77)
    dt = 1e-7
    for i in range(16):
        y = np.concatenate([[T[i]], Y[:, i]])
        lam = _lam_max(om, p[i], y)
        nsteps = int(max(64, np.ceil(dt * lam / 0.5)))
        assert nsteps < 400000
        a = oracle.rk4(om, p[i], y, dt, nsteps)
        b = oracle.rk4(om, p[i], y, dt, 2 * nsteps)
        ref = b + (b - a) / 15.0
        for rtol, tol in ((1e-6, None), (1e-11, 1e-8)):
            yo, st, na, nr, _ = oracle.integrate(om, p[i], y, dt,
                                                 opts=dict(rtol=rtol, atol_Y=1e-18, atol_T=1e-12))
            assert st == 0
            if tol is None:
                sc = 1e-12 + rtol * np.abs(ref)
                assert np.all(np.abs(yo - ref) <= 10 * sc), (i, np.max(np.abs(yo - ref) / sc))
            else:
                big = np.abs(ref) > 1e-10
                np.testing.assert_allclose(yo[big], ref[big], rtol=tol)


@pytest.mark.slow
@pytest.mark.parametrize("which,dt,ncell", [("h2", 1e-6, 4), ("ch4", 1e-5, 3)])
def test_radau_reference(which, dt, ncell, om_h2, om_ch4):
    """scipy Radau IIA at rtol 1e-12 with the oracle's analytic Jacobian."""
    om = om_h2 if which == "h2" else om_ch4
    T, p, Y = chemgen.make_states(om.mech, which, N=64, seed=123)
    idx = np.argsort(T)[np.linspace(8, 63, ncell).astype(int)]
    for i in idx:
        y = np.concatenate([[T[i]], Y[:, i]])
        sol = solve_ivp(lambda t, yy: oracle.rhs(om, p[i], yy), (0.0, dt), y, method="Radau",
                        rtol=1e-12, atol=1e-20, jac=lambda t, yy: oracle.jacobian(om, p[i], yy))
        assert sol.success
        ref = sol.y[:, -1]
        yo, st, _, _, _ = oracle.integrate(om, p[i], y, dt)
        assert st == 0
        sc = 1e-12 + 1e-6 * np.abs(ref)
        assert np.all(np.abs(yo - ref) <= 20 * sc), (i, np.max(np.abs(yo - ref) / sc))
        yt, st, _, _, _ = oracle.integrate(om, p[i], y, dt, opts=dict(rtol=1e-11, atol_Y=1e-18))
        big = np.abs(ref) > 1e-8
        np.testing.assert_allclose(yt[big], ref[big], rtol=5e-8)


def test_linear_invariants(om_ch4):
    """Element mass fractions and sum(Y) are linear invariants of the ODE; a
    Rosenbrock method with the exact Jacobian keeps them to rounding."""
    m = om_ch4.mech
    T, p, Y = chemgen.make_states(m, "ch4", N=48, seed=31)
    out = oracle.chem_step(om_ch4, 1e-5, T, p, Y)
    assert np.all(out["stats"][2] == 0)
    Mel = m.comp.T * m.awt[:, None] / m.W[None, :]
    np.testing.assert_allclose(Mel @ out["Y"], Mel @ Y, atol=1e-12)
    np.testing.assert_allclose(out["Y"].sum(axis=0), 1.0, atol=1e-12)


def test_enthalpy_conserved(om_ch4):
    """Adiabatic constant pressure: the mixture enthalpy is conserved by the
    exact solution; the integrated result keeps it to tolerance level."""
    m = om_ch4.mech
    T, p, Y = chemgen.make_states(m, "ch4", N=24, seed=32)
    out = oracle.chem_step(om_ch4, 1e-5, T, p, Y)
    for i in range(T.size):
        h0 = oracle.mixture_enthalpy(om_ch4, T[i], Y[:, i])
        h1 = oracle.mixture_enthalpy(om_ch4, out["T"][i], out["Y"][:, i])
        cpR, _, _ = oracle.thermo(om_ch4, T[i])
        cp = np.sum(Y[:, i] * oracle.RGAS * cpR / m.W)
        assert abs(h1 - h0) / (cp * T[i]) <= 1e-5


def test_rates_output_and_dt_cell(om_h2):
    m = om_h2.mech
    T, p, Y = chemgen.make_states(m, "h2", N=32, seed=8)
    out = oracle.chem_step(om_h2, 1e-6, T, p, Y)
    rho0 = p / (oracle.RGAS * T * (Y / m.W[:, None]).sum(axis=0))
    np.testing.assert_allclose(out["RR"], rho0 * (out["Y"] - Y) / 1e-6, rtol=1e-12, atol=1e-14)
    dtc = np.where(np.arange(32) % 2 == 0, 1e-6, 3e-7)
    o2 = oracle.chem_step(om_h2, 5.0, T, p, Y, dt_cell=dtc)
    o3 = oracle.chem_step(om_h2, 3e-7, T, p, Y)
    np.testing.assert_array_equal(o2["Y"][:, 0::2], out["Y"][:, 0::2])
    np.testing.assert_array_equal(o2["Y"][:, 1::2], o3["Y"][:, 1::2])


def test_h_hint_round_trip(om_ch4):
    m = om_ch4.mech
    T, p, Y = chemgen.make_states(m, "ch4", N=32, seed=10)
    h = np.zeros(32)
    a = oracle.chem_step(om_ch4, 1e-5, T, p, Y, h_hint=h)
    assert np.all(a["h_hint"] > 0)
    b = oracle.chem_step(om_ch4, 1e-5, a["T"], p, a["Y"], h_hint=a["h_hint"])
    c = oracle.chem_step(om_ch4, 1e-5, a["T"], p, a["Y"])
    assert b["stats"][0].sum() < c["stats"][0].sum()


def test_failure_modes(om_ch4):
    """Failed cells keep their input state, get RR = 0 and a status code."""
    m = om_ch4.mech
    T, p, Y = chemgen.make_states(m, "ch4", N=8, seed=12)
    T = T.copy()
    Y = Y.copy()
    T[0] = np.nan
    T[1] = -5.0
    Y[3, 2] = np.inf
    out = oracle.chem_step(om_ch4, 1e-5, T, p, Y)
    st = out["stats"][2]
    assert st[0] == 3 and st[1] == 3 and st[2] == 3
    for i in (0, 1, 2):
        np.testing.assert_array_equal(out["Y"][:, i], Y[:, i])
        assert np.all(out["RR"][:, i] == 0)
        assert out["stats"][0, i] == 0
    o1 = oracle.chem_step(om_ch4, 1e-5, T[3:], p[3:], Y[:, 3:], opts=dict(max_steps=1))
    assert np.all(o1["stats"][2] == 1)
    np.testing.assert_array_equal(o1["Y"], Y[:, 3:])
    o2 = oracle.chem_step(om_ch4, 1e-5, T[3:], p[3:], Y[:, 3:], opts=dict(h_min=1.0))
    assert np.all(o2["stats"][2] == 2)
    np.testing.assert_array_equal(o2["T"], T[3:])


def test_zero_cells(om_h2):
    out = oracle.chem_step(om_h2, 1e-6, np.zeros(0), np.zeros(0), np.zeros((om_h2.K, 0)))
    assert out["Y"].shape == (om_h2.K, 0)
