"""Pins of the oracle's thermo and kinetics against facts fixed by the
definitions (NASA-7 integral relations, element balance, equilibrium)."""
import numpy as np
import pytest

import chemgen
import oracle
from oracle import RGAS, PREF

pytestmark = pytest.mark.parametrize("which", ["h2", "ch4"])


def _om(which, om_h2, om_ch4):
    return om_h2 if which == "h2" else om_ch4


def _states(which, om, N=64, seed=5):
    cfg = "h2" if which == "h2" else "ch4"
    T, p, Y = chemgen.make_states(om.mech, cfg, N=N, seed=seed)
    return T, p, Y


def test_nasa_derivatives(which, om_h2, om_ch4):
    """dH/dT = c_p and dS/dT = c_p/T (Richardson-extrapolated central
    differences of the oracle's own h and s), away from the range switch."""
    om = _om(which, om_h2, om_ch4)
    for T in (450.0, 780.0, 1400.0, 2300.0, 3100.0):
        cp, _, _ = oracle.thermo(om, T)

        def H(t):
            return oracle.thermo(om, t)[1] * t

        def S(t):
            return oracle.thermo(om, t)[2]

        def d(fn, d1):
            a = (fn(T + d1) - fn(T - d1)) / (2 * d1)
            b = (fn(T + d1 / 2) - fn(T - d1 / 2)) / d1
            return (4 * b - a) / 3

        np.testing.assert_allclose(d(H, 2.0), cp, rtol=1e-9)
        np.testing.assert_allclose(d(S, 2.0), cp / T, rtol=1e-9)


def test_nasa_reference_values_and_continuity(which, om_h2, om_ch4):
    """h(298.15) and s(298.15) reproduce the generator's inputs; c_p, h, s are
    continuous at T_mid; c_p/R follows the generator's curve to ~1%."""
    om = _om(which, om_h2, om_ch4)
    m = om.mech
    cp, hRT, sR = oracle.thermo(om, 298.15)
    np.testing.assert_allclose(hRT * RGAS * 298.15, m.hf298, atol=1e-6)
    np.testing.assert_allclose(sR * RGAS, m.s298, rtol=1e-12)
    lo = oracle.thermo(om, 1000.0)
    hi = oracle.thermo(om, np.nextafter(1000.0, 2000.0))
    for a, b in zip(lo, hi):
        np.testing.assert_allclose(a, b, rtol=1e-11)
    assert np.all(cp > 2.0)
    cp3000, _, _ = oracle.thermo(om, 3000.0)
    assert np.all(cp3000 >= cp - 0.3)


def test_nasa_per_species_tmid(which, om_h2, om_ch4):
    """With per-species T_mid (the generator's tmid_range option) every
    species' c_p, h and s are continuous at its own T_mid, the reference
    values at 298.15 K still hold, and the kinetics are those of the default
    mechanism."""
    base = _om(which, om_h2, om_ch4).mech
    cfg = dict(chemgen.MECH_CONFIGS[which], tmid_range=(700.0, 1400.0), name=which + "_tmid")
    m = chemgen.make_mechanism(cfg)
    om = oracle.OracleMech(m)
    tm = m.nasa[:, 1]
    assert np.all((tm >= 700.0) & (tm <= 1400.0)) and np.unique(tm).size == m.K
    np.testing.assert_array_equal(m.A, base.A)
    np.testing.assert_array_equal(m.rsp, base.rsp)
    cp, hRT, sR = oracle.thermo(om, 298.15)
    np.testing.assert_allclose(hRT * RGAS * 298.15, m.hf298, atol=1e-6)
    np.testing.assert_allclose(sR * RGAS, m.s298, rtol=1e-12)
    for k in range(m.K):
        lo = oracle.thermo(om, tm[k])
        hi = oracle.thermo(om, np.nextafter(tm[k], 4000.0))
        for a, b in zip(lo, hi):
            np.testing.assert_allclose(a[k], b[k], rtol=1e-11)


def test_element_conservation_of_wdot(which, om_h2, om_ch4):
    """Every reaction conserves atoms, so sum_k a_ek wdot_k = 0 (P1) and, with
    W_k = sum_e a_ek A_e, sum_k W_k wdot_k = 0 i.e. sum_k dY_k/dt = 0 (P2)."""
    om = _om(which, om_h2, om_ch4)
    m = om.mech
    T, p, Y = _states(which, om)
    for i in range(T.size):
        y = np.concatenate([[T[i]], Y[:, i]])
        ev = oracle.evaluate(om, p[i], y)
        # magnitude of the largest one-way rate, the scale of rounding in wdot
        S = np.sum(Y[:, i] / m.W)
        Cc = p[i] / (RGAS * T[i] * S) * Y[:, i] / m.W
        scale = 0.0
        for r in range(m.R):
            f1 = ev["kf"][r] * np.prod([Cc[m.rsp[r, s]] ** m.rnu[r, s] for s in (0, 1)
                                        if m.rsp[r, s] >= 0])
            r1 = ev["kr"][r] * np.prod([Cc[m.rsp[r, s]] ** m.rnu[r, s] for s in (2, 3)
                                        if m.rsp[r, s] >= 0])
            scale = max(scale, f1, r1)
        el = m.comp.T.astype(float) @ ev["wdot"]
        assert np.all(np.abs(el) <= 1e-13 * scale * m.R * 4)
        assert abs(np.sum(m.W * ev["wdot"])) <= 1e-13 * scale * m.R * 4 * m.W.max()
        # a dropped or mis-signed term would leave O(scale) behind
        assert np.abs(ev["wdot"]).max() > 0


def test_arrhenius_direct(which, om_h2, om_ch4):
    """k_f equals A T^b exp(-Ea/RT) computed directly (not in log space)."""
    om = _om(which, om_h2, om_ch4)
    m = om.mech
    for T in (300.0, 1234.5, 2500.0):
        y = np.concatenate([[T], np.full(m.K, 1.0 / m.K)])
        ev = oracle.evaluate(om, PREF, y)
        kf = m.A * T ** m.b * np.exp(-m.Ea / (RGAS * T))
        np.testing.assert_allclose(ev["kf"], kf, rtol=1e-12)


def test_energy_equation_sign(which, om_h2, om_ch4):
    """c_p dT/dt = -sum_k h_k dY_k/dt per unit mass, with c_p and h_k taken
    from finite differences / values of the oracle's mixture enthalpy (an
    independent route to c_p)."""
    om = _om(which, om_h2, om_ch4)
    m = om.mech
    T, p, Y = _states(which, om, N=8)
    for i in range(T.size):
        if abs(T[i] - 1000.0) < 5:
            continue
        y = np.concatenate([[T[i]], Y[:, i]])
        f = oracle.rhs(om, p[i], y)
        d = 1e-3 * T[i]
        cp = (oracle.mixture_enthalpy(om, T[i] + d, Y[:, i]) -
              oracle.mixture_enthalpy(om, T[i] - d, Y[:, i])) / (2 * d)
        # dh/dt at fixed T along dY/dt: linear in Y, so exact with a unit step
        dh = oracle.mixture_enthalpy(om, T[i], Y[:, i] + f[1:]) - oracle.mixture_enthalpy(
            om, T[i], Y[:, i])
        np.testing.assert_allclose(cp * f[0], -dh, rtol=1e-6, atol=1e-9 * abs(dh) + 1e-12)


def test_mass_action_pressure_scaling(which, om_h2, om_ch4):
    """At fixed T and Y all concentrations scale with p, so for each reaction
    the forward term scales with p^(forward order) and the reverse with
    p^(reverse order); checked through k_f, k_r (which do not depend on p) and
    the one-reaction isolation of wdot via a single-reaction sub-mechanism."""
    om = _om(which, om_h2, om_ch4)
    m = om.mech
    T, p, Y = _states(which, om, N=2)
    for r in range(0, m.R, max(1, m.R // 7)):
        sub = chemgen.Mech(**{**m.__dict__, "rsp": m.rsp[r:r + 1].copy(),
                              "rnu": m.rnu[r:r + 1].copy(), "A": m.A[r:r + 1].copy(),
                              "b": m.b[r:r + 1].copy(), "Ea": m.Ea[r:r + 1].copy()})
        os_ = oracle.OracleMech(sub)
        y = np.concatenate([[T[1]], Y[:, 1]])
        e1 = oracle.evaluate(os_, PREF, y)
        e2 = oracle.evaluate(os_, 2 * PREF, y)
        S = np.sum(Y[:, 1] / m.W)
        Cc = PREF / (RGAS * T[1] * S) * Y[:, 1] / m.W
        fwd = e1["kf"][0] * np.prod([Cc[m.rsp[r, s]] ** m.rnu[r, s] for s in (0, 1)
                                     if m.rsp[r, s] >= 0])
        rev = e1["kr"][0] * np.prod([Cc[m.rsp[r, s]] ** m.rnu[r, s] for s in (2, 3)
                                     if m.rsp[r, s] >= 0])
        of = m.rnu[r, 0] + m.rnu[r, 1]
        orv = m.rnu[r, 2] + m.rnu[r, 3]
        k0 = m.rsp[r, 0]
        nu0 = -m.rnu[r, 0]
        np.testing.assert_allclose(e1["wdot"][k0], nu0 * (fwd - rev), rtol=1e-10,
                                   atol=1e-14 * (fwd + rev))
        np.testing.assert_allclose(e2["wdot"][k0], nu0 * (fwd * 2.0 ** of - rev * 2.0 ** orv),
                                   rtol=1e-10, atol=1e-14 * (fwd + rev) * 4)
