"""Pins of the PaSR closure oracle (Sec. 4.1: reacting fraction
tau_c / (tau_c + tau_mix), chemical time from the slowest formation rate,
mixing time the geometric mean of the Taylor and Kolmogorov times) against
closed forms: a first-order decay, whose chemical time is 1/k whatever the
state; limits of the fraction; the geometric mean; invariances and the
element balance of the scaled source."""
import numpy as np
import pytest

import chemgen
import oracle
from oracle import pasr

R_CODATA = 8.314462618  # J/mol/K


def _cell(mech, names_y, T=1500.0, p=101325.0):
    Y = np.zeros((mech.K, 1))
    for name, y in names_y.items():
        Y[mech.index(name), 0] = y
    Y[mech.index("N2"), 0] += 1.0 - Y[:, 0].sum()
    return np.array([T]), np.array([p]), Y


def _decay_rates(mech, T, p, Y, a, b, k):
    """Mass rates of a first-order decay a -> b (molar rate -k C_a), with the
    concentration from mole fractions: C_a = X_a p / (R T)."""
    n = Y[:, 0] / mech.W
    X = n / n.sum()
    Ca = X[mech.index(a)] * p[0] / (R_CODATA * T[0])
    RR = np.zeros_like(Y)
    RR[mech.index(a), 0] = -k * Ca * mech.W[mech.index(a)]
    RR[mech.index(b), 0] = -RR[mech.index(a), 0]
    return RR


def test_first_order_decay_time_is_one_over_k(mech_ch4):
    m = mech_ch4
    T, p, Y = _cell(m, {"CH4": 0.05, "CO2": 0.01})
    for k in (3.0, 250.0, 7.5e4):
        RR = _decay_rates(m, T, p, Y, "CH4", "CO2", k)
        tc = pasr.chemical_time(m, T, p, Y, RR)
        np.testing.assert_allclose(tc, [1.0 / k], rtol=1e-14)


def test_the_slowest_species_sets_the_time(mech_ch4):
    """Product b with Y_b = 3 Y_a is formed at the rate a decays: its time is
    3/k, the slower of the two."""
    m = mech_ch4
    T, p, Y = _cell(m, {"CH4": 0.02, "CO2": 0.06})
    k = 40.0
    RR = _decay_rates(m, T, p, Y, "CH4", "CO2", k)
    np.testing.assert_allclose(pasr.chemical_time(m, T, p, Y, RR), [3.0 / k], rtol=1e-14)


def test_activity_threshold_is_inclusive(mech_ch4):
    """A nearly inert abundant species just below eta times the largest rate
    is ignored; at eta times the largest rate it takes part and, being
    abundant, sets the time."""
    m = mech_ch4
    T, p, Y = _cell(m, {"CH4": 0.05, "CO2": 0.01})
    k = 100.0
    RR = _decay_rates(m, T, p, Y, "CH4", "CO2", k)
    amax = np.abs(RR).max()
    n2 = m.index("N2")
    below = RR.copy()
    below[n2, 0] = np.nextafter(pasr.ETA * amax, 0.0)
    np.testing.assert_allclose(pasr.chemical_time(m, T, p, Y, below), [1.0 / k], rtol=1e-14)
    at = RR.copy()
    at[n2, 0] = -(pasr.ETA * amax)
    tc = pasr.chemical_time(m, T, p, Y, at)
    rho = pasr.density(m, T, p, Y)
    np.testing.assert_allclose(tc, rho * Y[n2] / (pasr.ETA * amax), rtol=1e-14)
    assert tc[0] > 100.0 / k


def test_no_reaction_means_fully_reacting(mech_ch4):
    m = mech_ch4
    T, p, Y = _cell(m, {"CH4": 0.05})
    RR = np.zeros_like(Y)
    k, tc, out = pasr.scale(m, T, p, Y, RR, np.array([1e-3]), np.array([1e-4]))
    assert np.isposinf(tc[0]) and k[0] == 1.0
    assert not out.any()


def test_reacting_fraction_limits():
    assert pasr.kappa(2.5e-4, 2.5e-4) == 0.5
    assert pasr.kappa(1e-3, 0.0) == 1.0
    assert pasr.kappa(0.0, 0.0) == 1.0
    assert pasr.kappa(1e-3, np.inf) == 0.0
    assert pasr.kappa(np.inf, 1e-3) == 1.0
    assert pasr.kappa(0.0, 1e-3) == 0.0
    np.testing.assert_allclose(pasr.kappa(3.0, 1.0), 0.75, rtol=0, atol=0)


def test_mixing_time_is_the_geometric_mean():
    t = 3.0e-4
    np.testing.assert_allclose(pasr.mixing_time(4 * t, t), 2 * t, rtol=1e-15)
    np.testing.assert_allclose(pasr.mixing_time(t, 4 * t), 2 * t, rtol=1e-15)
    np.testing.assert_allclose(pasr.mixing_time(t, t), t, rtol=1e-15)
    assert pasr.mixing_time(0.0, t) == 0.0


def test_powers_of_two_scale_the_time_exactly(mech_ch4):
    """tau_c is a concentration over a rate: doubling every rate halves it,
    doubling the pressure (the density) doubles it, bit for bit."""
    m = mech_ch4
    T, p, Y = chemgen.make_states(m, "ch4", N=64, seed=5)
    rng = np.random.default_rng(6)
    RR = rng.standard_normal(Y.shape) * 10.0 ** rng.uniform(-3, 2, Y.shape)
    tc = pasr.chemical_time(m, T, p, Y, RR)
    np.testing.assert_array_equal(pasr.chemical_time(m, T, p, Y, 2.0 * RR), tc / 2.0)
    np.testing.assert_array_equal(pasr.chemical_time(m, T, 2.0 * p, Y, RR), tc * 2.0)


def test_bounded_and_monotone(mech_ch4):
    m = mech_ch4
    T, p, Y = chemgen.make_states(m, "ch4", N=512, seed=7)
    rng = np.random.default_rng(8)
    RR = rng.standard_normal(Y.shape) * 10.0 ** rng.uniform(-3, 2, Y.shape)
    tc = pasr.chemical_time(m, T, p, Y, RR)
    tm = 10.0 ** rng.uniform(-6, 2, T.size)
    k1 = pasr.kappa(tc, tm)
    k2 = pasr.kappa(tc, 2.0 * tm)
    assert np.all((k1 >= 0.0) & (k1 <= 1.0))
    assert np.all(k2 <= k1) and np.any(k2 < k1)


def test_scaled_source_keeps_the_element_balance(mech_ch4):
    """The step's rates conserve every element; one fraction per cell keeps
    that, and every species of a cell is scaled by the same number."""
    m = mech_ch4
    om = oracle.OracleMech(m)
    T, p, Y = chemgen.make_states(m, "ch4", N=96, seed=9)
    r = oracle.chem_step(om, 1e-5, T, p, Y)
    T1, Y1, RR = r["T"], r["Y"], r["RR"]
    tT, tK = chemgen.flow_times(T.size, seed=10)
    # slow mixing: fractions well inside (0, 1) for this mechanism's times
    k, tc, out = pasr.scale(m, T1, p, Y1, RR, 1e3 * tT, 1e3 * tK)
    assert np.all((k > 0.0) & (k < 1.0))
    A = m.comp.T.astype(np.float64) / m.W[None, :]
    # the step's rates balance up to the rounding of Y1 - Y0 over dt
    rho0 = pasr.density(m, T, p, Y)
    bound = 8 * np.finfo(float).eps * (np.abs(A) @ (np.abs(Y) + np.abs(Y1))) * rho0 / 1e-5
    assert np.all(np.abs(A @ RR) <= bound)
    # the scaled source's imbalance is kappa times that, nothing more
    mag = np.abs(A) @ np.abs(out)
    assert np.all(np.abs(A @ out - k * (A @ RR)) <= 1e-14 * mag)
    nz = RR != 0.0
    ratio = np.where(nz, out / np.where(nz, RR, 1.0), np.nan)
    np.testing.assert_allclose(np.nanmax(ratio, axis=0), k, rtol=1e-15)
    np.testing.assert_allclose(np.nanmin(ratio, axis=0), k, rtol=1e-15)
