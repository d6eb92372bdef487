"""Pins of the training-set sampler oracle (Sec. 3.1: Eqs. (Trand)-(Yrand),
the renormalisation, the mixing line and the Table 1 constraints) against
the paper's printed constants, closed forms and the composition recipe."""
import json
import os

import numpy as np
import pytest

import chemgen
from oracle import hfrd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_constants_are_the_papers():
    g = json.load(open(GOLDEN))
    a = g["augmentation"]
    assert (hfrd.ALPHA, hfrd.BETA, hfrd.GAMMA) == (a["alpha"], a["beta"], a["gamma"])
    t = g["constraints_table1"]
    assert hfrd.HC == tuple(t["HC_ratio"]) and hfrd.ON == tuple(t["ON_ratio"])
    assert hfrd.PHI == tuple(t["phi"])
    assert hfrd.T_KEEP == 500.0


def test_zero_draws_leave_the_seeds_unchanged(mech_ch4):
    m = mech_ch4
    T, p, Y = chemgen.make_states(m, "ch4", N=257, seed=3)
    n2 = m.index("N2")
    c = np.zeros((m.K + 3, T.size))
    Tn, pn, Yn = hfrd.perturb(T, p, Y, c, n2, hfrd.seed_ranges(T, p, Y, n2))
    np.testing.assert_array_equal(Tn, T)
    np.testing.assert_array_equal(pn, p)
    # y^1 = y, and the seeds already sum to one: the rescaling is 1 up to rounding
    np.testing.assert_allclose(Yn, Y, rtol=1e-14, atol=0)


def test_closed_forms_of_the_draws(mech_ch4):
    """T' = T + alpha c (T_max - T_min) and y' = y^(1 + gamma c) on hand-made
    seeds; 0.01^1.1 = 10^-2.2 exactly in closed form."""
    m = mech_ch4
    K, n2 = m.K, m.index("N2")
    iO2, iCO2 = m.index("O2"), m.index("CO2")
    T = np.array([1000.0, 1800.0])
    p = np.array([101325.0, 101325.0])
    Y = np.zeros((K, 2))
    Y[n2] = [0.70, 0.74]
    Y[iO2] = [0.29, 0.25]
    Y[iCO2] = [0.01, 0.01]
    c = np.zeros((K + 3, 2))
    c[0] = [1.0, -1.0]
    c[3 + iCO2] = [1.0, 1.0]
    Tn, pn, Yn = hfrd.perturb(T, p, Y, c, n2, hfrd.seed_ranges(T, p, Y, n2))
    np.testing.assert_allclose(Tn, [1000.0 + 0.125 * 800.0, 1800.0 - 0.125 * 800.0], rtol=1e-15)
    np.testing.assert_array_equal(pn, p)  # constant pressure: p_max - p_min = 0
    # before the rescaling the CO2 entry is 10^-2.2; the rescaling keeps the
    # ratio to O2 and puts the non-N2 sum at 1 - y_N2
    for i in range(2):
        ratio = 10.0 ** -2.2 / Y[iO2, i]
        assert abs(Yn[iCO2, i] / Yn[iO2, i] - ratio) <= 1e-13 * ratio
        assert abs(Yn[:, i].sum() - 1.0) <= 1e-15
        assert Yn[n2, i] == Y[n2, i]


def test_n2_draw_and_rescaling(mech_ch4):
    m = mech_ch4
    T, p, Y = chemgen.make_states(m, "ch4", N=64, seed=5)
    n2 = m.index("N2")
    rng = np.random.default_rng(0)
    c = rng.uniform(-1, 1, (m.K + 3, 64))
    r = hfrd.seed_ranges(T, p, Y, n2)
    Tn, pn, Yn = hfrd.perturb(T, p, Y, c, n2, r)
    np.testing.assert_allclose(Yn[n2], Y[n2] + 0.125 * c[2] * (r[5] - r[4]), rtol=1e-15)
    np.testing.assert_allclose(Yn.sum(axis=0), 1.0, rtol=0, atol=2e-15)
    assert np.all(Yn >= 0)
    # every species present in the seed stays present, absent ones stay absent
    assert np.array_equal(Yn > 0, Y > 0)


def test_mixing_line_ends(mech_ch4):
    m = mech_ch4
    eq = chemgen.burnt_state(m, 0.45, 1500.0)
    air = chemgen.air_state(m)
    T, p, Y = hfrd.mix(eq, air, np.array([0.0, 1.0, 0.5]))
    assert T[0] == eq[0] and T[1] == air[0] and T[2] == 0.5 * (eq[0] + air[0])
    np.testing.assert_array_equal(Y[:, 0], eq[2])
    np.testing.assert_array_equal(Y[:, 1], air[2])
    np.testing.assert_allclose(Y.sum(axis=0), 1.0, atol=1e-15)


def test_ratios_recover_the_recipe(mech_ch4):
    """Element ratios of the recipe's CH4/air states: H/C = 4, O/N = 2/(2 x
    3.76) and phi equal to the equivalence ratio each cell was built with,
    burnt or not (reactions conserve elements)."""
    m = mech_ch4
    N = 512
    rng = np.random.Generator(np.random.PCG64(22))
    phi_drawn = rng.uniform(0.5, 1.3, N)  # make_states draws phi first from this stream
    T, p, Y = chemgen.make_states(m, "ch4", N=N, seed=22)
    hc, on, phi = hfrd.ratios(m, Y)
    # the recipe seeds every radical at up to 1e-6 (H, O, OH, CH3, ... carry
    # H/C/O atoms) before the renormalisation: against about 1 mol/kg of each
    # element that moves the ratios by up to ~1e-4
    np.testing.assert_allclose(hc, 4.0, rtol=2e-4)
    np.testing.assert_allclose(on, 1.0 / 3.76, rtol=2e-4)
    np.testing.assert_allclose(phi, phi_drawn, rtol=5e-4)
    # unburnt and burnt states built without radicals: exact to rounding
    eq = chemgen.burnt_state(m, 0.45, 1500.0)
    hc, on, phi = hfrd.ratios(m, eq[2][:, None])
    np.testing.assert_allclose([hc[0], on[0], phi[0]], [4.0, 1.0 / 3.76, 0.45], rtol=1e-13)


def test_keep_rules(mech_ch4):
    m = mech_ch4
    n2 = m.index("N2")
    eq = chemgen.burnt_state(m, 0.45, 1500.0)
    air = chemgen.air_state(m)
    Y = np.stack([eq[2], eq[2], eq[2], air[2]], axis=1)
    T = np.array([1500.0, 499.9, 500.0, 300.0])
    k = hfrd.keep(m, T, Y, n2=n2)
    # below 500 K dropped, at 500 K kept; pure air has no C or H: H/C undefined
    assert k.tolist() == [True, False, True, False]
    # phi: 0.45 inside [0.20, 1.15]; the leanest mixing state still inside the
    # box is where the line crosses phi = 0.2
    s = np.linspace(0, 1, 1001)
    Tm, pm, Ym = hfrd.mix(eq, air, s)
    _, _, phi = hfrd.ratios(m, Ym)
    km = hfrd.keep(m, np.full(s.size, 1000.0), Ym, n2=n2)
    assert np.all(km == ((phi >= 0.2) & (phi <= 1.15)))
    assert km[0] and not km[-1]
