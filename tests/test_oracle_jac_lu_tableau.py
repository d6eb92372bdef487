"""Pins of the oracle's equilibrium behaviour, analytic Jacobian, pivoted LU
and the Rosenbrock tableau."""
import numpy as np
import pytest

import chemgen
import oracle
from oracle.equilibrium import equilibrium_state


@pytest.mark.parametrize("which", ["h2", "ch4"])
@pytest.mark.parametrize("T", [1100.0, 1800.0, 2600.0])
def test_equilibrium_zero_net_rates(which, T, om_h2, om_ch4):
    """At a constructed equilibrium state every reaction's forward and reverse
    rates balance (K_c = k_f/k_r is consistent with the Gibbs energies), so the
    RHS vanishes relative to the one-way rates and a chemistry step leaves the
    state unchanged."""
    om = om_h2 if which == "h2" else om_ch4
    m = om.mech
    rng = np.random.default_rng(int(T))
    Y = equilibrium_state(om, T, oracle.PREF, rng.uniform(-8, -2, m.E))
    y = np.concatenate([[T], Y])
    ev = oracle.evaluate(om, oracle.PREF, y)
    S = np.sum(Y / m.W)
    Cc = oracle.PREF / (oracle.RGAS * T * S) * Y / m.W
    for r in range(m.R):
        f1 = ev["kf"][r] * np.prod([Cc[m.rsp[r, s]] ** m.rnu[r, s] for s in (0, 1)
                                    if m.rsp[r, s] >= 0])
        r1 = ev["kr"][r] * np.prod([Cc[m.rsp[r, s]] ** m.rnu[r, s] for s in (2, 3)
                                    if m.rsp[r, s] >= 0])
        assert abs(f1 - r1) <= 1e-10 * max(f1, r1) + 1e-300
    out = oracle.chem_step(om, 1e-5, np.array([T]), np.array([oracle.PREF]), Y[:, None])
    assert out["stats"][2, 0] == 0
    assert abs(out["T"][0] - T) <= 1e-10 * T
    np.testing.assert_allclose(out["Y"][:, 0], Y, rtol=1e-10, atol=1e-16)


def _fd_jac(om, p, y):
    """Richardson-extrapolated central differences of the oracle RHS."""
    n = y.size
    J = np.zeros((n, n))
    for j in range(n):
        h = 1e-4 * y[0] if j == 0 else 1e-4 * max(abs(y[j]), 1e-3)

        def cd(d):
            yp, ym = y.copy(), y.copy()
            yp[j] += d
            ym[j] -= d
            return (oracle.rhs(om, p, yp) - oracle.rhs(om, p, ym)) / (2 * d)

        J[:, j] = (4 * cd(h / 2) - cd(h)) / 3
    return J


@pytest.mark.parametrize("which", ["h2", "ch4"])
def test_analytic_jacobian_vs_finite_differences(which, om_h2, om_ch4):
    om = om_h2 if which == "h2" else om_ch4
    cfg = "h2" if which == "h2" else "ch4"
    T, p, Y = chemgen.make_states(om.mech, cfg, N=12, seed=9)
    checked = 0
    for i in range(T.size):
        if abs(T[i] - 1000.0) < 20.0:  # NASA range switch: derivative jumps there
            continue
        y = np.concatenate([[T[i]], Y[:, i]])
        J = oracle.jacobian(om, p[i], y)
        Jfd = _fd_jac(om, p[i], y)
        big = np.abs(J) > 1e-7 * np.abs(J).max()
        rel = np.abs(J - Jfd)[big] / np.abs(J)[big]
        assert np.percentile(rel, 99) < 2e-5, (i, rel.max())
        # entries are allowed FD noise relative to their row scale
        row = np.abs(J).max(axis=1, keepdims=True)
        col = np.abs(J).max(axis=0, keepdims=True)
        assert np.all(np.abs(J - Jfd) <= 1e-5 * np.minimum(row, col) + 1e-300)
        checked += 1
    assert checked >= 8


def test_lu_matches_lapack():
    rng = np.random.default_rng(3)
    for n in (1, 2, 5, 10, 31, 32):
        for _ in range(5):
            A = rng.standard_normal((n, n)) * 10.0 ** rng.uniform(-3, 3, (n, 1))
            b = rng.standard_normal(n)
            st, F, order = oracle.lu(A)
            assert st == 0
            x = oracle.lu_solve(F, order, b)
            x_ref = np.linalg.solve(A, b)
            cond = np.linalg.cond(A)
            assert np.linalg.norm(x - x_ref) <= 1e-13 * cond * np.linalg.norm(x_ref)
            # pivot rule: step-0 pivot is the first row with max |a_i0|
            assert order[0] == int(np.argmax(np.abs(A[:, 0])))
            assert sorted(order.tolist()) == list(range(n))


def test_lu_on_actual_rosenbrock_matrix(om_ch4):
    T, p, Y = chemgen.make_states(om_ch4.mech, "ch4", N=4, seed=2)
    for i in range(4):
        y = np.concatenate([[T[i]], Y[:, i]])
        J = oracle.jacobian(om_ch4, p[i], y)
        for h in (1e-9, 1e-7, 1e-5):
            M = np.eye(J.shape[0]) / (0.5 * h) - J
            b = oracle.rhs(om_ch4, p[i], y)
            st, F, order = oracle.lu(M)
            assert st == 0
            x = oracle.lu_solve(F, order, b)
            r = M @ x - b
            assert np.linalg.norm(r) <= 1e-12 * np.linalg.cond(M) * np.linalg.norm(b) + 1e-300


def test_lu_singular_detected():
    A = np.array([[1.0, 2.0], [2.0, 4.0]])
    st, _, _ = oracle.lu(A)
    assert st == 1
    st, _, _ = oracle.lu(np.zeros((3, 3)))
    assert st == 1


def _ros_coeffs():
    tb = oracle.tableau()
    g, A, Cc = tb["gamma"], tb["A"], tb["C"]
    s = A.shape[0]
    Gam = np.linalg.inv(np.diag(np.full(s, 1.0 / g)) - Cc)  # Gamma = (diag(1/g) - C)^-1
    alpha = A @ Gam
    b = tb["m"] @ Gam
    bhat = (tb["m"] - tb["e"]) @ Gam
    return g, alpha, Gam, b, bhat, tb


def _order_conditions(g, alpha, Gam, bb):
    """Rosenbrock order conditions up to order 4 (Hairer & Wanner II, Table
    IV.7.1), residuals."""
    beta = alpha + Gam
    bp = beta - np.diag(np.diag(beta))
    betap = bp.sum(axis=1)
    al = alpha.sum(axis=1)
    return np.array([
        bb.sum() - 1.0,
        bb @ betap - (0.5 - g),
        bb @ al ** 2 - 1.0 / 3.0,
        bb @ (bp @ betap) - (1.0 / 6.0 - g + g * g),
        bb @ al ** 3 - 0.25,
        bb @ (al * (alpha @ betap)) - (1.0 / 8.0 - g / 3.0),
        bb @ (bp @ al ** 2) - (1.0 / 12.0 - g / 3.0),
        bb @ (bp @ (bp @ betap)) - (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g ** 3),
    ])


def test_tableau_order_conditions():
    g, alpha, Gam, b, bhat, tb = _ros_coeffs()
    np.testing.assert_allclose(np.diag(Gam), g)
    main = _order_conditions(g, alpha, Gam, b)
    emb = _order_conditions(g, alpha, Gam, bhat)
    assert np.all(np.abs(main[:4]) < 1e-14)          # order 3
    assert np.abs(main[4:]).max() > 1e-3              # not order 4
    assert np.all(np.abs(emb[:2]) < 1e-14)            # embedded order 2
    assert np.abs(emb[2:4]).max() > 1e-3
    # stage 2 has the same argument as stage 1, so it may reuse f
    assert np.all(tb["A"][1] == tb["A"][0]) and tb["newf"][1] == 0
    # stiffly accurate: y_new is the last stage argument plus K_4
    np.testing.assert_allclose(tb["m"][:3], tb["A"][3][:3])
    assert tb["m"][3] == 1.0


def test_tableau_stability_function():
    """On y' = lambda y the step multiplies y by R(h lambda); L-stability means
    |R| <= 1 on the left half-plane and R(-inf) = 0, for the main and the
    embedded solution; near 0, R(z) = e^z + O(z^4)."""
    for z in (-1e12, -1e6, -30.0, -2.0, -0.5):
        yn, ye = oracle.ros_step_generic(1, lambda y: z * y, lambda y: np.array([[z]]),
                                         np.array([1.0]), 1.0)
        assert abs(yn[0]) <= 1.0 and abs(ye[0]) <= 1.0
    yn, ye = oracle.ros_step_generic(1, lambda y: -1e15 * y, lambda y: np.array([[-1e15]]),
                                     np.array([1.0]), 1.0)
    assert abs(yn[0]) < 1e-12 and abs(ye[0]) < 1e-12
    errs = []
    for z in (1e-2, 5e-3):
        yn, _ = oracle.ros_step_generic(1, lambda y: -z * y, lambda y: np.array([[-z]]),
                                        np.array([1.0]), 1.0)
        errs.append(abs(yn[0] - np.exp(-z)))
    assert 12.0 < errs[0] / errs[1] < 20.0           # local error ~ z^4


def test_local_error_order_nonlinear():
    """Local error on a nonlinear system with known solution scales as h^4
    (order 3) for the main and h^3 (order 2) for the embedded solution."""
    # y1' = -y2 + y1(1 - y1^2 - y2^2), y2' = y1 + y2(1 - r^2): unit-circle limit cycle
    def f(y):
        r2 = y[0] ** 2 + y[1] ** 2
        return np.array([-y[1] + y[0] * (1 - r2), y[0] + y[1] * (1 - r2)])

    def jac(y):
        x, z = y
        r2 = x * x + z * z
        return np.array([[1 - r2 - 2 * x * x, -1 - 2 * x * z], [1 - 2 * x * z, 1 - r2 - 2 * z * z]])

    def exact(t, r0=0.5, th0=0.3):
        # r' = r(1 - r^2), theta' = 1
        r = 1.0 / np.sqrt(1.0 + (1.0 / r0 ** 2 - 1.0) * np.exp(-2 * t))
        return np.array([r * np.cos(th0 + t), r * np.sin(th0 + t)])

    y0 = exact(0.0)
    hs = [0.01, 0.005, 0.0025]
    em, ee = [], []
    for h in hs:
        yn, ye = oracle.ros_step_generic(2, f, jac, y0, h)
        em.append(np.linalg.norm(yn - exact(h)))
        ee.append(np.linalg.norm(ye - exact(h)))
    sm = np.polyfit(np.log(hs), np.log(em), 1)[0]
    se = np.polyfit(np.log(hs), np.log(ee), 1)[0]
    assert 3.8 < sm < 4.3, sm
    assert 2.8 < se < 3.3, se
