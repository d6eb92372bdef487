"""Pins of the surrogate-form oracle: the paper's printed constants, Box-Cox,
GELU, gradients, Adam, projection and the rounding emulators."""
import json
import math
import os

import numpy as np
import pytest
import torch

import chemgen
import oracle
from oracle import ann

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


@pytest.fixture(scope="module")
def paper():
    with open(GOLDEN) as f:
        return json.load(f)


def test_boxcox_endpoints_from_paper(paper):
    bc = paper["boxcox"]
    assert ann.LAMBDA == bc["lambda"]
    assert ann.boxcox(np.array([0.0]))[0] == bc["image_of_0"]
    assert ann.boxcox(np.array([1.0]))[0] == bc["image_of_1"]
    y = np.array([1e-30, 1e-12, 1e-6, 0.01, 0.3, 0.999])
    z = ann.boxcox(y)
    assert np.all((z >= bc["image_of_0"]) & (z <= 0)) and np.all(np.diff(z) > 0)
    np.testing.assert_allclose(ann.inv_boxcox(z), y, rtol=1e-10)
    # negative mass fractions are clamped to 0 before the transform
    assert ann.boxcox(np.array([-1e-9]))[0] == -10.0
    # the inverse maps anything at or below -1/lambda to 0
    assert ann.inv_boxcox(np.array([-10.0, -11.0]))[1] == 0.0
    # lambda -> 0 recovers the log transform
    np.testing.assert_allclose(ann.boxcox(y[1:], 1e-9), np.log(y[1:]), rtol=1e-6, atol=1e-6)


def test_network_shape_from_paper(paper, mech_ch4):
    hid = paper["network"]["hidden"]
    assert tuple(hid) == ann.HIDDEN
    p = ann.init_params([mech_ch4.K + paper["network"]["inputs_besides_species"], *hid,
                         mech_ch4.K], seed=0)
    assert [w.shape for w, _ in p] == [(1600, 32), (800, 1600), (400, 800), (30, 400)]
    nparam = sum(w.size + b.size for w, b in p)
    assert nparam == 1666030


def test_speedup_arithmetic_from_paper(paper):
    """The per-core ratio is the 32-core speed-up times 32."""
    s = paper["speedup"]
    chem = s["cpu_cores"] / (1 - s["chem_time_reduction"])
    flow = s["cpu_cores"] / (1 - s["flow_time_reduction"])
    assert abs(chem - s["chem_per_core_ratio"]) / s["chem_per_core_ratio"] < 0.005
    assert abs(flow - s["flow_per_core_ratio"]) / s["flow_per_core_ratio"] < 0.005


def test_gelu_properties():
    x = np.linspace(-6, 6, 1001)
    g = ann.gelu(x)
    np.testing.assert_allclose(g - ann.gelu(-x), x, atol=1e-15)   # Phi(-x) = 1 - Phi(x)
    assert ann.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(ann.gelu(np.array([8.0])), 8.0, rtol=1e-14)
    d = (ann.gelu(x + 1e-6) - ann.gelu(x - 1e-6)) / 2e-6
    np.testing.assert_allclose(ann.gelu_grad(x), d, atol=1e-8)
    # against math.erf
    ref = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in x[::50]])
    np.testing.assert_allclose(g[::50], ref, rtol=1e-14, atol=1e-300)


def test_l1_gradient_finite_differences():
    rng = np.random.default_rng(0)
    params = ann.init_params([5, 7, 6, 4, 3], seed=1)
    X = rng.standard_normal((9, 5))
    tgt = rng.standard_normal((9, 3))
    grads, loss = ann.backward(params, X, tgt)
    assert abs(loss - ann.l1_loss(ann.forward(params, X), tgt)) < 1e-15
    eps = 1e-7
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            flat = arr.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 6)):
                old = flat[idx]
                flat[idx] = old + eps
                lp = ann.l1_loss(ann.forward(params, X), tgt)
                flat[idx] = old - eps
                lm = ann.l1_loss(ann.forward(params, X), tgt)
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - g.reshape(-1)[idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx)


def test_adam_first_step_closed_form():
    """With m_0 = v_0 = 0 the bias-corrected first step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    params = [(rng.standard_normal((3, 2)), rng.standard_normal(3))]
    grads = [(rng.standard_normal((3, 2)), rng.standard_normal(3))]
    z = [(np.zeros((3, 2)), np.zeros(3))]
    p1, m1, v1 = ann.adam_update(params, grads, z, z, 1, lr=1e-3)
    for a, a1, g in ((params[0][0], p1[0][0], grads[0][0]), (params[0][1], p1[0][1], grads[0][1])):
        np.testing.assert_allclose(a1, a - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m1[0][0], 0.1 * grads[0][0])
    np.testing.assert_allclose(v1[0][0], 0.001 * grads[0][0] ** 2)


def test_projection_kkt(mech_ch4):
    """The weighted projection equals the solution of the KKT system of
    min sum_k (Y_k - Yp_k)^2 / d_k subject to M Y = M Y0, is idempotent and
    leaves a conserving input unchanged; the correction of a species is in
    proportion to its weight, so a species with a small spread (or a
    vanishing mass fraction) barely moves."""
    m = mech_ch4
    T, p, Y0 = chemgen.make_states(m, "ch4", N=6, seed=4)
    rng = np.random.default_rng(2)
    Yp = np.abs(Y0 * (1 + 0.05 * rng.standard_normal(Y0.shape)))
    sd = 10.0 ** rng.uniform(-7, -3, m.K)
    Y = ann.project(m, Y0, Yp, sd)
    M = ann.element_mass_matrix(m)
    np.testing.assert_allclose(M @ Y, M @ Y0, atol=1e-14)
    K, E = m.K, m.E
    for i in range(6):
        d = sd ** 2 * (Yp[:, i] + 1e-10) / (Yp[:, i] + sd)
        A = np.zeros((K + E, K + E))
        A[:K, :K] = np.diag(1.0 / d)
        A[:K, K:] = M.T
        A[K:, :K] = M
        rhs = np.concatenate([Yp[:, i] / d, M @ Y0[:, i]])
        sol = np.linalg.solve(A, rhs)
        np.testing.assert_allclose(Y[:, i], sol[:K], rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(ann.project(m, Y0, Y, sd), Y, atol=1e-15)
    np.testing.assert_allclose(ann.project(m, Y0, Y0, sd), Y0, atol=1e-15)
    # a species whose spread is 1e6 times smaller than the others' takes no
    # visible part of the correction
    sd2 = np.full(m.K, 1e-4)
    j = int(np.argmax(Y0[:, 0]))
    sd2[j] = 1e-10
    Y2 = ann.project(m, Y0[:, :1], Yp[:, :1], sd2)
    assert abs(Y2[j, 0] - Yp[j, 0]) <= 1e-9 * abs(Y2[:, 0] - Yp[:, 0]).max()
    # element mass fractions sum to one when the species ones do
    np.testing.assert_allclose(M.sum(axis=0), 1.0, rtol=1e-14)


def test_bf16_emulation_matches_torch():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 65504.0, 3.4e38, 1e-40]])
    ours = ann.round_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_e4m3_emulation_matches_torch():
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-4, 2.5, 20000),
                        [0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10, 1.5 * 2.0 ** -9, 240.0]])
    x = x[np.abs(x) <= 448.0]
    ours = ann.round_e4m3(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_temperature_newton_conserves_enthalpy(om_ch4):
    m = om_ch4.mech
    T, p, Y0 = chemgen.make_states(m, "ch4", N=5, seed=3)
    out = oracle.chem_step(om_ch4, 1e-5, T, p, Y0)
    Tn = ann.temperature_newton(om_ch4, T, Y0, out["Y"])
    for i in range(5):
        h0 = oracle.mixture_enthalpy(om_ch4, T[i], Y0[:, i])
        h1 = oracle.mixture_enthalpy(om_ch4, Tn[i], out["Y"][:, i])
        assert abs(h1 - h0) <= 1e-9 * abs(h0) + 1e-6
    np.testing.assert_allclose(Tn, out["T"], rtol=1e-5)


def test_forward_against_torch_reference():
    """The oracle's network against an independent evaluation: torch on the
    CPU in FP64, F.linear with exact-erf GELU on the hidden layers and a
    linear output layer; and the BF16 emulation against torch's own bfloat16
    casts of the same layer inputs and weights."""
    import torch.nn.functional as F
    rng = np.random.default_rng(11)
    sizes = [9, 40, 24, 16, 5]
    params = ann.init_params(sizes, seed=12)
    X = rng.standard_normal((33, 9)) * 2.0
    u = ann.forward(params, X)
    h = torch.from_numpy(X)
    for l, (W, b) in enumerate(params):
        h = F.linear(h, torch.from_numpy(W), torch.from_numpy(b))
        if l < len(params) - 1:
            h = F.gelu(h, approximate="none")
    np.testing.assert_allclose(u, h.numpy(), rtol=1e-12, atol=1e-14)

    def bf(t):
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    ub = ann.forward(params, X, prec="bf16")
    h = torch.from_numpy(X)
    for l, (W, b) in enumerate(params):
        h = F.linear(bf(h), bf(torch.from_numpy(W)), torch.from_numpy(b))
        if l < len(params) - 1:
            h = F.gelu(h, approximate="none")
    np.testing.assert_allclose(ub, h.numpy(), rtol=1e-12, atol=1e-14)
    # a dropped bias or a GELU on the output layer would move the result
    assert np.abs(ub - u).max() > 1e-4


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly
    m_hat = g and v_hat = g^2 at every step, so after t steps
    theta_t = theta_0 - t lr g / (|g| + eps), m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2 (Kingma & Ba 2015, Algorithm 1 and Sec. 3)."""
    rng = np.random.default_rng(3)
    th0 = [(rng.standard_normal((4, 3)), rng.standard_normal(4))]
    g = [(rng.standard_normal((4, 3)), rng.standard_normal(4))]
    z = [(np.zeros((4, 3)), np.zeros(4))]
    p, m, v = th0, z, z
    lr, b1, b2 = 2e-3, 0.9, 0.999
    for t in range(1, 6):
        p, m, v = ann.adam_update(p, g, m, v, t, lr=lr, beta1=b1, beta2=b2)
        for i in range(2):
            gg = g[0][i]
            np.testing.assert_allclose(p[0][i], th0[0][i] - t * lr * gg / (np.abs(gg) + 1e-8),
                                       rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(m[0][i], (1 - b1 ** t) * gg, rtol=1e-12)
            np.testing.assert_allclose(v[0][i], (1 - b2 ** t) * gg * gg, rtol=1e-12)


def test_adam_moments_are_exponential_averages():
    """With changing gradients the moments are the exponentially weighted
    sums m_t = (1 - b1) sum_i b1^(t-i) g_i and v_t = (1 - b2) sum_i
    b2^(t-i) g_i^2 (Kingma & Ba 2015, Sec. 3), computed here directly from
    the history; the step uses the bias-corrected moments, which for a
    gradient that flips sign every step are checked against the sum formula."""
    rng = np.random.default_rng(4)
    th = [(rng.standard_normal((2, 2)), rng.standard_normal(2))]
    hist = [[(rng.standard_normal((2, 2)), rng.standard_normal(2))] for _ in range(4)]
    z = [(np.zeros((2, 2)), np.zeros(2))]
    p, m, v = th, z, z
    b1, b2, lr = 0.9, 0.999, 1e-3
    for t in range(1, 5):
        prev = p
        p, m, v = ann.adam_update(p, hist[t - 1], m, v, t, lr=lr, beta1=b1, beta2=b2)
        for i in range(2):
            ms = sum((1 - b1) * b1 ** (t - j) * hist[j - 1][0][i] for j in range(1, t + 1))
            vs = sum((1 - b2) * b2 ** (t - j) * hist[j - 1][0][i] ** 2 for j in range(1, t + 1))
            np.testing.assert_allclose(m[0][i], ms, rtol=1e-12)
            np.testing.assert_allclose(v[0][i], vs, rtol=1e-12)
            # the bias-corrected step: m_t / sum of its weights, over sqrt of v_t / its weights
            wm = sum((1 - b1) * b1 ** (t - j) for j in range(1, t + 1))
            wv = sum((1 - b2) * b2 ** (t - j) for j in range(1, t + 1))
            step = lr * (ms / wm) / (np.sqrt(vs / wv) + 1e-8)
            np.testing.assert_allclose(prev[0][i] - p[0][i], step, rtol=1e-10, atol=1e-16)


def test_ood_flags_hand_built_boxes():
    """Out-of-distribution test on hand-made training boxes: the 5 % margin
    of a feature's span, the relative 1e-6 rule of a zero-span feature (the
    constant pressure), exact boundary values and non-finite features."""
    lo = np.array([0.0, 101325.0, -10.0])
    hi = np.array([10.0, 101325.0, 0.0])
    base = np.array([5.0, 101325.0, -5.0])

    def one(j, x):
        f = base.copy()
        f[j] = x
        return bool(ann.ood_flags(f[:, None], lo, hi)[0])
    assert not one(0, 5.0)
    assert not one(0, -0.5) and not one(0, 10.5)        # exactly on the widened edge
    assert one(0, -0.5000001) and one(0, 10.5000001)
    assert not one(1, 101325.0 * (1 + 0.9e-6)) and not one(1, 101325.0 * (1 - 0.9e-6))
    assert one(1, 101325.0 * (1 + 1.1e-6)) and one(1, 101325.0 * (1 - 1.1e-6))
    assert not one(2, 0.49) and one(2, 0.51) and one(2, -10.51)
    assert one(0, np.nan) and one(2, np.inf) and one(1, -np.inf)
    # several cells at once: a cell is flagged if any feature is outside
    F = np.stack([base, base, base], axis=1)
    F[2, 1] = 0.6
    F[0, 2] = -1.0
    np.testing.assert_array_equal(ann.ood_flags(F, lo, hi), [False, True, True])


def test_zstats_against_library_and_zero_spread():
    """Per-row mean and population standard deviation against Python's
    statistics module; rows without spread (constant, all zero, or spread
    below 1e-12 of the mean) get a standard deviation of 1."""
    import statistics
    rng = np.random.default_rng(8)
    A = np.stack([rng.standard_normal(50) * 3 + 7,
                  np.full(50, 101325.0),
                  np.zeros(50),
                  1e6 + 1e-8 * rng.standard_normal(50),
                  1e-20 * rng.standard_normal(50)])
    mu, sd = ann.zstats(A)
    for i in range(A.shape[0]):
        assert abs(mu[i] - statistics.fmean(A[i])) <= 1e-12 * max(1.0, abs(mu[i]))
    assert abs(sd[0] - statistics.pstdev(A[0])) <= 1e-12 * sd[0]
    assert sd[1] == 1.0 and sd[2] == 1.0 and sd[3] == 1.0
    assert abs(sd[4] - statistics.pstdev(A[4])) <= 1e-9 * sd[4]   # small but real spread


def test_post_residual_flags_judge_the_network(om_ch4):
    """Flag bit 1 is decided on the network's own state Y0 + dY: an output
    that breaks element conservation by more than the tolerance is flagged
    even though the projection repairs it; one that conserves elements (a
    multiple of a reaction's stoichiometry) is not; a NaN output is flagged."""
    m = om_ch4.mech
    T, p, Y0 = chemgen.make_states(m, "ch4", N=4, seed=9)
    K = m.K
    M = ann.element_mass_matrix(m)
    # a conserving change: move mass along reaction 0 (mass units)
    r = np.zeros(K)
    for s in range(4):
        k = m.rsp[0, s]
        if k >= 0:
            r[k] += (1 if s >= 2 else -1) * m.rnu[0, s] * m.W[k]
    assert np.abs(M @ r).max() < 1e-14 * np.abs(r).max()
    du = np.zeros((K, 4))
    # the reverse direction: products (all present at ~8e-7) give up 1e-7 at most
    du[:, 0] = -1e-7 * r / np.abs(r).max()
    assert np.all(Y0[:, 0] + du[:, 0] >= 0)
    iH2O = m.index("H2O")
    du[iH2O, 1] = 5e-6          # H and O mass appear from nowhere: residual ~ 5e-6 * 0.9
    du[iH2O, 2] = 5e-7          # below the tolerance
    du[:, 3] = np.nan
    o = ann.post(om_ch4, T, p, Y0, du, np.zeros(K), np.ones(K), 1e-5)
    assert o["residual_raw"][1] > 1e-6 and o["residual"][1] < 1e-9
    np.testing.assert_array_equal(o["flags"] & 2, [0, 2, 0, 2])


# ---------------------------------------------- physics terms of the loss


@pytest.fixture(scope="module")
def phys_batch(mech_ch4, om_ch4):
    """A few CH4/air states, their oracle step (the label), normalisation and
    a perturbed network output."""
    T, p, Y0 = chemgen.make_states(mech_ch4, "ch4", N=24, seed=61)
    o = oracle.chem_step(om_ch4, 1e-5, T, p, Y0)
    tgt_phys = ann.targets(Y0, o["Y"])
    mu, sd = ann.zstats(tgt_phys)
    tgt = ((tgt_phys - mu[:, None]) / sd[:, None]).T
    rng = np.random.default_rng(62)
    u = tgt + 0.3 * rng.standard_normal(tgt.shape)
    return dict(T=T, p=p, Y0=Y0, Y1=o["Y"], T1=o["T"], mu=mu, sd=sd, tgt=tgt, u=u,
                hT1=ann.species_enthalpy(om_ch4, o["T"]),
                href=ann.species_enthalpy(om_ch4, np.full(T.size, ann.T_REF_HRR)))


def test_phys_energy_term_is_an_enthalpy_difference(om_ch4, phys_batch):
    """The energy functional equals h(T1, Y0 + dY_pred) - h(T1, Y1), the
    mixture enthalpies taken from the C oracle (not from the linear form), and
    that is h(T1, Y0 + dY_pred) - h(T0, Y0) up to the reference step's own
    energy error (rtol-sized)."""
    b = phys_batch
    dYp = (b["u"] * b["sd"][None, :] + b["mu"][None, :]).T
    s = ((b["u"] - b["tgt"]) * b["sd"][None, :] * b["hT1"].T).sum(axis=1)
    for i in range(b["T"].size):
        h_pred = oracle.mixture_enthalpy(om_ch4, b["T1"][i], b["Y0"][:, i] + dYp[:, i])
        h_lab = oracle.mixture_enthalpy(om_ch4, b["T1"][i], b["Y1"][:, i])
        h_0 = oracle.mixture_enthalpy(om_ch4, b["T"][i], b["Y0"][:, i])
        assert abs(s[i] - (h_pred - h_lab)) <= 1e-9 * max(abs(h_lab), abs(s[i]))
        assert abs(h_lab - h_0) <= 1e-5 * abs(h_pred - h_lab) + 1e-8 * abs(h_0)
    terms, _ = ann.physics_terms(b["u"], b["tgt"], b["mu"], b["sd"], b["hT1"], b["href"],
                                 (1, 1, 1))
    D = (np.abs(b["hT1"]) * b["sd"][:, None]).sum(axis=0)
    assert abs(terms[1] - np.mean(np.abs(s) / D)) <= 1e-14 * terms[1]


def test_phys_hrr_term_is_the_heat_release(mech_ch4, om_ch4):
    """The heat-release functional, rho0/dt sum_k h_k(298.15 K) dY_k over a
    very short reference step, tends to the instantaneous heat release rate
    sum_k h_k(298.15 K) W_k wdot_k of the mechanism (C oracle rates); it is
    h(298.15, Y0 + dY) - h(298.15, Y0) by the C oracle's mixture enthalpy."""
    T, p, Y0 = chemgen.make_states(mech_ch4, "ch4", N=64, seed=63)
    sel = T > 1400.0
    T, p, Y0 = T[sel][:6], p[sel][:6], Y0[:, sel][:, :6]
    # the step average differs from the initial rate by O(dt) (1e-3 at 1e-10 s)
    dt = 1e-12
    o = oracle.chem_step(om_ch4, dt, T, p, Y0, opts=oracle.default_opts(rtol=1e-10,
                                                                          atol_Y=1e-20))
    dY = o["Y"] - Y0
    href = ann.species_enthalpy(om_ch4, np.full(T.size, ann.T_REF_HRR))
    rho0 = ann.density(mech_ch4, T, p, Y0)
    q_step = rho0 * (href * dY).sum(axis=0) / dt
    w, _ = oracle.chem_rates(om_ch4, T, p, Y0)
    q_inst = (href * mech_ch4.W[:, None] * w).sum(axis=0)
    np.testing.assert_allclose(q_step, q_inst, rtol=1e-4)
    for i in range(T.size):
        dh = (oracle.mixture_enthalpy(om_ch4, ann.T_REF_HRR, o["Y"][:, i])
              - oracle.mixture_enthalpy(om_ch4, ann.T_REF_HRR, Y0[:, i]))
        # the difference of two mixture enthalpies carries their rounding
        scale = (np.abs(href[:, i]) * (np.abs(Y0[:, i]) + np.abs(o["Y"][:, i]))).sum()
        assert abs((href[:, i] * dY[:, i]).sum() - dh) <= 1e-14 * scale


def test_phys_mass_term_special_cases(phys_batch):
    """A prediction whose changes sum to zero has no mass penalty; a uniform
    shift c of every physical change gives |K c| / sum_k sd_k; a perfect
    prediction has no energy or heat-release penalty."""
    b = phys_batch
    sd, mu = b["sd"], b["mu"]
    dY = b["u"] * sd[None, :] + mu[None, :]
    dY[:, 0] -= dY.sum(axis=1)                       # now sums to zero per sample
    u0 = (dY - mu[None, :]) / sd[None, :]
    terms, _ = ann.physics_terms(u0, b["tgt"], mu, sd, b["hT1"], b["href"], (1, 0, 0))
    assert terms[0] <= 1e-13
    c = 3e-5
    u1 = (dY + c - mu[None, :]) / sd[None, :]
    terms, _ = ann.physics_terms(u1, b["tgt"], mu, sd, b["hT1"], b["href"], (1, 0, 0))
    assert abs(terms[0] - mu.size * c / sd.sum()) <= 1e-9 * terms[0]
    terms, _ = ann.physics_terms(b["tgt"], b["tgt"], mu, sd, b["hT1"], b["href"], (1, 1, 1))
    assert terms[1] == 0.0 and terms[2] == 0.0


def test_phys_gradient_finite_differences(phys_batch):
    """d(sum_t w_t terms_t)/du by central differences, and backward_phys on a
    small network against finite differences of its total loss; with w = 0
    backward_phys is backward."""
    b = phys_batch
    w = (0.7, 1.3, 0.4)
    args = (b["mu"], b["sd"], b["hT1"], b["href"])
    terms, g = ann.physics_terms(b["u"], b["tgt"], *args, w)
    eps = 1e-7
    u = b["u"].copy()
    for i, k in ((0, 0), (3, 7), (11, 29), (23, 15)):
        old = u[i, k]
        u[i, k] = old + eps
        tp, _ = ann.physics_terms(u, b["tgt"], *args, w)
        u[i, k] = old - eps
        tm, _ = ann.physics_terms(u, b["tgt"], *args, w)
        u[i, k] = old
        fd = (np.dot(w, tp) - np.dot(w, tm)) / (2 * eps)
        # central differences of O(1) terms carry ~1e-16 / 1e-7 of rounding
        assert abs(fd - g[i, k]) <= 1e-6 * abs(fd) + 3e-9, (i, k)
    K = b["sd"].size
    params = ann.init_params([K + 2, 9, 7, 5, K], seed=64)
    rng = np.random.default_rng(65)
    X = rng.standard_normal((b["T"].size, K + 2))
    grads, tot, l1, terms = ann.backward_phys(params, X, b["tgt"], *args, w)

    def total():
        uu = ann.forward(params, X)
        t, _ = ann.physics_terms(uu, b["tgt"], *args, w)
        return ann.l1_loss(uu, b["tgt"]) + np.dot(w, t)
    assert abs(tot - total()) <= 1e-14 * tot
    for l, (W, bb) in enumerate(params):
        for arr, gg in ((W, grads[l][0]), (bb, grads[l][1])):
            flat = arr.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 5)):
                old = flat[idx]
                flat[idx] = old + eps
                lp = total()
                flat[idx] = old - eps
                lm = total()
                flat[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - gg.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx)
    g0, tot0, _, _ = ann.backward_phys(params, X, b["tgt"], *args, (0, 0, 0))
    g1, l1b = ann.backward(params, X, b["tgt"])
    assert tot0 == l1b
    for (a, c), (d, e) in zip(g0, g1):
        assert np.array_equal(a, d) and np.array_equal(c, e)


def _block_diagonal(members):
    """One network equal to the ensemble: the members' first layers stacked
    (they share the input), every later layer block-diagonal."""
    K = len(members)
    big = []
    for l in range(len(members[0])):
        Ws = [p[l][0] for p in members]
        bs = np.concatenate([p[l][1] for p in members])
        if l == 0:
            W = np.vstack(Ws)
        else:
            fo, fi = Ws[0].shape
            W = np.zeros((K * fo, K * fi))
            for k in range(K):
                W[k * fo:(k + 1) * fo, k * fi:(k + 1) * fi] = Ws[k]
        big.append((W, bs))
    return big


def test_ensemble_is_a_block_diagonal_network():
    """Five one-output members equal one wide network whose hidden layers are
    block-diagonal: same outputs, and the diagonal blocks of that network's
    L1 gradient (mean over samples and its five outputs) are the members'
    gradients of the ensemble loss."""
    rng = np.random.default_rng(41)
    K, sizes = 5, [7, 12, 9, 6, 1]
    members = [ann.init_params(sizes, 100 + k) for k in range(K)]
    X = rng.standard_normal((33, sizes[0]))
    target = rng.standard_normal((33, K))
    big = _block_diagonal(members)
    np.testing.assert_allclose(ann.ensemble_forward(members, X), ann.forward(big, X),
                               rtol=1e-12, atol=1e-14)
    g_ens, loss_ens = ann.ensemble_backward(members, X, target)
    g_big, loss_big = ann.backward(big, X, target)
    np.testing.assert_allclose(loss_ens, loss_big, rtol=1e-13)
    for l in range(len(sizes) - 1):
        fo, fi = members[0][l][0].shape
        for k in range(K):
            r = slice(k * fo, (k + 1) * fo)
            c = slice(0, fi) if l == 0 else slice(k * fi, (k + 1) * fi)
            np.testing.assert_allclose(g_ens[k][l][0], g_big[l][0][r, c], rtol=1e-11, atol=1e-15)
            np.testing.assert_allclose(g_ens[k][l][1], g_big[l][1][r], rtol=1e-11, atol=1e-15)
