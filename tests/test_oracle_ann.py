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
    leaves a conserving input unchanged."""
    m = mech_ch4
    T, p, Y0 = chemgen.make_states(m, "ch4", N=6, seed=4)
    rng = np.random.default_rng(2)
    Yp = np.abs(Y0 * (1 + 0.05 * rng.standard_normal(Y0.shape)))
    Y = ann.project(m, Y0, Yp)
    M = ann.element_mass_matrix(m)
    np.testing.assert_allclose(M @ Y, M @ Y0, atol=1e-14)
    K, E = m.K, m.E
    for i in range(6):
        d = Yp[:, i] + 1e-10
        A = np.zeros((K + E, K + E))
        A[:K, :K] = np.diag(1.0 / d)
        A[:K, K:] = M.T
        A[K:, :K] = M
        rhs = np.concatenate([Yp[:, i] / d, M @ Y0[:, i]])
        sol = np.linalg.solve(A, rhs)
        np.testing.assert_allclose(Y[:, i], sol[:K], rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(ann.project(m, Y0, Y), Y, atol=1e-15)
    np.testing.assert_allclose(ann.project(m, Y0, Y0), Y0, atol=1e-15)
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
