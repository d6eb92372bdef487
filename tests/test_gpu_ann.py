"""Parity of the HIP surrogate path (forward GEMMs, gradients, Adam,
statistics, post-processing, fallback) with the numpy oracle, through the
C ABI."""
import os
import sys
import tempfile

import numpy as np
import pytest

import chemgen
import oracle
from oracle import ann as oann
from gpu_util import need_gpu, to_dev, compare_state

pytestmark = pytest.mark.gpu

HID = (1600, 800, 400)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.fixture(scope="module")
def mech():
    return chemgen.make_mechanism("ch4")


@pytest.fixture(scope="module")
def data(mech):
    """A small seeded training set: CH4/air states and their oracle step."""
    om = oracle.OracleMech(mech)
    T, p, Y0 = chemgen.make_states(mech, "ch4", N=1024, seed=505)
    o = oracle.chem_step(om, 1e-5, T, p, Y0)
    return dict(T=T, p=p, Y0=Y0, Y1=o["Y"], T1=o["T"])


def _norm_from(data, lam=0.1):
    feat = oann.features(data["T"], data["p"], data["Y0"], lam)
    tgt = oann.targets(data["Y0"], data["Y1"], lam)
    mi, si = oann.zstats(feat)
    mo, so = oann.zstats(tgt)
    return dict(mu_in=mi, sd_in=si, lo=feat.min(axis=1), hi=feat.max(axis=1), mu_out=mo,
                sd_out=so)


def _model(mech, params, nm, dt=1e-5):
    import paper_2312_05800_amd as P
    K = mech.K
    m = P.AnnModel(K + 2, K, HID, seed=1)
    for l, (W, b) in enumerate(params):
        m.set_layer(l, W, b)
    m.set_norm(0.1, dt, nm["mu_in"], nm["sd_in"], nm["lo"], nm["hi"], nm["mu_out"], nm["sd_out"])
    return m


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _oracle_inputs(nm, T, p, Y):
    feat = oann.features(T, p, Y)
    return ((feat - _f32(nm["mu_in"])[:, None]) / _f32(nm["sd_in"])[:, None]).T


def _params32(params):
    return [(_f32(W), _f32(b)) for W, b in params]


def _near_threshold(o, tol=1e-6):
    """Cells whose residual (of the network's own state, or after projection)
    lies within a factor 2 of the tolerance: the FP32 de-normalisation may
    decide them either way."""
    r = np.maximum(o["residual"], o["residual_raw"])
    return (r > 0.5 * tol) & (r < 2 * tol)


def _check_post(Yg, Tg, RRg, o, Y0, U, nm, ok, dt=1e-5, T_rtol=1e-6):
    """Post-processing parity on the cells in `ok`, element by element on the
    change dY = Y - Y0.  The GPU forms dY' = sd u + mu in FP32 (at most two
    roundings, each within 2^-24 of |sd u| + |mu|) and does the rest in FP64;
    the projection spreads a per-species error over the cell's species with a
    gain of a few, so the bound is 16 * 2^-24 * max_k(|sd_k u_k| + |mu_k|) per
    cell plus FP64 rounding of Y.  T from the enthalpy Newton and RR follow."""
    sd, mu = _f32(nm["sd_out"]), _f32(nm["mu_out"])
    scale = (np.abs(U.T * sd[:, None]) + np.abs(mu)[:, None]).max(axis=0)
    bound = 16 * 2.0 ** -24 * scale[None, :] + 4 * 2.0 ** -52 * np.abs(Y0)
    dg = Yg - Y0
    do = o["Y"] - Y0
    err = np.abs(dg - do)[:, ok]
    ratio = float((err / bound[:, ok]).max(initial=0.0))
    _say(f"  dY error / bound: max {ratio:.3f} over {ok.sum()} cells "
         f"(max |dY| {np.abs(do[:, ok]).max(initial=0.0):.2e})")
    assert ratio <= 1.0
    np.testing.assert_allclose(Tg[ok], o["T"][ok], rtol=T_rtol)
    # RR = rho0 dY / dt: the same bound scaled by rho0 / dt, plus FP64 rounding
    rr_bound = (o["rho0"][None, :] / dt) * bound + 1e-13 * np.abs(o["RR"])
    rr_err = np.abs(RRg - o["RR"])
    assert np.all(rr_err[:, ok] <= rr_bound[:, ok])


@pytest.mark.parametrize("N", [3001, 64])
def test_forward_parity(dev, mech, data, N):
    import torch
    _say(f"[ann forward] N={N}")
    K = mech.K
    params = oann.init_params([K + 2, *HID, K], seed=7)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=606)
    U = m.forward(to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev), K)
    torch.cuda.synchronize()
    Ug = U.cpu().numpy().astype(np.float64)
    Uo = oann.forward(_params32(params), _oracle_inputs(nm, T, p, Y), prec="bf16")
    err = np.abs(Ug - Uo)
    _say(f"  max abs {err.max():.3e} rms {np.sqrt((err ** 2).mean()):.3e} |U| {np.abs(Uo).mean():.3f}")
    assert err.max() <= 2e-2 and np.sqrt((err ** 2).mean()) <= 2e-3
    # the BF16 emulation is the right reference: FP64 differs by more than the GPU does
    e64 = np.abs(oann.forward(_params32(params), _oracle_inputs(nm, T, p, Y)) - Uo)
    assert np.sqrt((err ** 2).mean()) < np.sqrt((e64 ** 2).mean())


@pytest.mark.parametrize("hid", [(1600, 400, 400), (1600, 1200, 400)])
def test_forward_parity_400_wide_tiles(dev, mech, data, hid):
    """Second-layer widths that are a multiple of 400 but not of 800 take the
    fused kernel with 400-feature tiles (the first layer recomputed per
    tile) instead of the paired-halves one; same parity bar."""
    import torch
    import paper_2312_05800_amd as P
    N = 3001
    _say(f"[ann forward] hidden={hid} N={N}")
    K = mech.K
    params = oann.init_params([K + 2, *hid, K], seed=9)
    nm = _norm_from(data)
    m = P.AnnModel(K + 2, K, hid, seed=1)
    for l, (W, b) in enumerate(params):
        m.set_layer(l, W, b)
    m.set_norm(0.1, 1e-5, nm["mu_in"], nm["sd_in"], nm["lo"], nm["hi"], nm["mu_out"], nm["sd_out"])
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=607)
    U = m.forward(to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev), K)
    torch.cuda.synchronize()
    Ug = U.cpu().numpy().astype(np.float64)
    Uo = oann.forward(_params32(params), _oracle_inputs(nm, T, p, Y), prec="bf16")
    err = np.abs(Ug - Uo)
    _say(f"  max abs {err.max():.3e} rms {np.sqrt((err ** 2).mean()):.3e}")
    assert err.max() <= 2e-2 and np.sqrt((err ** 2).mean()) <= 2e-3


def test_forward_full_size_sampled(dev, mech, data):
    import torch
    N = 1 << 20
    _say(f"[ann forward] full N={N}")
    K = mech.K
    params = oann.init_params([K + 2, *HID, K], seed=8)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    T, p, Y = chemgen.make_states(mech, "ch4_eval")
    U = m.forward(to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev), K)
    torch.cuda.synchronize()
    idx = np.linspace(0, N - 1, 257).astype(np.int64)
    Ug = U[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    Uo = oann.forward(_params32(params), _oracle_inputs(nm, T[idx], p[idx], Y[:, idx]),
                      prec="bf16")
    err = np.abs(Ug - Uo)
    assert err.max() <= 2e-2 and np.sqrt((err ** 2).mean()) <= 2e-3
    assert torch.isfinite(U).all()


def test_fit_norm(dev, mech, data):
    import paper_2312_05800_amd as P
    K = mech.K
    m = P.AnnModel(K + 2, K, HID, seed=1)
    m.fit_norm(to_dev(data["T"], dev), to_dev(data["p"], dev), to_dev(data["Y0"], dev),
               to_dev(data["Y1"], dev), 0.1, 1e-5)
    g = m.get_norm(K + 2, K)
    o = _norm_from(data)
    # GPU features use FP32 Box-Cox; statistics agree to FP32 feature rounding
    for k in ("mu_in", "lo", "hi"):
        np.testing.assert_allclose(g[k], o[k], rtol=2e-5, atol=2e-5)
    np.testing.assert_allclose(g["sd_in"], o["sd_in"], rtol=1e-3)
    # targets are FP64 differences on both sides, summed in FP64 and stored in
    # FP32: per species within a few FP32 ulps (the mean to a few ulps of the
    # spread where it nearly cancels)
    mu_o, sd_o = o["mu_out"], o["sd_out"]
    assert np.all(np.abs(g["sd_out"] - sd_o) <= 3e-7 * sd_o), (g["sd_out"], sd_o)
    assert np.all(np.abs(g["mu_out"] - mu_o) <= 3e-7 * np.abs(mu_o) + 1e-9 * sd_o), \
        (g["mu_out"], mu_o)
    assert np.all(sd_o < 1e-2) and np.all(sd_o > 0)   # physical dY scale, not O(1)
    assert g["sd_in"][1] == 1.0  # constant pressure: zero spread -> 1
    assert g["lambda"] == pytest.approx(0.1) and g["dt_model"] == 1e-5


@pytest.fixture(scope="module")
def data8k(mech):
    """8192 seeded CH4/air states (one training batch of the benchmark) and
    their oracle step."""
    om = oracle.OracleMech(mech)
    T, p, Y0 = chemgen.make_states(mech, "ch4", N=8192, seed=5050)
    o = oracle.chem_step(om, 1e-5, T, p, Y0)
    return dict(T=T, p=p, Y0=Y0, Y1=o["Y"], T1=o["T"])


@pytest.mark.parametrize("B", [256, 160, 8192])
def test_gradients_and_adam(dev, mech, data, data8k, B):
    """B = 256: 8-way split-K weight gradients; B = 160: no split, row tiles
    that end inside a 128-row tile and 64-wide K-steps that end with a
    zero-filled half; B = 8192: the benchmark's batch (16-way split-K for the
    two large layers)."""
    import torch
    _say(f"[ann grads] B={B}")
    K = mech.K
    params = oann.init_params([K + 2, *HID, K], seed=9)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    src = data if B <= 1024 else data8k
    T, p, Y0, Y1 = src["T"][:B], src["p"][:B], src["Y0"][:, :B], src["Y1"][:, :B]
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    args = [to_dev(a, dev) for a in (T, p, Y0, Y1)]
    m.train_step(*args, loss, lr=0.0)
    torch.cuda.synchronize()
    X = _oracle_inputs(nm, T, p, Y0)
    tgt = ((oann.targets(Y0, Y1) - _f32(nm["mu_out"])[:, None]) / _f32(nm["sd_out"])[:, None]).T
    grads, loss_o = oann.backward(_params32(params), X, tgt, prec="bf16")
    assert abs(loss.item() - loss_o) <= 1e-3 * loss_o
    shapes = [(HID[0], K + 2), (HID[1], HID[0]), (HID[2], HID[1]), (K, HID[2])]
    for l in range(4):
        gW, gb = m.get_grad(l, shapes[l])
        for a, b in ((gW, grads[l][0]), (gb, grads[l][1])):
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            cos = float(np.sum(a * b) / (np.linalg.norm(a) * np.linalg.norm(b)))
            _say(f"  layer {l} rel {rel:.2e} cos {cos:.6f}")
            assert rel <= 1e-2 and cos >= 0.999
    if B != 256:
        return
    # three Adam steps on the same batch, each fed the GPU's own gradients of
    # that step: weights, first and second moments against the oracle's
    # adam_update (FP64 from the same FP32 start); the moments carry over
    # from step to step and the bias correction changes with t
    cur = [tuple(a.astype(np.float64) for a in m.get_layer(l, shapes[l])) for l in range(4)]
    mo = [(np.zeros(sh), np.zeros(sh[0])) for sh in shapes]
    vo = [(np.zeros(sh), np.zeros(sh[0])) for sh in shapes]
    lr = 1e-3
    for t in range(1, 4):
        m.train_step(*args, loss, lr=lr)
        torch.cuda.synchronize()
        assert m.num_steps == t
        g = [tuple(a.astype(np.float64) for a in m.get_grad(l, shapes[l])) for l in range(4)]
        cur, mo, vo = oann.adam_update(cur, g, mo, vo, t, lr=lr)
        for l in range(4):
            Wg, bg = m.get_layer(l, shapes[l])
            mW, vW, mb, vb = m.get_moments(l, shapes[l])
            gs = max(np.abs(g[l][0]).max(), np.abs(g[l][1]).max())
            for a, b in ((Wg, cur[l][0]), (bg, cur[l][1])):
                # FP32 weights: a few ulps of |w| per step plus FP32 rounding of the step
                assert np.all(np.abs(a - b) <= 4 * t * 2.0 ** -24 * np.abs(b) + 1e-5 * lr), (t, l)
            for a, b in ((mW, mo[l][0]), (mb, mo[l][1])):
                assert np.all(np.abs(a - b) <= 1e-6 * np.abs(b) + 1e-7 * gs), (t, l, "m")
            for a, b in ((vW, vo[l][0]), (vb, vo[l][1])):
                assert np.all(np.abs(a - b) <= 1e-6 * np.abs(b) + 1e-7 * gs * gs), (t, l, "v")
        _say(f"  adam step {t}: weights, m, v match the oracle")


def test_gradients_with_physics_terms(dev, mech, data):
    """The physics terms of the loss (mass-fraction sum, energy at T1, heat
    release at 298.15 K) on the GPU against the oracle's backward_phys: the
    loss and the three terms, every layer's gradient, and -- to isolate the
    physics part from the L1 signs -- the change of the output layer's
    gradient when the terms are switched on."""
    import torch
    import paper_2312_05800_amd as P
    _say("[ann grads, physics terms]")
    K = mech.K
    om = oracle.OracleMech(mech)
    gm = P.Mechanism(mech)
    params = oann.init_params([K + 2, *HID, K], seed=19)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    B = 256
    T, p, Y0, Y1, T1 = (data["T"][:B], data["p"][:B], data["Y0"][:, :B], data["Y1"][:, :B],
                        data["T1"][:B])
    w = (0.3, 0.2, 0.1)
    args = [to_dev(a, dev) for a in (T, p, Y0, Y1)]
    T1d = to_dev(T1, dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    terms = torch.zeros(3, dtype=torch.float32, device=dev)
    shapes = [(HID[0], K + 2), (HID[1], HID[0]), (HID[2], HID[1]), (K, HID[2])]
    m.train_step(*args, loss, lr=0.0)
    torch.cuda.synchronize()
    g_plain = m.get_grad(3, shapes[3])[0].astype(np.float64)
    m.train_step(*args, loss, lr=0.0, mech=gm, T1=T1d, w_phys=w, terms=terms)
    torch.cuda.synchronize()
    X = _oracle_inputs(nm, T, p, Y0)
    mu, sd = _f32(nm["mu_out"]), _f32(nm["sd_out"])
    tgt = ((oann.targets(Y0, Y1) - mu[:, None]) / sd[:, None]).T
    h_T1 = oann.species_enthalpy(om, T1)
    h_ref = np.repeat(oann.species_enthalpy(om, oann.T_REF_HRR), B, axis=1)
    grads, total, l1, terms_o = oann.backward_phys(_params32(params), X, tgt, mu, sd, h_T1,
                                                   h_ref, w, prec="bf16")
    grads0, _ = oann.backward(_params32(params), X, tgt, prec="bf16")
    tg = terms.cpu().numpy().astype(np.float64)
    _say(f"  terms gpu {tg} oracle {terms_o}; loss {loss.item():.6f} oracle {total:.6f}")
    # u differs from the emulation by FP32 accumulation (~1e-3 relative)
    np.testing.assert_allclose(tg, terms_o, rtol=2e-2)
    assert abs(loss.item() - total) <= 1e-2 * total
    for l in range(4):
        gW, gb = m.get_grad(l, shapes[l])
        for a, b in ((gW, grads[l][0]), (gb, grads[l][1])):
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            cos = float(np.sum(a * b) / (np.linalg.norm(a) * np.linalg.norm(b)))
            _say(f"  layer {l} rel {rel:.2e} cos {cos:.6f}")
            assert rel <= 1e-2 and cos >= 0.999
    dg = m.get_grad(3, shapes[3])[0].astype(np.float64) - g_plain
    do = grads[3][0] - grads0[3][0]
    rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
    _say(f"  output-layer gradient of the physics terms: rel {rel:.2e}")
    assert rel <= 3e-2


def test_post_and_fallback(dev, mech, data):
    import torch
    import paper_2312_05800_amd as P
    _say("[ann post/fallback]")
    K = mech.K
    om = oracle.OracleMech(mech)
    params = oann.init_params([K + 2, *HID, K], seed=10)
    # scale the output layer down so that the step is a small perturbation
    params[3] = (params[3][0] * 0.02, params[3][1] * 0.02)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    gm = P.Mechanism(mech)
    N = 700
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=707)
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    U = m.forward(Td, pd, Yd, K).cpu().numpy().astype(np.float64)
    # surrogate only (no fallback): compare with the oracle's post-processing
    RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
    flags = torch.zeros(N, dtype=torch.uint8, device=dev)
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)
    m.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags, n_fallback=nfb, fallback=False)
    torch.cuda.synchronize()
    o = oann.post(om, T, p, Y, U.T, _f32(nm["mu_out"]), _f32(nm["sd_out"]), 1e-5,
                  lo=_f32(nm["lo"]), hi=_f32(nm["hi"]))
    fg = flags.cpu().numpy()
    near = _near_threshold(o)
    agree = (fg == o["flags"]) | near
    _say(f"  flagged gpu {np.count_nonzero(fg)} oracle {np.count_nonzero(o['flags'])} "
         f"near-threshold {np.count_nonzero(near)}")
    assert agree.all()
    assert int(nfb.item()) == np.count_nonzero(fg)
    ok = (fg == 0) & (o["flags"] == 0)
    assert ok.sum() > N // 4
    Yg, Tg, RRg = Yd.cpu().numpy(), Td.cpu().numpy(), RR.cpu().numpy()
    _check_post(Yg, Tg, RRg, o, Y, U, nm, ok)
    # flagged cells are untouched without fallback
    np.testing.assert_array_equal(Yg[:, fg != 0], Y[:, fg != 0])
    assert np.all(RRg[:, fg != 0] == 0)
    # everything flagged (dt differs from the training dt): fallback = chem_step
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    m.step(gm, 2e-6, Td, pd, Yd, RR=RR, flags=flags, n_fallback=nfb)
    torch.cuda.synchronize()
    assert int(nfb.item()) == N
    assert np.all(flags.cpu().numpy() & 1)
    oc = oracle.chem_step(om, 2e-6, T, p, Y)
    res = compare_state(Td.cpu().numpy(), Yd.cpu().numpy(), oc["T"], oc["Y"])
    assert res["ok"], res
    np.testing.assert_allclose(RR.cpu().numpy(), oc["RR"], rtol=1e-6,
                               atol=1e-8 * np.abs(oc["RR"]).max())


def test_post_tmid_crossing(dev, mech, data):
    """Post-processing on a mechanism whose species switch NASA ranges at
    different temperatures (T_mid drawn in [700, 1400] K), with cells started
    within +-0.05 K of some species' T_mid (about the size of the step's
    temperature change), so that the enthalpy Newton for T crosses range
    switches: flags, T, Y and RR match the oracle's
    post-processing of the same network output."""
    import torch
    import paper_2312_05800_amd as P
    _say("[ann post, per-species T_mid]")
    K = mech.K
    mt = chemgen.make_mechanism(dict(chemgen.MECH_CONFIGS["ch4"], tmid_range=(700.0, 1400.0),
                                     name="ch4_tmid"))
    om = oracle.OracleMech(mt)
    params = oann.init_params([K + 2, *HID, K], seed=17)
    params[3] = (params[3][0] * 0.05, params[3][1] * 0.05)
    nm = _norm_from(data)
    m = _model(mt, params, nm)
    gm = P.Mechanism(mt)
    N = 1200
    T, p, Y = chemgen.make_states(mt, "ch4", N=N, seed=1717)
    rng = np.random.default_rng(1718)
    tm = mt.nasa[:, 1]
    T[:600] = tm[rng.integers(0, K, 600)] + rng.uniform(-0.05, 0.05, 600)
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    U = m.forward(Td, pd, Yd, K).cpu().numpy().astype(np.float64)
    RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
    flags = torch.zeros(N, dtype=torch.uint8, device=dev)
    m.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags, fallback=False)
    torch.cuda.synchronize()
    o = oann.post(om, T, p, Y, U.T, _f32(nm["mu_out"]), _f32(nm["sd_out"]), 1e-5,
                  lo=_f32(nm["lo"]), hi=_f32(nm["hi"]))
    fg = flags.cpu().numpy()
    near = _near_threshold(o)
    assert ((fg == o["flags"]) | near).all()
    ok = (fg == 0) & (o["flags"] == 0)
    lo_t, hi_t = np.minimum(T, o["T"]), np.maximum(T, o["T"])
    crossed = ok & ((tm[:, None] > lo_t[None, :]) & (tm[:, None] <= hi_t[None, :])).any(axis=0)
    _say(f"  unflagged {ok.sum()} of {N}, Newton across a T_mid in {crossed.sum()} cells")
    assert crossed.sum() >= 20
    Yg, Tg, RRg = Yd.cpu().numpy(), Td.cpu().numpy(), RR.cpu().numpy()
    _check_post(Yg, Tg, RRg, o, Y, U, nm, ok, T_rtol=1e-7)
    np.testing.assert_allclose(Tg[crossed], o["T"][crossed], rtol=1e-7)


def test_save_load_roundtrip(dev, mech, data):
    import torch
    import paper_2312_05800_amd as P
    K = mech.K
    params = oann.init_params([K + 2, *HID, K], seed=11)
    m = _model(mech, params, _norm_from(data))
    T, p, Y = chemgen.make_states(mech, "ch4", N=100, seed=808)
    args = [to_dev(a, dev) for a in (T, p, Y)]
    U1 = m.forward(*args, K)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.bin")
        m.save(path)
        m2 = P.AnnModel.load(path)
        U2 = m2.forward(*args, K)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2)


def test_resume_from_file_is_bit_exact(dev, mech, data):
    """Training N + N steps in one run equals N steps, ann_save, ann_load and N
    more steps, bit for bit (weights, Adam moments, step count): the file
    carries the whole optimiser state."""
    import torch
    import paper_2312_05800_amd as P
    K = mech.K
    dv = {k: to_dev(v, dev) for k, v in data.items()}
    shapes = [(HID[0], K + 2), (HID[1], HID[0]), (HID[2], HID[1]), (K, HID[2])]
    m = P.AnnModel(K + 2, K, HID, seed=21)
    m.fit_norm(dv["T"], dv["p"], dv["Y0"], dv["Y1"], 0.1, 1e-5)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(22)
    idx = [torch.from_numpy(rng.permutation(1024)[:256].astype(np.int64)).to(dev)
           for _ in range(6)]

    def run(model, steps):
        for i in steps:
            model.train_step(dv["T"], dv["p"], dv["Y0"], dv["Y1"], loss, index=idx[i],
                             lr=1e-3 * (1 - 0.1 * i))
        torch.cuda.synchronize()
    run(m, range(3))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.bin")
        m.save(path)
        m2 = P.AnnModel.load(path)
    assert m2.num_steps == 3
    run(m, range(3, 6))
    run(m2, range(3, 6))
    assert m.num_steps == m2.num_steps == 6
    for l in range(4):
        for a, b in zip(m.get_layer(l, shapes[l]) + m.get_moments(l, shapes[l]),
                        m2.get_layer(l, shapes[l]) + m2.get_moments(l, shapes[l])):
            np.testing.assert_array_equal(a, b)


def test_residual_fallback_judges_the_network(dev, mech, data):
    """A network whose output weights are scaled up breaks element
    conservation in many cells by more than the 1e-6 tolerance: exactly the
    cells the oracle flags on the network's own residual are integrated by the
    FP64 fallback and then equal the oracle's chem_step; the others equal the
    oracle's post-processing.  The oracle post-processes the GPU's own network
    output, so the two residuals differ only by the FP32 de-normalisation
    sd u + mu: cells within that rounding of the threshold may go either
    way."""
    import torch
    import paper_2312_05800_amd as P
    _say("[ann residual fallback]")
    K = mech.K
    om = oracle.OracleMech(mech)
    params = oann.init_params([K + 2, *HID, K], seed=23)
    # untrained output weights scaled by 20 (bias unchanged) leave about 70 %
    # of these cells with an element residual of their own state above 1e-6,
    # spread from 3e-7 to 3e-6 (oracle, BF16 emulation)
    params[3] = (params[3][0] * 20.0, params[3][1])
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    gm = P.Mechanism(mech)
    N = 600
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=2323)
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    U = m.forward(Td, pd, Yd, K).cpu().numpy().astype(np.float64)
    RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
    flags = torch.zeros(N, dtype=torch.uint8, device=dev)
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)
    m.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags, n_fallback=nfb)
    torch.cuda.synchronize()
    o = oann.post(om, T, p, Y, U.T, _f32(nm["mu_out"]), _f32(nm["sd_out"]), 1e-5,
                  lo=_f32(nm["lo"]), hi=_f32(nm["hi"]))
    fg = flags.cpu().numpy()
    # rounding of the residual sum_k M_ek dY'_k: each dY'_k carries at most two
    # FP32 roundings of |sd_k u_k| + |mu_k|, and M_ek <= 1
    sd, mu = _f32(nm["sd_out"]), _f32(nm["mu_out"])
    rbound = 4 * 2.0 ** -24 * (np.abs(U.T * sd[:, None]) + np.abs(mu)[:, None]).sum(axis=0)
    r = np.maximum(o["residual"], o["residual_raw"])
    near = np.abs(r - 1e-6) <= rbound
    assert ((fg & 3) == o["flags"])[~near].all()
    res_only = (o["flags"] == 2) & ~near
    ok = (fg == 0) & (o["flags"] == 0)
    _say(f"  residual-flagged {res_only.sum()}, unflagged {ok.sum()} of {N}; "
         f"near the threshold {near.sum()}; n_fallback {int(nfb.item())}")
    assert res_only.sum() >= 20 and ok.sum() >= 20
    assert int(nfb.item()) == np.count_nonzero(fg)
    Tg, Yg, RRg = Td.cpu().numpy(), Yd.cpu().numpy(), RR.cpu().numpy()
    # flagged cells: the FP64 integrator's result
    oc = oracle.chem_step(om, 1e-5, T[fg != 0], p[fg != 0], Y[:, fg != 0])
    res = compare_state(Tg[fg != 0], Yg[:, fg != 0], oc["T"], oc["Y"])
    assert res["ok"], res
    np.testing.assert_allclose(RRg[:, fg != 0], oc["RR"], rtol=1e-6,
                               atol=1e-8 * np.abs(oc["RR"]).max())
    # the others: the surrogate's post-processing
    _check_post(Yg, Tg, RRg, o, Y, U, nm, ok)


def test_training_reduces_loss(dev, mech, data):
    import torch
    import paper_2312_05800_amd as P
    _say("[ann train]")
    K = mech.K
    m = P.AnnModel(K + 2, K, HID, seed=3)
    dv = {k: to_dev(v, dev) for k, v in data.items()}
    m.fit_norm(dv["T"], dv["p"], dv["Y0"], dv["Y1"], 0.1, 1e-5)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(0)
    losses = []
    for it in range(60):
        idx = torch.from_numpy(rng.permutation(1024)[:256].astype(np.int64)).to(dev)
        m.train_step(dv["T"], dv["p"], dv["Y0"], dv["Y1"], loss, index=idx, lr=1e-3)
        losses.append(loss.item())
    _say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.mean(losses[-10:]) < 0.6 * np.mean(losses[:5])


def test_fp8_forward_parity(dev, mech, data):
    """FP8 E4M3 hidden layers: the GPU's calibrated scales equal amax/448 of
    the oracle's BF16 activations and weights, and the output matches the
    oracle's FP8 emulation with those scales."""
    import torch
    _say("[ann fp8]")
    K = mech.K
    params = oann.init_params([K + 2, *HID, K], seed=12)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    Tc, pc, Yc = chemgen.make_states(mech, "ch4", N=2048, seed=909)
    m.quantize_fp8(to_dev(Tc, dev), to_dev(pc, dev), to_dev(Yc, dev))
    sa, sw = m.fp8_scales()
    p32 = _params32(params)
    _, _, hs = oann.forward(p32, _oracle_inputs(nm, Tc, pc, Yc), prec="bf16", keep=True)
    np.testing.assert_allclose(sa, [np.abs(hs[1]).max() / 448, np.abs(hs[2]).max() / 448],
                               rtol=1e-3)
    np.testing.assert_allclose(sw, [np.abs(p32[1][0]).max() / 448, np.abs(p32[2][0]).max() / 448],
                               rtol=1e-6)
    T, p, Y = chemgen.make_states(mech, "ch4", N=3001, seed=910)
    U = m.forward(to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev), K)
    torch.cuda.synchronize()
    Ug = U.cpu().numpy().astype(np.float64)
    sc = {1: (float(sa[0]), float(sw[0])), 2: (float(sa[1]), float(sw[1]))}
    X = _oracle_inputs(nm, T, p, Y)
    Uo = oann.forward(p32, X, prec="fp8", fp8_scales=sc)
    Ub = oann.forward(p32, X, prec="bf16")
    err = np.abs(Ug - Uo)
    e_fmt = np.abs(Uo - Ub)
    _say(f"  fp8 max abs {err.max():.3e} rms {np.sqrt((err ** 2).mean()):.3e}; "
         f"fp8-vs-bf16 rms {np.sqrt((e_fmt ** 2).mean()):.3e}")
    assert np.sqrt((err ** 2).mean()) < 0.25 * np.sqrt((e_fmt ** 2).mean())
    assert err.max() <= 5e-2
    # back to BF16
    m.set_precision(0)
    U2 = m.forward(to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev), K).cpu().numpy()
    assert np.sqrt(((U2 - Ub) ** 2).mean()) <= 2e-3


def test_fp8_step_row_major_fused_output(dev, mech, data):
    """FP8 ann_step on 70 001 cells: enough for the output layer to ride in
    the last FP8 layer's epilogue, too few for the K-blocked layouts (the
    row-major operands of that kernel); matches the oracle's post-processing
    of the FP8 forward output on sampled cells, the last ones included."""
    import torch
    import paper_2312_05800_amd as P
    K = mech.K
    N = 70001
    _say(f"[ann fp8 step] N={N}")
    params = oann.init_params([K + 2, *HID, K], seed=15)
    params[3] = (params[3][0] * 0.02, params[3][1] * 0.02)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    Tc, pc, Yc = chemgen.make_states(mech, "ch4", N=2048, seed=916)
    m.quantize_fp8(to_dev(Tc, dev), to_dev(pc, dev), to_dev(Yc, dev))
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=917)
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    U8 = m.forward(Td, pd, Yd, K).cpu().numpy().astype(np.float64)
    RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
    flags = torch.zeros(N, dtype=torch.uint8, device=dev)
    gm = P.Mechanism(mech)
    m.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags, fallback=False)
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([np.linspace(0, N - 1, 300).astype(np.int64),
                                    np.arange(N - 20, N)]))
    om = oracle.OracleMech(mech)
    o = oann.post(om, T[idx], p[idx], Y[:, idx], U8[idx].T, _f32(nm["mu_out"]),
                  _f32(nm["sd_out"]), 1e-5, lo=_f32(nm["lo"]), hi=_f32(nm["hi"]))
    fg = flags.cpu().numpy()[idx]
    near = _near_threshold(o)
    assert ((fg == o["flags"]) | near).all()
    ok = (fg == 0) & (o["flags"] == 0)
    _say(f"  unflagged {ok.sum()} of {idx.size} sampled cells")
    assert ok.sum() > idx.size // 4
    Yg = Yd.cpu().numpy()[:, idx]
    _check_post(Yg, Td.cpu().numpy()[idx], RR.cpu().numpy()[:, idx], o, Y[:, idx], U8[idx], nm,
                ok)


def test_inference_2p23_cells_in_chunks(dev, mech, data):
    """2^23 cells (the low-precision inference size: four 2^21-cell chunks of
    the inference workspace): BF16 and FP8 forward passes match the oracle's
    emulation on rows sampled across all chunks, with the first and last rows
    of every chunk."""
    import torch
    K = mech.K
    N = 1 << 23
    C = 1 << 21
    _say(f"[ann {N} cells in chunks of {C}]")
    params = oann.init_params([K + 2, *HID, K], seed=14)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    p32 = _params32(params)
    T, p, Y = chemgen.make_states(mech, "ch4_infer")
    assert T.size == N
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    edges = [np.array([c * C - 1, c * C]) for c in range(1, N // C)]
    idx = np.unique(np.concatenate([np.linspace(0, N - 1, 97).astype(np.int64),
                                    np.array([0, 1, N - 2, N - 1]), *edges]))
    it = torch.from_numpy(idx).to(dev)
    X = _oracle_inputs(nm, T[idx], p[idx], Y[:, idx])
    del T, p, Y
    U = m.forward(Td, pd, Yd, K)
    torch.cuda.synchronize()
    assert torch.isfinite(U).all()
    Ug = U[it].cpu().numpy().astype(np.float64)
    del U
    Uo = oann.forward(p32, X, prec="bf16")
    err = np.abs(Ug - Uo)
    _say(f"  bf16 max abs {err.max():.3e} rms {np.sqrt((err ** 2).mean()):.3e} ({idx.size} rows)")
    assert err.max() <= 2e-2 and np.sqrt((err ** 2).mean()) <= 2e-3
    Tc, pc, Yc = chemgen.make_states(mech, "ch4_val")
    m.quantize_fp8(to_dev(Tc, dev), to_dev(pc, dev), to_dev(Yc, dev))
    sa, sw = m.fp8_scales()
    U8 = m.forward(Td, pd, Yd, K)
    torch.cuda.synchronize()
    assert torch.isfinite(U8).all()
    U8g = U8[it].cpu().numpy().astype(np.float64)
    del U8
    sc = {1: (float(sa[0]), float(sw[0])), 2: (float(sa[1]), float(sw[1]))}
    Uo8 = oann.forward(p32, X, prec="fp8", fp8_scales=sc)
    err8 = np.abs(U8g - Uo8)
    e_fmt = np.abs(Uo8 - Uo)
    _say(f"  fp8 max abs {err8.max():.3e} rms {np.sqrt((err8 ** 2).mean()):.3e}; "
         f"fp8-vs-bf16 rms {np.sqrt((e_fmt ** 2).mean()):.3e}")
    assert np.sqrt((err8 ** 2).mean()) < 0.25 * np.sqrt((e_fmt ** 2).mean())
    assert err8.max() <= 5e-2


def test_large_tile_paths_ragged(dev, mech, data):
    """At a cell count that selects the 256-cell direct-to-LDS GEMM tiles and
    leaves a ragged last tile (3 * 2^16 + 37 cells), BF16 and FP8 forward
    passes match the oracle on sampled rows (the last 40 included), and
    ann_step (padded 32-wide output layer, out-of-distribution bits from the
    feature kernel) matches the oracle's post-processing of the same U."""
    import torch
    import paper_2312_05800_amd as P
    K = mech.K
    N = 3 * (1 << 16) + 37
    _say(f"[ann large tiles] N={N}")
    params = oann.init_params([K + 2, *HID, K], seed=13)
    params[3] = (params[3][0] * 0.02, params[3][1] * 0.02)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    p32 = _params32(params)
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=911)
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    idx = np.unique(np.concatenate([np.linspace(0, N - 41, 200).astype(np.int64),
                                    np.arange(N - 40, N)]))
    it = torch.from_numpy(idx).to(dev)
    X = _oracle_inputs(nm, T[idx], p[idx], Y[:, idx])
    # BF16
    U = m.forward(Td, pd, Yd, K)
    torch.cuda.synchronize()
    assert torch.isfinite(U).all()
    Ug = U[it].cpu().numpy().astype(np.float64)
    Uo = oann.forward(p32, X, prec="bf16")
    err = np.abs(Ug - Uo)
    _say(f"  bf16 max abs {err.max():.3e} rms {np.sqrt((err ** 2).mean()):.3e}")
    assert err.max() <= 2e-2 and np.sqrt((err ** 2).mean()) <= 2e-3
    # ann_step on the same cells (no fallback): oracle post of the GPU forward
    RR = torch.zeros((K, N), dtype=torch.float64, device=dev)
    flags = torch.zeros(N, dtype=torch.uint8, device=dev)
    Ufull = U.cpu().numpy().astype(np.float64)
    gm = P.Mechanism(mech)
    m.step(gm, 1e-5, Td, pd, Yd, RR=RR, flags=flags, fallback=False)
    torch.cuda.synchronize()
    om = oracle.OracleMech(mech)
    o = oann.post(om, T[idx], p[idx], Y[:, idx], Ufull[idx].T, _f32(nm["mu_out"]),
                  _f32(nm["sd_out"]), 1e-5, lo=_f32(nm["lo"]), hi=_f32(nm["hi"]))
    fg = flags[it].cpu().numpy()
    near = _near_threshold(o)
    assert ((fg == o["flags"]) | near).all()
    ok = (fg == 0) & (o["flags"] == 0)
    assert ok.sum() > len(idx) // 4
    Yg = Yd[:, it].cpu().numpy()
    _check_post(Yg, Td[it].cpu().numpy(), RR[:, it].cpu().numpy(), o, Y[:, idx], Ufull[idx],
                nm, ok)
    del gm
    # FP8 hidden layers on the same inputs (state restored)
    Td, Yd = to_dev(T, dev), to_dev(Y, dev)
    Tc, pc, Yc = chemgen.make_states(mech, "ch4", N=4096, seed=912)
    m.quantize_fp8(to_dev(Tc, dev), to_dev(pc, dev), to_dev(Yc, dev))
    sa, sw = m.fp8_scales()
    U8 = m.forward(Td, pd, Yd, K)
    torch.cuda.synchronize()
    assert torch.isfinite(U8).all()
    sc = {1: (float(sa[0]), float(sw[0])), 2: (float(sa[1]), float(sw[1]))}
    Uo8 = oann.forward(p32, X, prec="fp8", fp8_scales=sc)
    err8 = np.abs(U8[it].cpu().numpy().astype(np.float64) - Uo8)
    e_fmt = np.abs(Uo8 - Uo)
    _say(f"  fp8 max abs {err8.max():.3e} rms {np.sqrt((err8 ** 2).mean()):.3e}; "
         f"fp8-vs-bf16 rms {np.sqrt((e_fmt ** 2).mean()):.3e}")
    assert np.sqrt((err8 ** 2).mean()) < 0.25 * np.sqrt((e_fmt ** 2).mean())
    assert err8.max() <= 5e-2
    # ann_step on the FP8 path (the output layer fused into the last hidden
    # layer's epilogue): the oracle's post-processing of the FP8 forward output
    RR8 = torch.zeros((K, N), dtype=torch.float64, device=dev)
    flags8 = torch.zeros(N, dtype=torch.uint8, device=dev)
    U8full = U8.cpu().numpy().astype(np.float64)
    gm = P.Mechanism(mech)
    m.step(gm, 1e-5, Td, pd, Yd, RR=RR8, flags=flags8, fallback=False)
    torch.cuda.synchronize()
    o8 = oann.post(om, T[idx], p[idx], Y[:, idx], U8full[idx].T, _f32(nm["mu_out"]),
                   _f32(nm["sd_out"]), 1e-5, lo=_f32(nm["lo"]), hi=_f32(nm["hi"]))
    fg8 = flags8[it].cpu().numpy()
    near8 = _near_threshold(o8)
    assert ((fg8 == o8["flags"]) | near8).all()
    ok8 = (fg8 == 0) & (o8["flags"] == 0)
    assert ok8.sum() > len(idx) // 4
    Yg8 = Yd[:, it].cpu().numpy()
    _check_post(Yg8, Td[it].cpu().numpy(), RR8[:, it].cpu().numpy(), o8, Y[:, idx],
                U8full[idx], nm, ok8)


@pytest.mark.parametrize("N,frac", [(3001, 0.01), ((1 << 21) + 4097, 1.0 / 3000)])
def test_step_audit(dev, mech, data, N, frac):
    """The audit inside ann_step (the integrator judging the network): every
    s-th cell (s the integer nearest 1/f, counted over the whole batch, across the
    2^21-cell chunks) is integrated from its input and compared with what the
    network left.  Against the oracle's step on the same cells and the GPU's
    own outputs: the counts exactly, the largest |T - T_ref|, the per-species
    sums of squared differences and the range of the reference change (the
    GPU's reference integrator agrees with the oracle to ~1e-12)."""
    import torch
    import paper_2312_05800_amd as P
    _say(f"[ann step audit] N={N} f={frac:.5f}")
    K = mech.K
    om = oracle.OracleMech(mech)
    params = oann.init_params([K + 2, *HID, K], seed=31)
    params[3] = (params[3][0] * 0.02, params[3][1] * 0.02)
    nm = _norm_from(data)
    m = _model(mech, params, nm)
    gm = P.Mechanism(mech)
    T, p, Y = chemgen.make_states(mech, "ch4", N=N, seed=32)
    Td, pd, Yd = to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev)
    flags = torch.zeros(N, dtype=torch.uint8, device=dev)
    audit = torch.full((3 + 3 * K,), -7.0, dtype=torch.float64, device=dev)
    m.step(gm, 1e-5, Td, pd, Yd, flags=flags, residual_tol=1e-2, audit_fraction=frac,
           audit=audit)
    torch.cuda.synchronize()
    s = int(np.floor(1.0 / np.float64(np.float32(frac)) + 0.5))
    idx = np.arange(0, N, s)
    o = oracle.chem_step(om, 1e-5, T[idx], p[idx], Y[:, idx])
    fg = flags.cpu().numpy()[idx]
    ok = (fg == 0) & (o["stats"][2] == 0)
    Tg, Yg = Td.cpu().numpy()[idx], Yd.cpu().numpy()[:, idx]
    a = audit.cpu().numpy()
    _say(f"  audited {idx.size}: compared {int(a[0])}, not compared {int(a[1])}")
    assert a[0] == ok.sum() and a[1] == idx.size - ok.sum() and ok.sum() > idx.size // 2
    np.testing.assert_allclose(a[2], np.abs(Tg - o["T"])[ok].max(), rtol=1e-6)
    d = Yg[:, ok] - o["Y"][:, ok]
    dref = o["Y"][:, ok] - Y[:, idx][:, ok]
    sums = (d ** 2).sum(axis=1)
    np.testing.assert_allclose(a[3::3], sums, rtol=1e-6, atol=1e-30)
    np.testing.assert_allclose(a[4::3], dref.min(axis=1), rtol=1e-9, atol=1e-18)
    np.testing.assert_allclose(a[5::3], dref.max(axis=1), rtol=1e-9, atol=1e-18)
