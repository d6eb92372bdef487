"""Parity of the GPU PaSR closure (chem_pasr_scale) with the oracle of
Sec. 4.1 on the same states, rates and flow time scales: which species take
part is an exact FP64 comparison on both sides; the density's sum of K
positive terms is added in another order (four partial sums per cell), which
moves it by at most (K - 1) ulps, and three more roundings follow, so the
chemical time, the fraction and the scaled rates agree to (K + 4) ulps.
Covers the three register widths of the kernel (9, 30 and 44 species),
ragged sizes, the benchmarked 2^20 cells and the degenerate cells (no
reaction, no mixing time, infinite mixing time, negative times)."""
import sys

import numpy as np
import pytest

import chemgen
import oracle
from oracle import pasr
from gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _rtol(K):
    return (K + 4) * np.finfo(float).eps


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


_MECHS = {}


def _mech(which):
    if which not in _MECHS:
        import paper_2312_05800_amd as P
        m = chemgen.make_mechanism(which)
        _MECHS[which] = (m, P.Mechanism(m))
    return _MECHS[which]


def _synthetic_rates(K, N, seed):
    """Rates over eight decades with whole zero cells and zero species."""
    rng = np.random.default_rng(seed)
    RR = rng.standard_normal((K, N)) * 10.0 ** rng.uniform(-4, 4, (K, N))
    RR[rng.uniform(size=(K, N)) < 0.1] = 0.0
    RR[:, rng.uniform(size=N) < 0.02] = 0.0
    return RR


def _gpu(dev, gmech, T, p, Y, RR, tT, tK, eta=1e-3):
    import torch
    import paper_2312_05800_amd as P
    RRd = to_dev(RR, dev)
    k, tc = P.pasr_scale(gmech, to_dev(T, dev), to_dev(p, dev), to_dev(Y, dev), RRd,
                         to_dev(tT, dev), to_dev(tK, dev), eta=eta)
    torch.cuda.synchronize()
    return k.cpu().numpy(), tc.cpu().numpy(), RRd.cpu().numpy()


def _check(mech, T, p, Y, RR, tT, tK, got, eta=1e-3):
    RTOL = _rtol(mech.K)
    k_g, tc_g, RR_g = got
    k_o, tc_o, RR_o = pasr.scale(mech, T, p, Y, RR, tT, tK, eta)
    np.testing.assert_array_equal(np.isposinf(tc_g), np.isposinf(tc_o))
    fin = np.isfinite(tc_o)
    np.testing.assert_allclose(tc_g[fin], tc_o[fin], rtol=RTOL, atol=0)
    np.testing.assert_allclose(k_g, k_o, rtol=RTOL, atol=0)
    np.testing.assert_allclose(RR_g, RR_o, rtol=RTOL, atol=0)
    exact = np.mean(k_g == k_o)
    _say(f"  kappa bit-identical on {exact:.4f} of the cells; "
         f"kappa range [{k_o.min():.3g}, {k_o.max():.3g}]")


@pytest.mark.parametrize("which,N", [("h2", 4097), ("ch4", 1), ("ch4", 70001), ("wide", 3333)])
def test_pasr_parity_synthetic(dev, which, N):
    _say(f"[pasr] {which} N={N} synthetic rates")
    mech, gm = _mech(which)
    T, p, Y = chemgen.make_states(mech, "h2" if which == "h2" else "ch4", N=N, seed=61)
    RR = _synthetic_rates(mech.K, N, 62)
    tT, tK = chemgen.flow_times(N, seed=63, log_taylor=(-6.0, 2.0), log_kolmogorov=(-7.0, 1.0))
    _check(mech, T, p, Y, RR, tT, tK, _gpu(dev, gm, T, p, Y, RR, tT, tK))


def test_pasr_parity_on_step_rates(dev):
    """Rates of a real step (the oracle's integrator over 1e-5 s) and the
    state after it, with mixing times near this mechanism's chemical times."""
    _say("[pasr] ch4 N=2048 oracle step rates")
    mech, gm = _mech("ch4")
    om = oracle.OracleMech(mech)
    T, p, Y = chemgen.make_states(mech, "ch4", N=2048, seed=64)
    r = oracle.chem_step(om, 1e-5, T, p, Y)
    tT, tK = chemgen.flow_times(T.size, seed=65)
    tT, tK = 1e3 * tT, 1e3 * tK
    _check(mech, r["T"], p, r["Y"], r["RR"], tT, tK,
           _gpu(dev, gm, r["T"], p, r["Y"], r["RR"], tT, tK))


@pytest.mark.parametrize("eta", [0.0, 0.5, 1.0])
def test_pasr_threshold_values(dev, eta):
    _say(f"[pasr] ch4 N=999 eta={eta}")
    mech, gm = _mech("ch4")
    T, p, Y = chemgen.make_states(mech, "ch4", N=999, seed=66)
    RR = _synthetic_rates(mech.K, 999, 67)
    tT, tK = chemgen.flow_times(999, seed=68, log_taylor=(-6.0, 2.0), log_kolmogorov=(-7.0, 1.0))
    _check(mech, T, p, Y, RR, tT, tK, _gpu(dev, gm, T, p, Y, RR, tT, tK, eta=eta), eta=eta)


def test_pasr_degenerate_cells(dev):
    """Cell 0: no reaction (kappa 1, tau_c inf, rates stay 0); 1: zero mixing
    time (kappa 1, rates unchanged bit for bit); 2: infinite mixing time
    (kappa 0); 3: negative time product (kappa NaN); 4: mixing time equal to
    the chemical time (kappa 1/2)."""
    _say("[pasr] degenerate cells")
    mech, gm = _mech("ch4")
    T, p, Y = chemgen.make_states(mech, "ch4", N=5, seed=69)
    RR = _synthetic_rates(mech.K, 5, 70)
    RR[:, 0] = 0.0
    tc = pasr.chemical_time(mech, T, p, Y, RR)
    tT = np.array([1e-3, 0.0, np.inf, -1e-3, tc[4]])
    tK = np.array([1e-4, 1e-4, 1e-4, 1e-4, tc[4]])
    k_g, tc_g, RR_g = _gpu(dev, gm, T, p, Y, RR, tT, tK)
    assert k_g[0] == 1.0 and np.isposinf(tc_g[0]) and not RR_g[:, 0].any()
    assert k_g[1] == 1.0
    np.testing.assert_array_equal(RR_g[:, 1], RR[:, 1])
    assert k_g[2] == 0.0 and not RR_g[:, 2].any()
    assert np.isnan(k_g[3]) and np.all(np.isnan(RR_g[:, 3][RR[:, 3] != 0.0]))
    np.testing.assert_allclose(k_g[4], 0.5, rtol=_rtol(mech.K))


def test_pasr_full_size(dev):
    """The benchmarked 2^20 CH4/air cells, every cell against the oracle."""
    N = 1 << 20
    _say(f"[pasr] ch4 full N={N}")
    mech, gm = _mech("ch4")
    T, p, Y = chemgen.make_states(mech, "ch4")
    RR = _synthetic_rates(mech.K, N, 71)
    tT, tK = chemgen.flow_times(N, seed=72, log_taylor=(-6.0, 2.0), log_kolmogorov=(-7.0, 1.0))
    _check(mech, T, p, Y, RR, tT, tK, _gpu(dev, gm, T, p, Y, RR, tT, tK))


def test_pasr_rejects_bad_arguments(dev):
    import torch
    import paper_2312_05800_amd as P
    mech, gm = _mech("ch4")
    T, p, Y = chemgen.make_states(mech, "ch4", N=8, seed=73)
    RR = _synthetic_rates(mech.K, 8, 74)
    tT, tK = chemgen.flow_times(8, seed=75)
    args = [to_dev(a, dev) for a in (T, p, Y, RR, tT, tK)]
    for eta in (-0.1, 1.5, float("nan")):
        with pytest.raises(P.ChemError):
            P.pasr_scale(gm, *args, eta=eta)
    with pytest.raises(ValueError):
        P.pasr_scale(gm, args[0], args[1], args[2], args[3][:, :4], args[4], args[5])
    torch.cuda.synchronize()
