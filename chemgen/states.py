"""Seeded synthetic cell states (T, p, Y_k) in SoA layout.

Stand-ins for the paper's LES cell states and flamelet samples (Sec. 3.1,
Sec. 4.1), which are not available:

* stratified fuel/air mixtures with a per-cell equivalence ratio phi, mixed
  with their complete-combustion products by a per-cell progress variable c:
  Y = (1-c) Y_unburnt(phi) + c Y_burnt(phi), radicals seeded at
  1e-6 * 4c(1-c) each, then every species except N2 rescaled so the mass
  fractions sum to one (the renormalisation rule of Sec. 3.1);
* air is O2:N2 = 1:3.76 by moles; lean products are CO2/H2O/O2/N2; rich
  products put C into CO, H into H2O with the remaining O, turn CO into CO2
  with any O left over, and any H left over into H2.

Layout: T[N], p[N] and Y[K, N] float64 (row k holds species k of every cell).
"""
from __future__ import annotations

import numpy as np

from .mech import Mech

P_ATM = 101325.0

STATE_CONFIGS = {
    # small H2/air case: T independent of the progress variable
    "h2": dict(fuel="H2", phi=(0.5, 1.5), T=("uniform", 1000.0, 2500.0), N=4096, seed=11,
               dt=1e-6),
    # stratified CH4/air: T = 300 + 2000 c
    "ch4": dict(fuel="CH4", phi=(0.5, 1.3), T=("progress", 300.0, 2300.0), N=1 << 20, seed=22,
                dt=1e-5),
    "ch4_eval": dict(fuel="CH4", phi=(0.5, 1.3), T=("progress", 300.0, 2300.0), N=1 << 20,
                     seed=33, dt=1e-5),
    "ch4_train": dict(fuel="CH4", phi=(0.5, 1.3), T=("progress", 300.0, 2300.0), N=1 << 22,
                      seed=55, dt=1e-5, perturb=(0.05, 50.0)),
    "ch4_val": dict(fuel="CH4", phi=(0.5, 1.3), T=("progress", 300.0, 2300.0), N=1 << 16,
                    seed=56, dt=1e-5, perturb=(0.05, 50.0)),
    "ch4_infer": dict(fuel="CH4", phi=(0.5, 1.3), T=("progress", 300.0, 2300.0), N=1 << 23,
                      seed=57, dt=1e-5),
}


def _moles_unburnt(mech: Mech, fuel: str, phi: np.ndarray) -> np.ndarray:
    K, N = mech.K, phi.size
    X = np.zeros((K, N))
    iO2, iN2 = mech.index("O2"), mech.index("N2")
    if fuel == "CH4":
        X[mech.index("CH4")] = 1.0
        X[iO2] = 2.0 / phi
    elif fuel == "H2":
        X[mech.index("H2")] = 2.0 * phi
        X[iO2] = 1.0
    else:
        raise ValueError(fuel)
    X[iN2] = 3.76 * X[iO2]
    return X


def _moles_burnt(mech: Mech, fuel: str, phi: np.ndarray) -> np.ndarray:
    K, N = mech.K, phi.size
    X = np.zeros((K, N))
    iO2, iN2, iH2O, iH2 = (mech.index(s) for s in ("O2", "N2", "H2O", "H2"))
    if fuel == "CH4":
        nC, nH, nO = np.ones(N), 4.0 * np.ones(N), 4.0 / phi   # O atoms from 2/phi O2
        nN2 = 3.76 * 2.0 / phi
    else:
        nC, nH, nO = np.zeros(N), 4.0 * phi, 2.0 * np.ones(N)
        nN2 = 3.76 * np.ones(N)
    lean = nO >= 2.0 * nC + 0.5 * nH
    # lean: complete oxidation
    co2 = np.where(lean, nC, 0.0)
    h2o = np.where(lean, 0.5 * nH, 0.0)
    o2 = np.where(lean, 0.5 * (nO - 2.0 * nC - 0.5 * nH), 0.0)
    # rich: C -> CO, then H -> H2O with the O that is left, then CO -> CO2
    o_left = nO - nC
    h2o_r = np.minimum(0.5 * nH, np.maximum(o_left, 0.0))
    o_left = o_left - h2o_r
    co2_r = np.minimum(nC, np.maximum(o_left, 0.0))
    co_r = nC - co2_r
    h2_r = 0.5 * nH - h2o_r
    co2 = np.where(lean, co2, co2_r)
    h2o = np.where(lean, h2o, h2o_r)
    X[iH2O] = h2o
    X[iO2] = o2
    X[iH2] = np.where(lean, 0.0, h2_r)
    if fuel == "CH4":
        X[mech.index("CO2")] = co2
        X[mech.index("CO")] = np.where(lean, 0.0, co_r)
    X[iN2] = nN2
    return X


def _mass_fractions(mech: Mech, X: np.ndarray) -> np.ndarray:
    m = X * mech.W[:, None]
    return m / m.sum(axis=0, keepdims=True)


def _renormalise(mech: Mech, Y: np.ndarray) -> np.ndarray:
    iN2 = mech.index("N2")
    others = np.ones(mech.K, dtype=bool)
    others[iN2] = False
    s = Y[others].sum(axis=0)
    Y = Y.copy()
    Y[others] *= (1.0 - Y[iN2]) / s
    return Y


def make_states(mech: Mech, cfg: str | dict, N: int | None = None, seed: int | None = None):
    """Return (T[N], p[N], Y[K,N]) float64 for the state recipe ``cfg``."""
    c = dict(STATE_CONFIGS[cfg]) if isinstance(cfg, str) else dict(cfg)
    N = int(c["N"] if N is None else N)
    seed = int(c["seed"] if seed is None else seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    phi = rng.uniform(c["phi"][0], c["phi"][1], N)
    prog = rng.uniform(0.0, 1.0, N)
    kind, lo, hi = c["T"]
    if kind == "uniform":
        T = rng.uniform(lo, hi, N)
    else:
        T = lo + (hi - lo) * prog
    Yu = _mass_fractions(mech, _moles_unburnt(mech, c["fuel"], phi))
    Yb = _mass_fractions(mech, _moles_burnt(mech, c["fuel"], phi))
    Y = (1.0 - prog) * Yu + prog * Yb
    Y[mech.radical] += 1e-6 * 4.0 * prog * (1.0 - prog)
    Y = _renormalise(mech, Y)
    p = np.full(N, c.get("p", P_ATM))
    if "perturb" in c:
        T, p, Y = perturb_states(mech, T, p, Y, seed + 1000003, *c["perturb"])
    return np.ascontiguousarray(T), np.ascontiguousarray(p), np.ascontiguousarray(Y)


def perturb_states(mech: Mech, T, p, Y, seed: int, frac_Y: float = 0.05, dT: float = 50.0):
    """Y_k <- Y_k (1 + frac_Y u_k), T <- T + dT u_T with u ~ U(-1, 1), then the
    Sec. 3.1 renormalisation of every species except N2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    uY = rng.uniform(-1.0, 1.0, Y.shape)
    uT = rng.uniform(-1.0, 1.0, T.shape)
    Y2 = _renormalise(mech, Y * (1.0 + frac_Y * uY))
    return T + dT * uT, p.copy(), Y2


def multiset_workload(mech: Mech, seed: int = 44, n_sets: int = 64, log_size=(3.0, 6.0),
                      log_dt=(-7.0, -4.0), max_total: int | None = None):
    """Uneven batched workload: ``n_sets`` independent cell sets with sizes
    floor(10^U(log_size)) and per-set dt = 10^U(log_dt); per cell T ~ U(300, 2500)
    and a stratified CH4/air composition.  Returns a list of dicts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(10.0 ** rng.uniform(log_size[0], log_size[1], n_sets)).astype(np.int64)
    if max_total is not None and sizes.sum() > max_total:
        sizes = np.maximum(1, (sizes * (max_total / sizes.sum())).astype(np.int64))
    dts = 10.0 ** rng.uniform(log_dt[0], log_dt[1], n_sets)
    sets = []
    for s in range(n_sets):
        cfg = dict(fuel="CH4", phi=(0.5, 1.3), T=("uniform", 300.0, 2500.0), N=int(sizes[s]),
                   seed=seed * 1000 + s)
        T, p, Y = make_states(mech, cfg)
        sets.append(dict(N=int(sizes[s]), dt=float(dts[s]), T=T, p=p, Y=Y))
    return sets


def element_matrix(mech: Mech) -> np.ndarray:
    """Atoms of element e per species k, as float64 [E, K] (pure bookkeeping of
    the mechanism's composition table)."""
    return mech.comp.T.astype(np.float64)


def hfrd_randoms(K: int, N: int, seed: int, mix_fraction: float = 0.1):
    """Random numbers of the training-set sampler for N seeds of K species:
    c [K + 3, N] uniform in [-1, 1] (rows: T, p, N2, then one per species)
    and s [N]: -1 for a seed that is perturbed, a mixing fraction uniform in
    [0, 1] for the share mix_fraction of seeds replaced by a mixing-line
    state."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(-1.0, 1.0, (K + 3, N))
    s = np.full(N, -1.0)
    m = rng.uniform(0.0, 1.0, N) < mix_fraction
    s[m] = rng.uniform(0.0, 1.0, int(m.sum()))
    return np.ascontiguousarray(c), s


def air_state(mech: Mech, T: float = 300.0, p: float = P_ATM):
    """Ambient air, O2:N2 = 1:3.76 by moles: (T, p, Y[K])."""
    X = np.zeros((mech.K, 1))
    X[mech.index("O2")] = 1.0
    X[mech.index("N2")] = 3.76
    return T, p, _mass_fractions(mech, X)[:, 0].copy()


def burnt_state(mech: Mech, phi: float, T: float, fuel: str = "CH4", p: float = P_ATM):
    """The recipe's complete-combustion products at equivalence ratio phi and
    temperature T: (T, p, Y[K])."""
    Y = _mass_fractions(mech, _moles_burnt(mech, fuel, np.array([phi])))
    return T, p, Y[:, 0].copy()


def flow_times(N: int, seed: int, log_taylor=(-4.0, -2.0), log_kolmogorov=(-5.0, -3.0)):
    """Per-cell turbulence time scales a flow solver would hand to the
    chemistry closure: Taylor time 10^U(log_taylor) s and Kolmogorov time
    10^U(log_kolmogorov) s (magnitudes of a laboratory jet flame's resolved
    and sub-grid scales).  Returns (tau_taylor[N], tau_kolmogorov[N])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tT = 10.0 ** rng.uniform(log_taylor[0], log_taylor[1], N)
    tK = 10.0 ** rng.uniform(log_kolmogorov[0], log_kolmogorov[1], N)
    return tT, tK
