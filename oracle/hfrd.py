"""Random-data sampler of the training set (Sec. 3.1) -- TEST INFRASTRUCTURE ONLY.

Plain NumPy (FP64) statement of how the paper widens its flamelet samples
into a training set, used to check the GPU sampler:

* every seed composition is perturbed by Eqs. (Trand), (Prand), (N2rand) and
  (Yrand): T' = T + alpha c_T (T_max - T_min), p' = p + beta c_p (p_max -
  p_min), y'_N2 = y_N2 + alpha c_N2 (y_N2,max - y_N2,min) and
  y'_j = y_j^(1 + gamma c_j) for every other species, with alpha = 0.125,
  beta = 10, gamma = 0.1 and c uniform in [-1, 1]; max and min are taken
  over the seed set;
* the species other than N2 are then rescaled so that all mass fractions sum
  to one (their sum becomes 1 - y'_N2);
* further samples lie on the straight line between the equilibrium state of
  the leanest mixture (phi = 0.45) and ambient air, for the lean reactants
  that large eddies mix into hot products;
* a sample is kept if T >= 500 K and its molar H/C ratio, O/N ratio and
  equivalence ratio lie inside the limits of Table 1.

Readings where the paper is silent: each c is an independent draw (one per
quantity, one per species); a species with y_j <= 0 stays at 0; the
equivalence ratio of a C/H/O/N composition is phi = (2 n_C + n_H / 2) / n_O
from the element moles (the oxygen that burning all C to CO2 and all H to
H2O needs over the oxygen present; it equals the phi of the unburnt fuel/air
mixture and is conserved by reactions); the two ends of the mixing line and
the mixing fraction s of each mixing sample are inputs.  The random numbers
themselves are drawn by the caller (chemgen) and passed in.
"""
from __future__ import annotations

import numpy as np

ALPHA, BETA, GAMMA = 0.125, 10.0, 0.1
T_KEEP = 500.0
HC = (2.65, 4.67)
ON = (0.254, 0.32)
PHI = (0.20, 1.15)


def seed_ranges(T, p, Y, n2):
    """(T_min, T_max, p_min, p_max, y_N2 min, y_N2 max) over the seed set."""
    return (float(np.min(T)), float(np.max(T)), float(np.min(p)), float(np.max(p)),
            float(np.min(Y[n2])), float(np.max(Y[n2])))


def perturb(T, p, Y, c, n2, ranges, alpha=ALPHA, beta=BETA, gamma=GAMMA):
    """Eqs. (Trand)-(Yrand) and the renormalisation, for every seed.
    c: [K + 3, N] uniform in [-1, 1] (rows: T, p, N2, then species j at row
    3 + j; the row of N2 itself is unused).  Returns (T', p', Y')."""
    T = np.asarray(T, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    K, N = Y.shape
    Tmin, Tmax, pmin, pmax, nmin, nmax = ranges
    Tn = T + alpha * c[0] * (Tmax - Tmin)
    pn = p + beta * c[1] * (pmax - pmin)
    Yn = np.zeros_like(Y)
    yn2 = Y[n2] + alpha * c[2] * (nmax - nmin)
    for j in range(K):
        if j == n2:
            continue
        pos = Y[j] > 0.0
        Yn[j, pos] = np.power(Y[j, pos], 1.0 + gamma * c[3 + j, pos])
    others = np.ones(K, dtype=bool)
    others[n2] = False
    s = Yn[others].sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = (1.0 - yn2) / s
    Yn[others] *= scale[None, :]
    Yn[n2] = yn2
    return Tn, pn, Yn


def mix(end_eq, end_air, s):
    """States on the line from the equilibrium end (s = 0) to air (s = 1):
    each end is (T, p, Y[K]); returns (T, p, Y[K, N])."""
    s = np.asarray(s, dtype=np.float64)
    T = (1.0 - s) * end_eq[0] + s * end_air[0]
    p = (1.0 - s) * end_eq[1] + s * end_air[1]
    Y = (1.0 - s)[None, :] * np.asarray(end_eq[2])[:, None] + \
        s[None, :] * np.asarray(end_air[2])[:, None]
    return T, p, Y


def element_moles(mech, Y):
    """Moles of each element per kg of mixture: [E, N]."""
    Y = np.asarray(Y, dtype=np.float64)
    n = np.zeros((mech.E, Y.shape[1]))
    for e in range(mech.E):
        for k in range(mech.K):
            if mech.comp[k, e]:
                n[e] += mech.comp[k, e] * Y[k] / mech.W[k]
    return n


def ratios(mech, Y):
    """(H/C, O/N, phi) of every composition (NaN where undefined)."""
    n = element_moles(mech, Y)
    eC, eH, eO, eN = (mech.elements.index(x) for x in ("C", "H", "O", "N"))
    with np.errstate(divide="ignore", invalid="ignore"):
        hc = n[eH] / n[eC]
        on = n[eO] / n[eN]
        phi = (2.0 * n[eC] + 0.5 * n[eH]) / n[eO]
    return hc, on, phi


def keep(mech, T, Y, T_min=T_KEEP, hc=HC, on=ON, phi=PHI, n2=None):
    """Table 1 and the temperature threshold; a sample with a non-finite
    value, a negative mass fraction or a N2 fraction outside [0, 1) is
    dropped."""
    r_hc, r_on, r_phi = ratios(mech, Y)
    ok = np.isfinite(T) & (T >= T_min)
    ok &= np.all(np.isfinite(Y), axis=0) & np.all(Y >= 0.0, axis=0)
    if n2 is not None:
        ok &= (Y[n2] >= 0.0) & (Y[n2] < 1.0)
    for v, (lo, hi) in ((r_hc, hc), (r_on, on), (r_phi, phi)):
        ok &= np.isfinite(v) & (v >= lo) & (v <= hi)
    return ok


def sample(mech, T, p, Y, c, s, end_eq, end_air, n2, alpha=ALPHA, beta=BETA, gamma=GAMMA):
    """The whole sampler: seed i is perturbed when s[i] < 0, replaced by the
    mixing-line state at s[i] otherwise.  Returns (T', p', Y', keep)."""
    ranges = seed_ranges(T, p, Y, n2)
    Tn, pn, Yn = perturb(T, p, Y, c, n2, ranges, alpha, beta, gamma)
    s = np.asarray(s, dtype=np.float64)
    m = s >= 0.0
    if m.any():
        Tm, pm, Ym = mix(end_eq, end_air, s[m])
        Tn[m], pn[m], Yn[:, m] = Tm, pm, Ym
    return Tn, pn, Yn, keep(mech, Tn, Yn, n2=n2)
