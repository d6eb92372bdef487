"""Constructed chemical-equilibrium states -- TEST INFRASTRUCTURE ONLY.

Pick T, p and element potentials lambda_e; set the mole fractions
X_k = (p_ref/p) exp(-g_k/RT + sum_e lambda_e a_ek).  For every reaction the
Gibbs energy change sum_k nu_k (g_k/RT + ln(X_k p/p_ref)) = sum_e lambda_e
sum_k nu_k a_ek vanishes by element balance, so every forward and reverse rate
of progress are equal.  A common shift of all lambda_e is found by bisection
(sum_k X_k grows monotonically with it) so that the X_k sum to one.
"""
from __future__ import annotations

import numpy as np

from . import OracleMech, thermo, PREF


def equilibrium_state(om: OracleMech, T: float, p: float, lam):
    m = om.mech
    cp, hRT, sR = thermo(om, T)
    gRT = hRT - sR
    a = m.comp.astype(np.float64)            # [K, E]
    lam = np.asarray(lam, dtype=np.float64)
    base = -gRT + a @ lam + np.log(PREF / p)
    natoms = a.sum(axis=1)

    def total(delta):
        return np.exp(base + delta * natoms).sum()

    lo, hi = -200.0, 200.0
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if total(mid) > 1.0:
            hi = mid
        else:
            lo = mid
    X = np.exp(base + 0.5 * (lo + hi) * natoms)
    X /= X.sum()
    Y = X * m.W
    return Y / Y.sum()
