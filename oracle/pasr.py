"""Partially stirred reactor (PaSR) scaling of the chemistry source (Sec. 4.1)
-- TEST INFRASTRUCTURE ONLY.

Plain NumPy (FP64) statement of the turbulence-chemistry closure the paper
couples to the network, used to check the GPU kernel.  The filtered source of
every species is the reactor's rate times the reacting fraction of the cell,

    kappa = tau_c / (tau_c + tau_mix),

where the mixing time is the geometric mean of the Taylor and Kolmogorov
times the flow solver supplies, tau_mix = sqrt(tau_T tau_K), and the chemical
time is set by the slowest formation rate of the species.

Readings where the paper gives no formula:

* the formation rate of species k is the step's mass rate RR_k (kg/m^3/s);
  its time is tau_k = rho Y_k / |RR_k| (concentration over the rate of change
  of concentration; the molar mass cancels), with Y_k (clipped at 0) and rho
  (ideal gas) those of the state after the step;
* only species that take part in the step count: |RR_k| >= eta max_j |RR_j|
  and RR_k != 0, eta = 1e-3 by default.  Without it a nearly inert species
  (N2, whose rate is about 1e-5 of the largest on the benchmark states) would
  set tau_c to hours;
* tau_c is the largest tau_k of those species (the slowest); a cell with no
  such species (all rates zero) has tau_c = inf and kappa = 1; kappa = 1 also
  when tau_c + tau_mix = 0.
"""
from __future__ import annotations

import numpy as np

from . import RGAS

ETA = 1e-3


def density(mech, T, p, Y):
    """Ideal-gas density p / (R T sum_k Y_k / W_k), kg/m^3, for [K, N] Y."""
    Y = np.asarray(Y, dtype=np.float64)
    s = (Y / np.asarray(mech.W)[:, None]).sum(axis=0)
    return np.asarray(p, dtype=np.float64) / (RGAS * np.asarray(T, dtype=np.float64) * s)


def chemical_time(mech, T, p, Y, RR, eta=ETA):
    """tau_c of every cell (inf where no species reacts)."""
    Y = np.asarray(Y, dtype=np.float64)
    a = np.abs(np.asarray(RR, dtype=np.float64))
    rho = density(mech, T, p, Y)
    amax = a.max(axis=0)
    active = (a > 0.0) & (a >= eta * amax[None, :])
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = np.where(active, rho[None, :] * np.maximum(Y, 0.0) / np.where(active, a, 1.0),
                       -np.inf)
    tc = tau.max(axis=0)
    return np.where(active.any(axis=0), tc, np.inf)


def mixing_time(tau_taylor, tau_kolmogorov):
    """Geometric mean of the two flow time scales."""
    return np.sqrt(np.asarray(tau_taylor, dtype=np.float64) *
                   np.asarray(tau_kolmogorov, dtype=np.float64))


def kappa(tau_c, tau_mix):
    """Reacting fraction tau_c / (tau_c + tau_mix) with the limits above."""
    tau_c = np.asarray(tau_c, dtype=np.float64)
    tau_mix = np.asarray(tau_mix, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        k = tau_c / (tau_c + tau_mix)
    k = np.where(tau_c + tau_mix == 0.0, 1.0, k)
    return np.where(np.isposinf(tau_c), 1.0, k)


def scale(mech, T, p, Y, RR, tau_taylor, tau_kolmogorov, eta=ETA):
    """The whole closure: returns (kappa, tau_c, kappa * RR)."""
    tc = chemical_time(mech, T, p, Y, RR, eta)
    k = kappa(tc, mixing_time(tau_taylor, tau_kolmogorov))
    return k, tc, k[None, :] * np.asarray(RR, dtype=np.float64)
