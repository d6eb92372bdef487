"""Seeded synthetic reaction mechanisms.

A mechanism is a set of species over a few elements, NASA-7 thermodynamic
coefficients for each species, and reversible elementary reactions with
modified-Arrhenius forward parameters.  The paper integrates DRM19 (20
species, 85 reactions; Sec. 3.1), which is not available here; these seeded
mechanisms stand in for it:

* ``"h2"``  : 9 species (H2, O2, H2O, H, O, OH, HO2, H2O2, N2), elements
  H/O/N, 20 reactions.
* ``"ch4"`` : 30 species over C/H/O/N, 150 reactions.

Construction (all seeded, numpy PCG64):

* Reactions: every element-balanced pairing of two "sides", a side being one
  molecule, two of one molecule, or two distinct molecules, with no species on
  both sides and at least one open-shell species (radical) taking part (a
  molecule-only exchange is not an elementary step).  Candidates are shuffled;
  first every reactive species is covered by one reaction, then the list is
  filled up to R.  Each reaction is oriented so that it is exothermic forward at
  298 K (judged on the formation enthalpies below), which keeps reverse
  activation energies non-negative.
* Arrhenius: A log-uniform in CGS units ((cm^3/mol)^(order-1)/s), converted to
  SI by (1e-6)^(order-1); b uniform; Ea uniform (J/mol).
* Thermo: formation enthalpy and standard entropy at 298.15 K start from rough
  textbook magnitudes for each named species and are perturbed per seed
  (element reference species H2, O2, N2 keep h_f = 0).  c_p/R follows a
  saturating curve from a 300 K value to a 3000 K value fixed by the atom count
  (2.5/3.5/4+0.5(n-3) and 2.5/4.5/3n-2 for mono-, di- and polyatomic), scaled
  by U(0.9, 1.1) with a seeded knee temperature.  Its NASA-7 fit (a1..a5) is a
  least-squares fit on [200, T_mid] K and [T_mid, 3500] K; a1 of the high range
  is shifted for c_p continuity at T_mid, a6/a7 of the low range reproduce
  h_f and s at 298.15 K, and a6/a7 of the high range make h and s continuous
  at T_mid.  T_mid = 1000 K for every species, unless the configuration has
  ``tmid_range = (lo, hi)``: then each species' T_mid is drawn uniformly from
  it by a generator of its own (seed + 7919), leaving the other draws as they
  are.

NASA array layout per species (17 doubles): T_low, T_mid, T_high,
a1..a7 of the low range, a1..a7 of the high range.
"""
from __future__ import annotations

import dataclasses
import itertools
import json
from typing import Dict, List, Sequence

import numpy as np

R_GAS = 8.314462618  # J/(mol K)
ATOMIC_WEIGHT = {"H": 1.008e-3, "C": 12.011e-3, "N": 14.007e-3, "O": 15.999e-3}  # kg/mol

# name: (composition, open-shell?, h_f(298) kJ/mol, s(298) J/(mol K)) -- rough magnitudes
_SPECIES_TABLE: Dict[str, tuple] = {
    "H2":    ({"H": 2}, False, 0.0, 130.7),
    "O2":    ({"O": 2}, False, 0.0, 205.2),
    "H2O":   ({"H": 2, "O": 1}, False, -241.8, 188.8),
    "H":     ({"H": 1}, True, 218.0, 114.7),
    "O":     ({"O": 1}, True, 249.2, 161.1),
    "OH":    ({"H": 1, "O": 1}, True, 39.0, 183.7),
    "HO2":   ({"H": 1, "O": 2}, True, 12.0, 229.0),
    "H2O2":  ({"H": 2, "O": 2}, False, -136.1, 232.7),
    "CH4":   ({"C": 1, "H": 4}, False, -74.9, 186.3),
    "CH3":   ({"C": 1, "H": 3}, True, 146.0, 194.2),
    "CH2":   ({"C": 1, "H": 2}, True, 390.0, 194.9),
    "CH":    ({"C": 1, "H": 1}, True, 595.0, 183.0),
    "CH2O":  ({"C": 1, "H": 2, "O": 1}, False, -116.0, 218.8),
    "HCO":   ({"C": 1, "H": 1, "O": 1}, True, 42.0, 224.7),
    "CH3O":  ({"C": 1, "H": 3, "O": 1}, True, 17.0, 228.5),
    "CH2OH": ({"C": 1, "H": 3, "O": 1}, True, -17.0, 244.0),
    "CH3OH": ({"C": 1, "H": 4, "O": 1}, False, -201.0, 239.9),
    "CO":    ({"C": 1, "O": 1}, False, -110.5, 197.7),
    "CO2":   ({"C": 1, "O": 2}, False, -393.5, 213.8),
    "C2H6":  ({"C": 2, "H": 6}, False, -84.0, 229.2),
    "C2H5":  ({"C": 2, "H": 5}, True, 119.0, 247.0),
    "C2H4":  ({"C": 2, "H": 4}, False, 52.5, 219.3),
    "C2H3":  ({"C": 2, "H": 3}, True, 300.0, 233.6),
    "C2H2":  ({"C": 2, "H": 2}, False, 227.0, 200.9),
    "N2":    ({"N": 2}, False, 0.0, 191.6),
    "N":     ({"N": 1}, True, 473.0, 153.3),
    "NO":    ({"N": 1, "O": 1}, True, 90.3, 210.8),
    "NO2":   ({"N": 1, "O": 2}, True, 33.1, 240.1),
    "N2O":   ({"N": 2, "O": 1}, False, 82.1, 219.9),
    "NH":    ({"N": 1, "H": 1}, True, 376.0, 181.2),
    "C":     ({"C": 1}, True, 716.7, 158.1),
    "C2H":   ({"C": 2, "H": 1}, True, 568.0, 207.4),
    "CH2CO": ({"C": 2, "H": 2, "O": 1}, False, -47.7, 241.8),
    "HCCO":  ({"C": 2, "H": 1, "O": 1}, True, 177.0, 255.0),
    "CH3CHO": ({"C": 2, "H": 4, "O": 1}, False, -166.2, 263.8),
    "C3H8":  ({"C": 3, "H": 8}, False, -104.7, 270.3),
    "C3H6":  ({"C": 3, "H": 6}, False, 20.0, 266.6),
    "NH2":   ({"N": 1, "H": 2}, True, 190.0, 194.7),
    "NH3":   ({"N": 1, "H": 3}, False, -45.9, 192.8),
    "HNO":   ({"H": 1, "N": 1, "O": 1}, True, 99.6, 220.7),
    "HCN":   ({"H": 1, "C": 1, "N": 1}, False, 135.1, 201.8),
    "CN":    ({"C": 1, "N": 1}, True, 438.7, 202.6),
    "NCO":   ({"N": 1, "C": 1, "O": 1}, True, 131.8, 232.6),
    "HNCO":  ({"H": 1, "N": 1, "C": 1, "O": 1}, False, -101.7, 238.0),
}
_REFERENCE_SPECIES = ("H2", "O2", "N2")

H2_SPECIES = ["H2", "O2", "H2O", "H", "O", "OH", "HO2", "H2O2", "N2"]
CH4_SPECIES = ["H2", "O2", "H2O", "H", "O", "OH", "HO2", "H2O2", "CH4", "CH3", "CH2", "CH",
               "CH2O", "HCO", "CH3O", "CH2OH", "CH3OH", "CO", "CO2", "C2H6", "C2H5", "C2H4",
               "C2H3", "C2H2", "N2", "N", "NO", "NO2", "N2O", "NH"]
WIDE_SPECIES = CH4_SPECIES + ["C", "C2H", "CH2CO", "HCCO", "CH3CHO", "C3H8", "C3H6", "NH2",
                              "NH3", "HNO", "HCN", "CN", "NCO", "HNCO"]

MECH_CONFIGS = {
    # 9 species / 20 reactions over H, O, N (small correctness case)
    "h2": dict(species=H2_SPECIES, elements=["H", "O", "N"], n_reactions=20, seed=1001,
               logA=(8.0, 14.0), b=(-1.0, 1.0), Ea=(0.0, 150e3)),
    # 30 species / 150 reactions over C, H, O, N (the full-size case)
    "ch4": dict(species=CH4_SPECIES, elements=["C", "H", "O", "N"], n_reactions=150, seed=2002,
                logA=(8.0, 14.0), b=(-1.0, 1.0), Ea=(0.0, 150e3)),
    # 44 species / 220 reactions: above 32 species, so every kernel takes its
    # widest form (a 64-lane group per cell in the integrator)
    "wide": dict(species=WIDE_SPECIES, elements=["C", "H", "O", "N"], n_reactions=220,
                 seed=3003, logA=(8.0, 14.0), b=(-1.0, 1.0), Ea=(0.0, 150e3)),
    # mild kinetics on the small species set, for explicit brute-force checks
    "h2_mild": dict(species=H2_SPECIES, elements=["H", "O", "N"], n_reactions=20, seed=1003,
                    logA=(8.0, 10.0), b=(-1.0, 1.0), Ea=(40e3, 150e3)),
}


@dataclasses.dataclass
class Mech:
    name: str
    species: List[str]
    elements: List[str]
    comp: np.ndarray      # int32 [K, E] atoms of element e in species k
    W: np.ndarray         # f64 [K] kg/mol (sum of atomic weights)
    awt: np.ndarray       # f64 [E] kg/mol
    nasa: np.ndarray      # f64 [K, 17]
    rsp: np.ndarray       # int32 [R, 4] reactant0, reactant1, product0, product1 (-1 = none)
    rnu: np.ndarray       # int32 [R, 4] stoichiometric coefficients of those slots
    A: np.ndarray         # f64 [R] SI: (m^3/mol)^(order-1)/s
    b: np.ndarray         # f64 [R]
    Ea: np.ndarray        # f64 [R] J/mol
    hf298: np.ndarray     # f64 [K] J/mol, the formation enthalpies the thermo was built from
    s298: np.ndarray      # f64 [K] J/(mol K)
    radical: np.ndarray   # bool [K]

    @property
    def K(self) -> int:
        return len(self.species)

    @property
    def R(self) -> int:
        return int(self.rsp.shape[0])

    @property
    def E(self) -> int:
        return len(self.elements)

    def index(self, name: str) -> int:
        return self.species.index(name)

    def reactive_mask(self) -> np.ndarray:
        m = np.zeros(self.K, dtype=bool)
        for r in range(self.R):
            for s in range(4):
                if self.rsp[r, s] >= 0:
                    m[self.rsp[r, s]] = True
        return m

    def to_json(self) -> str:
        d = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            d[f.name] = v.tolist() if isinstance(v, np.ndarray) else v
        return json.dumps(d)

    @staticmethod
    def from_json(s: str) -> "Mech":
        d = json.loads(s)
        ints = {"comp", "rsp", "rnu"}
        out = {}
        for f in dataclasses.fields(Mech):
            v = d[f.name]
            if f.name in ints:
                v = np.asarray(v, dtype=np.int32)
            elif f.name == "radical":
                v = np.asarray(v, dtype=bool)
            elif isinstance(v, list) and f.name not in ("species", "elements"):
                v = np.asarray(v, dtype=np.float64)
            out[f.name] = v
        return Mech(**out)


def _cp_curve(T, lo, hi, theta, scale):
    Tc = np.maximum(T, 300.0)
    s = (1.0 - np.exp(-(Tc - 300.0) / theta)) / (1.0 - np.exp(-2700.0 / theta))
    return scale * (lo + (hi - lo) * s)


def _fit_range(T, cp):
    # least squares in a scaled variable, converted back to powers of T
    x = T / 1000.0
    V = np.vander(x, 5, increasing=True)
    c, *_ = np.linalg.lstsq(V, cp, rcond=None)
    return c / (1000.0 ** np.arange(5))


def _h_poly(a, T):  # H/R without the a6 constant
    return a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4 + a[4] * T**5 / 5


def _s_poly(a, T):  # S/R without the a7 constant
    return a[0] * np.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4


def _make_thermo(species, comp_counts, rng, tmid=None):
    K = len(species)
    nasa = np.zeros((K, 17))
    hf = np.zeros(K)
    s298 = np.zeros(K)
    for k, name in enumerate(species):
        _, _, hf0, s0 = _SPECIES_TABLE[name]
        n_at = comp_counts[k]
        if name in _REFERENCE_SPECIES:
            hf[k] = 0.0
            rng.uniform()  # keep the stream aligned across species
        else:
            hf[k] = (hf0 + rng.uniform(-10.0, 10.0)) * 1e3
        s298[k] = s0 * rng.uniform(0.98, 1.02)
        if n_at == 1:
            lo, hi = 2.5, 2.5
        elif n_at == 2:
            lo, hi = 3.5, 4.5
        else:
            lo, hi = 4.0 + 0.5 * (n_at - 3), 3.0 * n_at - 2.0
        scale = 1.0 if n_at == 1 else rng.uniform(0.9, 1.1)
        theta = rng.uniform(500.0, 1500.0)
        tm = 1000.0 if tmid is None else float(tmid[k])
        Tl = np.linspace(200.0, tm, 81)
        Th = np.linspace(tm, 3500.0, 126)
        al = _fit_range(Tl, _cp_curve(Tl, lo, hi, theta, scale))
        ah = _fit_range(Th, _cp_curve(Th, lo, hi, theta, scale))
        cpl = sum(al[i] * tm**i for i in range(5))
        cph = sum(ah[i] * tm**i for i in range(5))
        ah[0] += cpl - cph
        T0 = 298.15
        a6l = hf[k] / R_GAS - _h_poly(al, T0)
        a7l = s298[k] / R_GAS - _s_poly(al, T0)
        a6h = (_h_poly(al, tm) + a6l) - _h_poly(ah, tm)
        a7h = (_s_poly(al, tm) + a7l) - _s_poly(ah, tm)
        nasa[k, 0:3] = (200.0, tm, 3500.0)
        nasa[k, 3:8] = al
        nasa[k, 8] = a6l
        nasa[k, 9] = a7l
        nasa[k, 10:15] = ah
        nasa[k, 15] = a6h
        nasa[k, 16] = a7h
    return nasa, hf, s298


def _enumerate_candidates(comp, radical):
    K = comp.shape[0]
    sides = [((i, 1),) for i in range(K)] + [((i, 2),) for i in range(K)]
    sides += [((i, 1), (j, 1)) for i, j in itertools.combinations(range(K), 2)]
    groups: Dict[tuple, list] = {}
    for s in sides:
        ev = tuple(int(v) for v in sum(nu * comp[i] for i, nu in s))
        groups.setdefault(ev, []).append(s)
    cands = []
    for ev in sorted(groups):
        g = groups[ev]
        for a, b in itertools.combinations(g, 2):
            sa = {i for i, _ in a}
            sb = {i for i, _ in b}
            if sa & sb:
                continue
            if not any(radical[i] for i in sa | sb):
                continue
            cands.append((a, b))
    return cands


def make_mechanism(cfg: str | dict, seed: int | None = None) -> Mech:
    """Build the seeded mechanism named ``cfg`` (a key of MECH_CONFIGS) or
    described by a dict with the same keys."""
    c = dict(MECH_CONFIGS[cfg]) if isinstance(cfg, str) else dict(cfg)
    name = cfg if isinstance(cfg, str) else c.get("name", "custom")
    if seed is None:
        seed = c["seed"]
    rng = np.random.Generator(np.random.PCG64(seed))
    species = list(c["species"])
    elements = list(c["elements"])
    K, E = len(species), len(elements)
    comp = np.zeros((K, E), dtype=np.int32)
    radical = np.zeros(K, dtype=bool)
    for k, s in enumerate(species):
        cdict, rad, _, _ = _SPECIES_TABLE[s]
        radical[k] = rad
        for el, n in cdict.items():
            comp[k, elements.index(el)] = n
    awt = np.array([ATOMIC_WEIGHT[e] for e in elements])
    W = np.zeros(K)
    for k in range(K):  # summed in element order so that sum_k W_k wdot_k cancels to rounding
        w = 0.0
        for e in range(E):
            w += comp[k, e] * awt[e]
        W[k] = w
    tmid = None
    if c.get("tmid_range") is not None:
        trng = np.random.Generator(np.random.PCG64(seed + 7919))
        tmid = trng.uniform(*c["tmid_range"], size=K)
    nasa, hf, s298 = _make_thermo(species, comp.sum(axis=1), rng, tmid)

    cands = _enumerate_candidates(comp, radical)
    order = rng.permutation(len(cands))
    shuffled = [cands[i] for i in order]
    R = int(c["n_reactions"])
    chosen: List[int] = []
    covered = np.zeros(K, dtype=bool)
    for k in rng.permutation(K):
        if covered[k]:
            continue
        for idx, (a, b) in enumerate(shuffled):
            sp = {i for i, _ in a} | {i for i, _ in b}
            if k in sp and idx not in chosen:
                chosen.append(idx)
                for i in sp:
                    covered[i] = True
                break
    for idx in range(len(shuffled)):
        if len(chosen) >= R:
            break
        if idx not in chosen:
            chosen.append(idx)
    if len(chosen) > R:
        raise ValueError("R too small to cover every reactive species")
    rsp = -np.ones((R, 4), dtype=np.int32)
    rnu = np.zeros((R, 4), dtype=np.int32)
    for r, idx in enumerate(chosen):
        a, b = shuffled[idx]
        dh = sum(nu * hf[i] for i, nu in b) - sum(nu * hf[i] for i, nu in a)
        if dh > 0:  # make the forward direction exothermic
            a, b = b, a
        for s, (i, nu) in enumerate(a):
            rsp[r, s], rnu[r, s] = i, nu
        for s, (i, nu) in enumerate(b):
            rsp[r, 2 + s], rnu[r, 2 + s] = i, nu
    lo, hi = c["logA"]
    A_cgs = 10.0 ** rng.uniform(lo, hi, R)
    order_r = rnu[:, 0] + rnu[:, 1]
    A = A_cgs * (1e-6) ** (order_r - 1)
    b = rng.uniform(c["b"][0], c["b"][1], R)
    Ea = rng.uniform(c["Ea"][0], c["Ea"][1], R)
    return Mech(name=name, species=species, elements=elements, comp=comp, W=W, awt=awt,
                nasa=nasa, rsp=rsp, rnu=rnu, A=A, b=b, Ea=Ea, hf298=hf, s298=s298,
                radical=radical)


def isomer_mechanism(k: float = 1e5) -> Mech:
    """A <=> B between two isomers with identical thermo, plus inert N2.

    With equal thermo the equilibrium constant is 1 and k_r = k_f = k; with
    b = Ea = 0 the rate constant is T independent, and with equal molar
    masses and zero reaction enthalpy T and rho stay constant, so
    Y_A(t) = s/2 + (Y_A(0) - s/2) exp(-2 k t) with s = Y_A + Y_B.
    """
    base = make_mechanism("ch4")
    i1, i2, n2 = base.index("CH3O"), base.index("CH2OH"), base.index("N2")
    species = ["CH3O", "CH2OH", "N2"]
    comp = base.comp[[i1, i2, n2]].copy()
    W = base.W[[i1, i2, n2]].copy()
    nasa = base.nasa[[i1, i1, n2]].copy()  # identical thermo for the isomers
    hf = base.hf298[[i1, i1, n2]].copy()
    s298 = base.s298[[i1, i1, n2]].copy()
    rsp = np.array([[0, -1, 1, -1]], dtype=np.int32)
    rnu = np.array([[1, 0, 1, 0]], dtype=np.int32)
    return Mech(name="isomer", species=species, elements=list(base.elements), comp=comp, W=W,
                awt=base.awt.copy(), nasa=nasa, rsp=rsp, rnu=rnu, A=np.array([k]),
                b=np.zeros(1), Ea=np.zeros(1), hf298=hf, s298=s298,
                radical=np.array([True, True, False]))
