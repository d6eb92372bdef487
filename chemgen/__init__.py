"""Seeded synthetic inputs for the per-cell chemistry step.

This package builds *inputs only*: reaction mechanisms (species, elements,
NASA-7 thermo coefficients, Arrhenius parameters) and cell states
(T, p, Y_k in SoA layout).  It holds none of the step's arithmetic (no rates,
no Jacobian, no integrator, no network); both the CPU oracle and the HIP
library consume what it produces.

The paper's own inputs (DRM19 and 1-D flamelet data, Sec. 3.1) are not
available, so these seeded generators stand in for them with the same shape:
a few tens of species over C/H/O/N, a hundred-odd reversible elementary
reactions, and stratified CH4/air (or H2/air) states at 1 atm.
"""
from .mech import Mech, make_mechanism, MECH_CONFIGS, isomer_mechanism
from .states import (make_states, perturb_states, STATE_CONFIGS, multiset_workload,
                     element_matrix, hfrd_randoms, air_state, burnt_state, flow_times)

__all__ = ["Mech", "make_mechanism", "MECH_CONFIGS", "isomer_mechanism",
           "make_states", "perturb_states", "STATE_CONFIGS", "multiset_workload",
           "element_matrix", "hfrd_randoms", "air_state", "burnt_state", "flow_times"]
