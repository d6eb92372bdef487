"""MI355X-native per-cell chemistry step (arXiv 2312.05800, Sec. 2-3).

The computation lives in libchemstep.so (hand-written HIP kernels for gfx950,
C ABI in include/chemstep.h); this package is its thin Python binding.
"""
from .binding import (ChemError, Graph, Mechanism, chem_autotune, chem_get_tuning, chem_rates,
                      chem_set_tuning, chem_step, chem_step_graph, chem_step_sets,
                      chem_step_sets_device, set_table_device,
                      chem_step_sets_graph, lib,
                      status_name, LIB_PATH, measure_peaks, pasr_scale, profile_enable,
                      profile_read, sample_states)
from .ann import AnnModel

CELL_STATUS = {0: "OK", 1: "MAX_STEPS", 2: "H_UNDERFLOW", 3: "NONFINITE", 4: "SINGULAR"}

__all__ = ["ChemError", "Graph", "Mechanism", "chem_autotune", "chem_get_tuning", "chem_rates",
           "chem_set_tuning", "chem_step", "chem_step_graph", "chem_step_sets",
           "chem_step_sets_graph", "chem_step_sets_device", "set_table_device", "lib",
           "status_name", "LIB_PATH", "CELL_STATUS", "AnnModel", "profile_enable",
           "profile_read", "measure_peaks", "pasr_scale", "sample_states"]
