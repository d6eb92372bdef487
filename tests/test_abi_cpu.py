"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every function include/chemstep.h declares; status strings."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*"
                                r"([a-z][a-z0-9_]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_declared_symbols():
    import paper_2312_05800_amd as P
    L = P.lib()
    names = _declared()
    assert "chem_step" in names and "chem_rates" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    import paper_2312_05800_amd as P
    assert P.status_name(0) == "CHEM_OK"
    assert P.status_name(1) == "CHEM_EINVAL"
    assert P.status_name(6) == "CHEM_EUNSUPPORTED"


def test_invalid_mechanism_rejected_on_host():
    """Validation runs before any device call, so it works without a GPU."""
    import numpy as np
    import chemgen
    import paper_2312_05800_amd as P
    m = chemgen.make_mechanism("h2")
    bad = chemgen.Mech(**{**m.__dict__, "rnu": m.rnu.copy()})
    bad.rnu[0, 2] = 2 if bad.rnu[0, 2] == 1 else 1  # breaks the element balance of reaction 0
    with pytest.raises(P.ChemError) as e:
        P.Mechanism(bad)
    assert e.value.status == 4
    big = chemgen.Mech(**{**m.__dict__, "W": np.zeros(70), "nasa": np.zeros((70, 17)),
                          "comp": np.zeros((70, 3), dtype=np.int32)})
    with pytest.raises(P.ChemError) as e:
        P.Mechanism(big)
    assert e.value.status == 6


def test_tuning_and_graph_arguments_rejected_on_host():
    """Null handles are rejected before any device call (no GPU needed);
    destroying a null graph is a no-op."""
    import ctypes as C
    import paper_2312_05800_amd as P
    L = P.lib()
    assert L.chem_set_tuning(None, None) == 1
    assert L.chem_get_tuning(None, None) == 1
    assert L.chem_graph_launch(None, None) == 1
    L.chem_graph_destroy(None)
    h = C.c_void_p()
    assert L.chem_autotune(None, P.binding.Batch(1, 1), 1e-6, None, None, None, None, None,
                           None) == 1
    assert L.chem_step_graph_create(None, P.binding.Batch(1, 1), 1e-6, None, None, None, None,
                                    None, None, None, None, None, C.byref(h)) == 1
    assert L.ann_step_graph_create(None, None, P.binding.Batch(1, 1), 1e-6, None, None, None,
                                   None, None, None, None, None, None, C.byref(h)) == 1
    assert not h.value


def test_audit_arguments_rejected_on_host():
    """ann_step rejects an audit fraction outside [0, 1], or above 0 without
    an audit array, before anything else (no model or GPU needed)."""
    import ctypes as C
    import paper_2312_05800_amd as P
    from paper_2312_05800_amd.ann import StepOptsANN
    L = P.lib()
    for f, arr in ((1.5, 1), (-0.1, 1), (float("nan"), 1), (0.25, None)):
        o = StepOptsANN(1e-6, 0.05, 1, f, arr)
        assert L.ann_step(None, None, P.binding.Batch(1, 1), 1e-5, None, None, None, None, None,
                          None, C.byref(o), None, None) == 1
        assert b"audit_fraction" in L.chem_last_error()
    o = StepOptsANN(1e-6, 0.05, 1, 0.0, None)
    assert L.ann_step(None, None, P.binding.Batch(1, 1), 1e-5, None, None, None, None, None,
                      None, C.byref(o), None, None) == 1
    assert b"null model" in L.chem_last_error()


def test_binding_rejects_bad_1d_arrays():
    """The binding checks every 1-D array for shape, contiguity and length
    before calling the library (no GPU needed: the checks raise first)."""
    import torch
    from paper_2312_05800_amd.binding import _vec

    class FakeCuda(torch.Tensor):
        @property
        def is_cuda(self):
            return True
    short = torch.zeros(4, dtype=torch.float64).as_subclass(FakeCuda)
    with pytest.raises(ValueError):
        _vec(short, 5, "T", torch.float64)
    strided = torch.zeros(10, dtype=torch.float64)[::2].as_subclass(FakeCuda)
    with pytest.raises(ValueError):
        _vec(strided, 5, "T", torch.float64)
    twod = torch.zeros((2, 3), dtype=torch.float64).as_subclass(FakeCuda)
    with pytest.raises(ValueError):
        _vec(twod, 2, "T", torch.float64)
    assert _vec(None, 5, "T") is None
    with pytest.raises(TypeError):
        _vec(torch.zeros(5, dtype=torch.float64), 5, "T")


def test_pasr_arguments_rejected_on_host():
    """chem_pasr_scale rejects a null handle, a bad batch and eta outside
    [0, 1] before any device call; an empty batch needs no arrays.  The
    mechanism handle is made on the host alone (its upload needs the GPU), so
    only the null-handle case runs here."""
    import paper_2312_05800_amd as P
    L = P.lib()
    B = P.binding.Batch
    assert L.chem_pasr_scale(None, B(1, 1), *([None] * 6), None, None, None, None) == 1
    assert L.chem_pasr_scale(None, B(0, 0), *([None] * 6), None, None, None, None) == 1
