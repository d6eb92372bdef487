"""ctypes binding of libchemstep.so (include/chemstep.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Arrays are torch CUDA tensors (device memory); the calls are
enqueued on torch's current stream.  If the library has not been built the
first call raises -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchemstep.so")

_lock = threading.Lock()
_lib = None

_P = C.c_void_p


class ChemError(RuntimeError):
    def __init__(self, fn, status, detail):
        super().__init__(f"{fn} failed: {status_name(status)} ({detail})")
        self.status = status


class MechDesc(C.Structure):
    _fields_ = [("K", C.c_int32), ("R", C.c_int32), ("E", C.c_int32), ("W", _P), ("comp", _P),
                ("awt", _P), ("nasa", _P), ("rsp", _P), ("rnu", _P), ("A", _P), ("b", _P),
                ("Ea", _P)]


class Batch(C.Structure):
    _fields_ = [("n", C.c_int64), ("ld", C.c_int64)]


class ChemSet(C.Structure):
    _fields_ = [("n", C.c_int64), ("ld", C.c_int64), ("dt", C.c_double), ("T", _P), ("p", _P),
                ("Y", _P), ("RR", _P), ("h_hint", _P), ("stats", _P)]


class Tuning(C.Structure):
    _fields_ = [("lanes_per_cell", C.c_int32), ("waves_per_cu", C.c_int32),
                ("cells_per_s", C.c_double)]


class StepOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_Y", C.c_double), ("atol_T", C.c_double),
                ("h0", C.c_double), ("h_min", C.c_double), ("max_steps", C.c_int32)]


def lib():
    """Load libchemstep.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it first (python -m paper_2312_05800_amd.build)")
            L = C.CDLL(LIB_PATH)
            L.chem_status_string.restype = C.c_char_p
            L.chem_status_string.argtypes = [C.c_int]
            L.chem_last_error.restype = C.c_char_p
            L.chem_mech_create.argtypes = [C.POINTER(MechDesc), C.POINTER(_P)]
            L.chem_mech_destroy.argtypes = [_P]
            L.chem_mech_num_species.argtypes = [_P]
            L.chem_mech_num_reactions.argtypes = [_P]
            L.chem_rates.argtypes = [_P, Batch, _P, _P, _P, _P, _P, _P, _P]
            L.chem_step.argtypes = [_P, Batch, C.c_double, _P, _P, _P, _P, _P, _P, _P, _P, _P]
            L.chem_step_sets.argtypes = [_P, C.c_int32, _P, _P, _P]
            L.chem_autotune.argtypes = [_P, Batch, C.c_double, _P, _P, _P, _P, _P, _P]
            L.chem_set_tuning.argtypes = [_P, _P]
            L.chem_get_tuning.argtypes = [_P, _P]
            L.chem_step_graph_create.argtypes = [_P, Batch, C.c_double, _P, _P, _P, _P, _P, _P,
                                                 _P, _P, _P, C.POINTER(_P)]
            L.chem_step_sets_graph_create.argtypes = [_P, C.c_int32, _P, _P, _P, C.POINTER(_P)]
            L.chem_step_sets_device.argtypes = [_P, C.c_int32, _P, _P, _P, _P]
            L.chem_graph_launch.argtypes = [_P, _P]
            L.chem_graph_destroy.argtypes = [_P]
            L.chem_measure_peaks.argtypes = [_P, _P]
            L.chem_sample_states.argtypes = [_P, Batch, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                             _P, _P, _P]
            L.chem_pasr_scale.argtypes = [_P, Batch, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
            L.chem_profile_enable.argtypes = [C.c_int32]
            L.chem_profile_read.argtypes = [_P, _P, _P, C.c_int32]
            L.chem_profile_read.restype = C.c_int32
            _setup_ann(L)
            _lib = L
    return _lib


def _setup_ann(L):
    """Prototypes of the surrogate-form entry points, when the library has them."""
    if hasattr(L, "ann_create"):
        from . import ann as _ann
        _ann._prototypes(L)


def status_name(s: int) -> str:
    try:
        return lib().chem_status_string(int(s)).decode()
    except Exception:  # the library itself failed to load
        return str(s)


def check(fn: str, st: int):
    if st != 0:
        raise ChemError(fn, st, lib().chem_last_error().decode())


def _dptr(t, dtype=None, name="array"):
    """Device pointer of a torch CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _vec(t, n, name, dtype=None):
    """Device pointer of a 1-D contiguous tensor holding at least n elements
    (None -> NULL).  Raises ValueError before anything is launched."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dim() != 1 or (t.numel() > 1 and t.stride(0) != 1):
        raise ValueError(f"{name} must be a contiguous 1-D tensor")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, {n} needed")
    return _dptr(t, dtype, name)


def _soa(t, K, n, name):
    """Checks a [K][ld] species array and returns its leading dimension."""
    if n == 0 and t.dim() == 2 and t.shape[0] == K:
        return t.shape[1]
    if t.dim() != 2 or t.shape[0] != K or t.shape[1] < n or t.stride(1) != 1:
        raise ValueError(f"{name} must be a [K={K}, >=n] row-major view")
    return t.stride(0) if K > 1 else t.shape[1]


class Mechanism:
    """Device copy of a reaction mechanism (chem_mech handle).

    ``desc`` is any object with the chem_mech_desc fields as numpy arrays:
    W, comp, awt, nasa, rsp, rnu, A, b, Ea (e.g. a chemgen.Mech)."""

    def __init__(self, desc):
        self._keep = {}
        arrs = {}
        for name, dt in (("W", np.float64), ("comp", np.int32), ("awt", np.float64),
                         ("nasa", np.float64), ("rsp", np.int32), ("rnu", np.int32),
                         ("A", np.float64), ("b", np.float64), ("Ea", np.float64)):
            a = np.ascontiguousarray(getattr(desc, name), dtype=dt)
            arrs[name] = a
            self._keep[name] = a
        K = arrs["W"].shape[0]
        R = arrs["rsp"].shape[0]
        E = arrs["awt"].shape[0]
        d = MechDesc(K, R, E, *(arrs[k].ctypes.data for k in
                                ("W", "comp", "awt", "nasa", "rsp", "rnu", "A", "b", "Ea")))
        h = _P()
        check("chem_mech_create", lib().chem_mech_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.K, self.R, self.E = K, R, E
        self.desc = desc

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.chem_mech_destroy(h)
            self.handle = None


def _opts(opts):
    if opts is None:
        return None
    o = dict(rtol=1e-6, atol_Y=1e-12, atol_T=1e-6, h0=1e-8, h_min=1e-20, max_steps=100000)
    o.update(opts)
    return StepOpts(o["rtol"], o["atol_Y"], o["atol_T"], o["h0"], o["h_min"], int(o["max_steps"]))


def chem_rates(mech: Mechanism, T, p, Y, dTdt: bool = True, kfkr: bool = False, stream=None):
    """Instantaneous wdot [K, n] (mol/m^3/s), dT/dt [n] (K/s) and optionally
    k_f/k_r [2R, n] of every cell.  Returns new tensors."""
    import torch
    n = T.shape[0]
    ld = _soa(Y, mech.K, n, "Y")
    dev = T.device
    wdot = torch.empty((mech.K, ld), dtype=torch.float64, device=dev)
    dT = torch.empty(n, dtype=torch.float64, device=dev) if dTdt else None
    kk = torch.empty((2 * mech.R, ld), dtype=torch.float64, device=dev) if kfkr else None
    f64 = torch.float64
    check("chem_rates", lib().chem_rates(
        mech.handle, Batch(n, ld), _vec(T, n, "T", f64), _vec(p, n, "p", f64), _dptr(Y, f64, "Y"),
        _dptr(wdot), _dptr(dT), _dptr(kk), _stream(stream)))
    out = dict(wdot=wdot[:, :n])
    if dTdt:
        out["dTdt"] = dT
    if kfkr:
        out["kf"] = kk[:mech.R, :n]
        out["kr"] = kk[mech.R:, :n]
    return out


def chem_step(mech: Mechanism, dt, T, p, Y, dt_cell=None, RR=None, h_hint=None, stats=None,
              opts=None, stream=None):
    """Advance T [n] and Y [K, ld] in place by one chemistry step.  RR
    ([K, ld] float64), h_hint ([n] float64) and stats ([3, ld] int32) are
    optional caller-provided output tensors."""
    import torch
    n = T.shape[0]
    ld = _soa(Y, mech.K, n, "Y")
    if RR is not None and _soa(RR, mech.K, n, "RR") != ld:
        raise ValueError("RR must have the leading dimension of Y")
    if stats is not None and (stats.dim() != 2 or stats.shape[0] != 3 or stats.stride(0) != ld
                              or stats.dtype != torch.int32):
        raise ValueError("stats must be an int32 [3, ld] tensor with the leading dimension of Y")
    o = _opts(opts)
    f64 = torch.float64
    check("chem_step", lib().chem_step(
        mech.handle, Batch(n, ld), float(dt), _vec(dt_cell, n, "dt_cell", f64),
        _vec(T, n, "T", f64), _vec(p, n, "p", f64), _dptr(Y, f64, "Y"), _dptr(RR, f64, "RR"),
        _vec(h_hint, n, "h_hint", f64), _dptr(stats, torch.int32, "stats"),
        None if o is None else C.byref(o), _stream(stream)))


def _set_table(mech, sets):
    import torch
    f64 = torch.float64
    arr = (ChemSet * max(1, len(sets)))()
    for i, st in enumerate(sets):
        n = st["T"].shape[0]
        ld = _soa(st["Y"], mech.K, n, "Y")
        RR, stats = st.get("RR"), st.get("stats")
        if RR is not None and _soa(RR, mech.K, n, "RR") != ld:
            raise ValueError("RR must have the leading dimension of Y")
        if stats is not None and (stats.dim() != 2 or stats.shape[0] != 3
                                  or (n > 0 and stats.stride(0) != ld)):
            raise ValueError("stats must be an int32 [3, ld] tensor with the leading dimension "
                             "of Y")
        arr[i] = ChemSet(n, ld, float(st["dt"]), _vec(st["T"], n, "T", f64),
                         _vec(st["p"], n, "p", f64), _dptr(st["Y"], f64, "Y"),
                         _dptr(RR, f64, "RR"), _vec(st.get("h_hint"), n, "h_hint", f64),
                         _dptr(stats, torch.int32, "stats"))
    return arr


def chem_step_sets(mech: Mechanism, sets, opts=None, stream=None):
    """chem_step over several cell sets in one launch.  ``sets``: sequence of
    dicts with keys dt, T, p, Y and optionally RR, h_hint, stats (tensors as
    in chem_step); updated in place."""
    arr = _set_table(mech, sets)
    o = _opts(opts)
    check("chem_step_sets", lib().chem_step_sets(mech.handle, len(sets), C.addressof(arr),
                                                 None if o is None else C.byref(o),
                                                 _stream(stream)))


def set_table_device(mech: Mechanism, sets, device=None):
    """The chem_set table of ``sets`` (as for chem_step_sets) copied into a
    device uint8 tensor, for chem_step_sets_device.  Returns (table, n)."""
    import torch
    arr = _set_table(mech, sets)
    host = torch.frombuffer(bytearray(C.string_at(C.addressof(arr), C.sizeof(arr))),
                            dtype=torch.uint8)
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    return host.to(dev), len(sets)


def chem_step_sets_device(mech: Mechanism, table, n_sets, opts=None, n_bad=None, stream=None):
    """chem_step_sets on a table already in device memory (set_table_device);
    n_bad: optional device int32 [1] receiving the number of skipped sets."""
    import torch
    if not isinstance(table, torch.Tensor) or not table.is_cuda or \
            table.numel() < n_sets * C.sizeof(ChemSet):
        raise ValueError("table must be a device tensor holding n_sets chem_set descriptors")
    o = _opts(opts)
    check("chem_step_sets_device", lib().chem_step_sets_device(
        mech.handle, int(n_sets), table.data_ptr(), None if o is None else C.byref(o),
        _vec(n_bad, 1, "n_bad", torch.int32), _stream(stream)))


def chem_step_sets_graph(mech: Mechanism, sets, opts=None, stream=None):
    """chem_step_sets captured as a graph on these sets (see chem_step_sets)."""
    arr = _set_table(mech, sets)
    o = _opts(opts)
    h = _P()
    check("chem_step_sets_graph_create", lib().chem_step_sets_graph_create(
        mech.handle, len(sets), C.addressof(arr), None if o is None else C.byref(o),
        _stream(stream), C.byref(h)))
    return Graph(h, (mech, [dict(st) for st in sets]))


def chem_autotune(mech: Mechanism, dt, T, p, Y, opts=None, stream=None):
    """Time the integrator's launch shapes on these cells (not modified) and
    keep the fastest in the mechanism; returns it as a dict."""
    import torch
    n = T.shape[0]
    ld = _soa(Y, mech.K, n, "Y")
    o = _opts(opts)
    t = Tuning()
    f64 = torch.float64
    check("chem_autotune", lib().chem_autotune(
        mech.handle, Batch(n, ld), float(dt), _vec(T, n, "T", f64), _vec(p, n, "p", f64),
        _dptr(Y, f64, "Y"), None if o is None else C.byref(o), _stream(stream), C.byref(t)))
    return dict(lanes_per_cell=t.lanes_per_cell, waves_per_cu=t.waves_per_cu,
                cells_per_s=t.cells_per_s)


def chem_set_tuning(mech: Mechanism, lanes_per_cell=0, waves_per_cu=0, default=False):
    """Set the integrator launch shape (default=True: the built-in heuristic)."""
    t = Tuning(int(lanes_per_cell), int(waves_per_cu), 0.0)
    check("chem_set_tuning", lib().chem_set_tuning(mech.handle, None if default else C.byref(t)))


def chem_get_tuning(mech: Mechanism):
    t = Tuning()
    check("chem_get_tuning", lib().chem_get_tuning(mech.handle, C.byref(t)))
    return dict(lanes_per_cell=t.lanes_per_cell, waves_per_cu=t.waves_per_cu,
                cells_per_s=t.cells_per_s)


class Graph:
    """A captured step (chem_graph).  Holds references to the objects and
    arrays it was captured with, so none of them is freed before it."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def launch(self, stream=None):
        check("chem_graph_launch", lib().chem_graph_launch(self.handle, _stream(stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.chem_graph_destroy(h)
            self.handle = None


def chem_step_graph(mech: Mechanism, dt, T, p, Y, dt_cell=None, RR=None, h_hint=None, stats=None,
                    opts=None):
    """chem_step captured as a graph on these arrays (see chem_step)."""
    import torch
    n = T.shape[0]
    ld = _soa(Y, mech.K, n, "Y")
    o = _opts(opts)
    f64 = torch.float64
    h = _P()
    if RR is not None and _soa(RR, mech.K, n, "RR") != ld:
        raise ValueError("RR must have the leading dimension of Y")
    if stats is not None and (stats.dim() != 2 or stats.shape[0] != 3 or stats.stride(0) != ld
                              or stats.dtype != torch.int32):
        raise ValueError("stats must be an int32 [3, ld] tensor with the leading dimension of Y")
    check("chem_step_graph_create", lib().chem_step_graph_create(
        mech.handle, Batch(n, ld), float(dt), _vec(dt_cell, n, "dt_cell", f64),
        _vec(T, n, "T", f64), _vec(p, n, "p", f64), _dptr(Y, f64, "Y"), _dptr(RR, f64, "RR"),
        _vec(h_hint, n, "h_hint", f64), _dptr(stats, torch.int32, "stats"),
        None if o is None else C.byref(o), None, C.byref(h)))
    return Graph(h, (mech, T, p, Y, dt_cell, RR, h_hint, stats))


class SampleOpts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("gamma", C.c_double),
                ("T_min", C.c_double), ("hc_min", C.c_double), ("hc_max", C.c_double),
                ("on_min", C.c_double), ("on_max", C.c_double), ("phi_min", C.c_double),
                ("phi_max", C.c_double), ("n2", C.c_int32), ("el_C", C.c_int32),
                ("el_H", C.c_int32), ("el_O", C.c_int32), ("el_N", C.c_int32)]


def sample_states(mech: Mechanism, mech_desc, T, p, Y, c, s=None, end_eq=None, end_air=None,
                  alpha=0.125, beta=10.0, gamma=0.1, T_min=500.0, hc=(2.65, 4.67),
                  on=(0.254, 0.32), phi=(0.20, 1.15), stream=None):
    """Training-set sampler (chem_sample_states): returns (T', p', Y', keep)
    device tensors.  mech_desc names the N2 species and the C/H/O/N elements
    (a chemgen.Mech); c: [K+3, ld] draws, s: [n] mixing fractions (< 0:
    perturb the seed) or None; end_eq / end_air: [K+2] device tensors."""
    import torch
    n = T.shape[0]
    ld = _soa(Y, mech.K, n, "Y")
    if _soa(c, mech.K + 3, n, "c") != ld:
        raise ValueError("c must have the leading dimension of Y")
    el = [mech_desc.elements.index(x) for x in ("C", "H", "O", "N")]
    o = SampleOpts(alpha, beta, gamma, T_min, hc[0], hc[1], on[0], on[1], phi[0], phi[1],
                   mech_desc.index("N2"), *el)
    f64 = torch.float64
    To = torch.empty(n, dtype=f64, device=T.device)
    po = torch.empty(n, dtype=f64, device=T.device)
    Yo = torch.empty((mech.K, ld), dtype=f64, device=T.device)
    keep = torch.empty(n, dtype=torch.uint8, device=T.device)
    check("chem_sample_states", lib().chem_sample_states(
        mech.handle, Batch(n, ld), _vec(T, n, "T", f64), _vec(p, n, "p", f64),
        _dptr(Y, f64, "Y"), _dptr(c, f64, "c"), _vec(s, n, "s", f64),
        _vec(end_eq, mech.K + 2, "end_eq", f64), _vec(end_air, mech.K + 2, "end_air", f64),
        C.byref(o), _dptr(To, f64), _dptr(po, f64), _dptr(Yo, f64), _dptr(keep, torch.uint8),
        _stream(stream)))
    return To, po, Yo, keep


class PasrOpts(C.Structure):
    _fields_ = [("eta", C.c_double)]


def pasr_scale(mech: Mechanism, T, p, Y, RR, tau_taylor, tau_kolmogorov, eta=1e-3,
               want_tau_c=True, stream=None):
    """PaSR closure (chem_pasr_scale): RR [K, ld] is scaled in place by each
    cell's reacting fraction; returns (kappa [n], tau_c [n] or None) device
    tensors."""
    import torch
    n = T.shape[0]
    ld = _soa(Y, mech.K, n, "Y")
    if _soa(RR, mech.K, n, "RR") != ld:
        raise ValueError("RR must have the leading dimension of Y")
    f64 = torch.float64
    kappa = torch.empty(n, dtype=f64, device=T.device)
    tc = torch.empty(n, dtype=f64, device=T.device) if want_tau_c else None
    o = PasrOpts(eta)
    check("chem_pasr_scale", lib().chem_pasr_scale(
        mech.handle, Batch(n, ld), _vec(T, n, "T", f64), _vec(p, n, "p", f64),
        _dptr(Y, f64, "Y"), _dptr(RR, f64, "RR"), _vec(tau_taylor, n, "tau_taylor", f64),
        _vec(tau_kolmogorov, n, "tau_kolmogorov", f64), C.byref(o), _dptr(kappa, f64),
        _dptr(tc, f64), _stream(stream)))
    return kappa, tc


def measure_peaks(stream=None):
    """Measured TFLOP/s of dense BF16 MFMA, FP8 MFMA and FP64 vector FMA."""
    out = (C.c_double * 3)()
    check("chem_measure_peaks", lib().chem_measure_peaks(out, _stream(stream)))
    return {"bf16_mfma": out[0], "fp8_mfma": out[1], "fp64_vector": out[2]}


def profile_enable(on: bool = True):
    """Bracket every library launch with HIP events on its own stream."""
    lib().chem_profile_enable(1 if on else 0)


def profile_read(cap: int = 64):
    """{label: (launches, total_ms)} since the previous read (synchronises)."""
    names = (C.c_char * 48 * cap)()
    cnt = (C.c_int64 * cap)()
    tot = (C.c_double * cap)()
    n = lib().chem_profile_read(names, cnt, tot, cap)
    return {bytes(names[i]).split(b"\0")[0].decode(): (int(cnt[i]), float(tot[i]))
            for i in range(n)}
