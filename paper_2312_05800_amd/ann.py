"""ctypes binding of the surrogate-form entry points (ann_* in
include/chemstep.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np

from .binding import Batch, StepOpts, _dptr, _opts, _soa, _stream, _vec, check, lib

_P = C.c_void_p


class Arch(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_out", C.c_int32), ("hidden", C.c_int32 * 3),
                ("prec", C.c_int32), ("members", C.c_int32)]


class Norm(C.Structure):
    _fields_ = [("lambda_", C.c_float), ("dt_model", C.c_double), ("mu_in", _P), ("sd_in", _P),
                ("lo", _P), ("hi", _P), ("mu_out", _P), ("sd_out", _P)]


class StepOptsANN(C.Structure):
    _fields_ = [("residual_tol", C.c_float), ("ood_margin", C.c_float), ("fallback", C.c_int32),
                ("audit_fraction", C.c_float), ("audit", _P)]


class TrainOpts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("w_mass", C.c_float), ("w_energy", C.c_float),
                ("w_hrr", C.c_float)]


def _prototypes(L):
    L.ann_create.argtypes = [C.POINTER(Arch), C.c_uint64, C.POINTER(_P)]
    L.ann_destroy.argtypes = [_P]
    L.ann_set_layer.argtypes = [_P, C.c_int32, _P, _P]
    L.ann_get_layer.argtypes = [_P, C.c_int32, _P, _P]
    L.ann_get_grad.argtypes = [_P, C.c_int32, _P, _P]
    L.ann_get_moments.argtypes = [_P, C.c_int32, _P, _P, _P, _P]
    L.ann_set_norm.argtypes = [_P, C.POINTER(Norm)]
    L.ann_get_norm.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.ann_fit_norm.argtypes = [_P, Batch, _P, _P, _P, _P, C.c_float, C.c_double, _P]
    L.ann_forward.argtypes = [_P, Batch, _P, _P, _P, _P, _P]
    L.ann_step.argtypes = [_P, _P, Batch, C.c_double, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.ann_step_noalloc.argtypes = [_P, _P, Batch, C.c_double, _P, _P, _P, _P, _P, _P, _P, _P,
                                   _P]
    L.ann_train_step.argtypes = [_P, _P, Batch, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.ann_num_steps.argtypes = [_P]
    L.ann_autotune_train.argtypes = [_P, C.c_int64, _P, _P, _P]
    L.ann_num_steps.restype = C.c_int64
    L.ann_quantize_fp8.argtypes = [_P, Batch, _P, _P, _P, _P]
    L.ann_set_precision.argtypes = [_P, C.c_int32]
    L.ann_get_fp8_scales.argtypes = [_P, _P, _P]
    L.ann_step_graph_create.argtypes = [_P, _P, Batch, C.c_double, _P, _P, _P, _P, _P, _P, _P,
                                        _P, _P, C.POINTER(_P)]
    L.ann_save.argtypes = [_P, C.c_char_p]
    L.ann_load.argtypes = [C.c_char_p, C.POINTER(_P)]


class AnnModel:
    """Handle of a surrogate network (ann_model); members = n_out makes the
    per-species ensemble (layer index 4 g + l addresses member g)."""

    def __init__(self, n_in=None, n_out=None, hidden=(1600, 800, 400), seed=0, prec=0,
                 members=1, _handle=None):
        lib()
        if _handle is not None:
            self.handle = _handle
        else:
            a = Arch(int(n_in), int(n_out), (C.c_int32 * 3)(*hidden), int(prec), int(members))
            h = _P()
            check("ann_create", lib().ann_create(C.byref(a), C.c_uint64(seed), C.byref(h)))
            self.handle = h
        self._dims = None

    @classmethod
    def load(cls, path):
        h = _P()
        check("ann_load", lib().ann_load(str(path).encode(), C.byref(h)))
        return cls(_handle=h)

    def save(self, path):
        check("ann_save", lib().ann_save(self.handle, str(path).encode()))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                lib().ann_destroy(h)
            except Exception:
                pass
            self.handle = None

    def autotune_train(self, B, stream=None):
        """Pick the training products' tilings for batch B by measurement
        (ann_autotune_train); returns the summed product times in ms with the
        built-in rules and with the chosen tilings."""
        d0, d1 = C.c_double(), C.c_double()
        check("ann_autotune_train", lib().ann_autotune_train(
            self.handle, C.c_int64(int(B)), C.byref(d0), C.byref(d1), _stream(stream)))
        return {"products_ms_default": d0.value, "products_ms_tuned": d1.value}

    @property
    def num_steps(self):
        return int(lib().ann_num_steps(self.handle))

    def _layer_shapes(self, dims):
        return [(dims[i + 1], dims[i]) for i in range(4)]

    def set_layer(self, layer, W, b):
        W = np.ascontiguousarray(W, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        check("ann_set_layer", lib().ann_set_layer(self.handle, int(layer), W.ctypes.data,
                                                   b.ctypes.data))

    def get_layer(self, layer, shape):
        W = np.zeros(shape, dtype=np.float32)
        b = np.zeros(shape[0], dtype=np.float32)
        check("ann_get_layer", lib().ann_get_layer(self.handle, int(layer), W.ctypes.data,
                                                   b.ctypes.data))
        return W, b

    def get_grad(self, layer, shape):
        W = np.zeros(shape, dtype=np.float32)
        b = np.zeros(shape[0], dtype=np.float32)
        check("ann_get_grad", lib().ann_get_grad(self.handle, int(layer), W.ctypes.data,
                                                 b.ctypes.data))
        return W, b

    def get_moments(self, layer, shape):
        """Adam's (mW, vW, mb, vb) of a layer as host FP32 arrays."""
        mW = np.zeros(shape, dtype=np.float32)
        vW = np.zeros(shape, dtype=np.float32)
        mb = np.zeros(shape[0], dtype=np.float32)
        vb = np.zeros(shape[0], dtype=np.float32)
        check("ann_get_moments", lib().ann_get_moments(
            self.handle, int(layer), mW.ctypes.data, vW.ctypes.data, mb.ctypes.data,
            vb.ctypes.data))
        return mW, vW, mb, vb

    def set_norm(self, lam, dt_model, mu_in, sd_in, lo, hi, mu_out, sd_out):
        arrs = [np.ascontiguousarray(a, dtype=np.float32)
                for a in (mu_in, sd_in, lo, hi, mu_out, sd_out)]
        self._keep = arrs
        n = Norm(float(lam), float(dt_model), *(a.ctypes.data for a in arrs))
        check("ann_set_norm", lib().ann_set_norm(self.handle, C.byref(n)))

    def get_norm(self, n_in, n_out):
        out = dict(mu_in=np.zeros(n_in, np.float32), sd_in=np.zeros(n_in, np.float32),
                   lo=np.zeros(n_in, np.float32), hi=np.zeros(n_in, np.float32),
                   mu_out=np.zeros(n_out, np.float32), sd_out=np.zeros(n_out, np.float32))
        lam = C.c_float()
        dtm = C.c_double()
        check("ann_get_norm", lib().ann_get_norm(
            self.handle, *(out[k].ctypes.data for k in ("mu_in", "sd_in", "lo", "hi", "mu_out",
                                                        "sd_out")), C.byref(lam), C.byref(dtm)))
        out["lambda"] = lam.value
        out["dt_model"] = dtm.value
        return out

    def quantize_fp8(self, T, p, Y, stream=None):
        """Calibrate per-tensor scales on these cells and switch the hidden
        layers to FP8 E4M3."""
        import torch
        n = T.shape[0]
        ld = _soa(Y, Y.shape[0], n, "Y")
        f64 = torch.float64
        check("ann_quantize_fp8", lib().ann_quantize_fp8(
            self.handle, Batch(n, ld), _vec(T, n, "T", f64), _vec(p, n, "p", f64),
            _dptr(Y, f64, "Y"), _stream(stream)))

    def set_precision(self, prec):
        check("ann_set_precision", lib().ann_set_precision(self.handle, int(prec)))

    def fp8_scales(self):
        a = np.zeros(2, np.float32)
        w = np.zeros(2, np.float32)
        check("ann_get_fp8_scales", lib().ann_get_fp8_scales(self.handle, a.ctypes.data,
                                                             w.ctypes.data))
        return a, w

    def fit_norm(self, T, p, Y0, Y1, lam=0.1, dt_model=1e-5, stream=None):
        import torch
        n = T.shape[0]
        ld = _soa(Y0, Y0.shape[0], n, "Y0")
        if Y1.shape[0] != Y0.shape[0] or _soa(Y1, Y0.shape[0], n, "Y1") != ld:
            raise ValueError("Y1 must have the shape and leading dimension of Y0")
        f64 = torch.float64
        check("ann_fit_norm", lib().ann_fit_norm(
            self.handle, Batch(n, ld), _vec(T, n, "T", f64), _vec(p, n, "p", f64),
            _dptr(Y0, f64, "Y0"), _dptr(Y1, f64, "Y1"), float(lam), float(dt_model),
            _stream(stream)))

    def forward(self, T, p, Y, n_out, stream=None):
        import torch
        n = T.shape[0]
        ld = _soa(Y, Y.shape[0], n, "Y")
        U = torch.empty((n, n_out), dtype=torch.float32, device=T.device)
        f64 = torch.float64
        check("ann_forward", lib().ann_forward(
            self.handle, Batch(n, ld), _vec(T, n, "T", f64), _vec(p, n, "p", f64),
            _dptr(Y, f64, "Y"), _dptr(U), _stream(stream)))
        return U

    def step(self, mech, dt, T, p, Y, RR=None, flags=None, n_fallback=None, residual_tol=1e-6,
             ood_margin=0.05, fallback=True, fb_opts=None, stream=None, noalloc=False,
             audit_fraction=0.0, audit=None):
        """Surrogate chemistry step, in place on T and Y.  RR ([K, ld] float64),
        flags ([n] uint8) and n_fallback ([1] int64) are optional outputs.
        noalloc=True calls ann_step_noalloc (workspace in the library's static
        device array; the batch must fit in it).  audit_fraction > 0 with
        audit ([3 + 3K] float64 device tensor): the integrator also runs on
        that share of the cells and judges the network (see ann_step)."""
        import torch
        n = T.shape[0]
        ld = _soa(Y, mech.K, n, "Y")
        if RR is not None and _soa(RR, mech.K, n, "RR") != ld:
            raise ValueError("RR must have the leading dimension of Y")
        o = StepOptsANN(float(residual_tol), float(ood_margin), 1 if fallback else 0,
                        float(audit_fraction),
                        _vec(audit, 3 + 3 * mech.K, "audit", torch.float64))
        fo = _opts(fb_opts)
        f64 = torch.float64
        fn = "ann_step_noalloc" if noalloc else "ann_step"
        check(fn, getattr(lib(), fn)(
            self.handle, mech.handle, Batch(n, ld), float(dt), _vec(T, n, "T", f64),
            _vec(p, n, "p", f64), _dptr(Y, f64, "Y"), _dptr(RR, f64, "RR"),
            _vec(flags, n, "flags", torch.uint8),
            _vec(n_fallback, 1, "n_fallback", torch.int64),
            C.byref(o), None if fo is None else C.byref(fo), _stream(stream)))

    def step_graph(self, mech, dt, T, p, Y, RR=None, flags=None, n_fallback=None,
                   residual_tol=1e-6, ood_margin=0.05, fallback=True, fb_opts=None,
                   audit_fraction=0.0, audit=None):
        """ann_step captured as a graph on these arrays (see step)."""
        import torch
        from .binding import Graph
        n = T.shape[0]
        ld = _soa(Y, mech.K, n, "Y")
        if RR is not None and _soa(RR, mech.K, n, "RR") != ld:
            raise ValueError("RR must have the leading dimension of Y")
        o = StepOptsANN(float(residual_tol), float(ood_margin), 1 if fallback else 0,
                        float(audit_fraction),
                        _vec(audit, 3 + 3 * mech.K, "audit", torch.float64))
        fo = _opts(fb_opts)
        f64 = torch.float64
        h = _P()
        check("ann_step_graph_create", lib().ann_step_graph_create(
            self.handle, mech.handle, Batch(n, ld), float(dt), _vec(T, n, "T", f64),
            _vec(p, n, "p", f64), _dptr(Y, f64, "Y"), _dptr(RR, f64, "RR"),
            _vec(flags, n, "flags", torch.uint8),
            _vec(n_fallback, 1, "n_fallback", torch.int64),
            C.byref(o), None if fo is None else C.byref(fo), None, C.byref(h)))
        return Graph(h, (self, mech, T, p, Y, RR, flags, n_fallback))

    def train_step(self, T, p, Y0, Y1, loss, index=None, B=None, lr=1e-3, beta1=0.9,
                   beta2=0.999, eps=1e-8, stream=None, mech=None, T1=None, w_phys=(0.0, 0.0, 0.0),
                   terms=None):
        """One Adam step on B pairs (cells index[0..B) of the [K, ld] arrays, or
        the first B cells).  loss: device float32 [1] receiving the loss.
        w_phys = (mass, energy, heat release) weights of the physics terms;
        with any non-zero, or terms (device float32 [3]) given, mech and T1
        (the reference final temperatures, like T) are needed."""
        import torch
        if index is not None:
            # cells are gathered through the index: every array must hold the
            # cells it can name (the library does not see their extent)
            B = index.shape[0]
            ncell = T.shape[0]
            ld = _soa(Y0, Y0.shape[0], ncell, "Y0")
        else:
            B = T.shape[0] if B is None else B
            ncell = B
            ld = _soa(Y0, Y0.shape[0], B, "Y0")
        if Y1.shape[0] != Y0.shape[0] or _soa(Y1, Y0.shape[0], ncell, "Y1") != ld:
            raise ValueError("Y1 must have the shape and leading dimension of Y0")
        wm, we, wh = (float(x) for x in w_phys)
        o = TrainOpts(float(lr), float(beta1), float(beta2), float(eps), wm, we, wh)
        f64 = torch.float64
        check("ann_train_step", lib().ann_train_step(
            self.handle, None if mech is None else mech.handle, Batch(B, ld),
            _vec(T, ncell, "T", f64), _vec(p, ncell, "p", f64),
            _dptr(Y0, f64, "Y0"), _dptr(Y1, f64, "Y1"),
            None if T1 is None else _vec(T1, ncell, "T1", f64),
            _vec(index, B, "index", torch.int64),
            C.byref(o), _vec(loss, 1, "loss", torch.float32),
            None if terms is None else _vec(terms, 3, "terms", torch.float32), _stream(stream)))
