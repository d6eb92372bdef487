"""CPU oracle for the per-cell chemistry step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls anything here, and this
package never imports the product.

* ``chem_oracle.c`` (plain C, FP64, one cell at a time) holds the plain form:
  NASA-7 thermo, mass-action kinetics, the analytic Jacobian, pivoted LU, the
  RODAS3 Rosenbrock integrator with error control, and RK4.  This module
  compiles it with gcc and wraps it with ctypes.
* ``ann.py`` (numpy, FP64 with optional BF16/FP8 rounding emulation) holds the
  surrogate form: Box-Cox transform, z-scoring, the GELU MLP, its L1 loss and
  gradients, Adam, and the post-processing (element projection, residual and
  out-of-distribution flags, enthalpy Newton for T).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chem_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libchem_oracle.so")
_lock = threading.Lock()
_lib = None

STATUS = {0: "OK", 1: "MAX_STEPS", 2: "H_UNDERFLOW", 3: "NONFINITE", 4: "SINGULAR"}
RGAS = 8.314462618
PREF = 101325.0


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, -O2 -ffp-contract=off, OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mech(C.Structure):
    _fields_ = [("K", C.c_int), ("R", C.c_int), ("W", C.c_void_p), ("nasa", C.c_void_p),
                ("rsp", C.c_void_p), ("rnu", C.c_void_p), ("A", C.c_void_p), ("b", C.c_void_p),
                ("Ea", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_Y", C.c_double), ("atol_T", C.c_double),
                ("h0", C.c_double), ("h_min", C.c_double), ("max_steps", C.c_int)]


RHS_CB = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double))
JAC_CB = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                     C.POINTER(C.c_double))

_P = C.c_void_p


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = C.CDLL(build())
            L.or_eval.argtypes = [_P, C.c_double, _P, _P, _P, _P, _P, _P]
            L.or_thermo.argtypes = [_P, C.c_double, _P, _P, _P]
            L.or_species_thermo.argtypes = [_P, C.c_int, C.c_double, _P, _P, _P, _P]
            L.or_mixture_enthalpy.argtypes = [_P, C.c_double, _P]
            L.or_mixture_enthalpy.restype = C.c_double
            L.or_chem_rates.argtypes = [_P, C.c_long, C.c_long, _P, _P, _P, _P, _P, _P, _P]
            L.or_lu.argtypes = [C.c_int, _P, _P]
            L.or_lu.restype = C.c_int
            L.or_lu_solve.argtypes = [C.c_int, _P, _P, _P]
            L.or_ros_tableau.argtypes = [_P, _P, _P, _P, _P, _P]
            L.or_ros_step_generic.argtypes = [C.c_int, RHS_CB, JAC_CB, _P, _P, C.c_double, _P,
                                              _P]
            L.or_ros_step_generic.restype = C.c_int
            L.or_integrate.argtypes = [_P, C.c_double, _P, C.c_double, _P, _P, _P, _P]
            L.or_integrate.restype = C.c_int
            L.or_chem_step.argtypes = [_P, C.c_long, C.c_long, C.c_double, _P, _P, _P, _P, _P,
                                       _P, _P, _P, C.c_int]
            L.or_rk4.argtypes = [_P, C.c_double, _P, C.c_double, C.c_long]
            L.or_max_threads.restype = C.c_int
            _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleMech:
    """Holds contiguous copies of a chemgen.Mech and the C descriptor."""

    def __init__(self, mech):
        self.mech = mech
        self.K, self.R = mech.K, mech.R
        self.n = self.K + 1
        self._W = _f64(mech.W)
        self._nasa = _f64(mech.nasa)
        self._rsp = np.ascontiguousarray(mech.rsp, dtype=np.int32)
        self._rnu = np.ascontiguousarray(mech.rnu, dtype=np.int32)
        self._A = _f64(mech.A)
        self._b = _f64(mech.b)
        self._Ea = _f64(mech.Ea)
        self.c = _Mech(self.K, self.R, _ptr(self._W), _ptr(self._nasa), _ptr(self._rsp),
                       _ptr(self._rnu), _ptr(self._A), _ptr(self._b), _ptr(self._Ea))
        self.p = C.addressof(self.c)


def default_opts(**kw):
    o = dict(rtol=1e-6, atol_Y=1e-12, atol_T=1e-6, h0=1e-8, h_min=1e-20, max_steps=100000)
    o.update(kw)
    return o


def _opts(o):
    o = default_opts(**(o or {}))
    return _Opts(o["rtol"], o["atol_Y"], o["atol_T"], o["h0"], o["h_min"], int(o["max_steps"]))


# ---------------------------------------------------------------- wrappers

def thermo(om: OracleMech, T: float):
    """(c_p/R, h/RT, s/R) of every species at T."""
    cp, h, s = (np.zeros(om.K) for _ in range(3))
    lib().or_thermo(om.p, float(T), _ptr(cp), _ptr(h), _ptr(s))
    return cp, h, s


def species_dcp(om: OracleMech, k: int, T: float) -> float:
    a, b, c, d = (C.c_double() for _ in range(4))
    lib().or_species_thermo(om.p, k, float(T), C.byref(a), C.byref(b), C.byref(c), C.byref(d))
    return d.value


def mixture_enthalpy(om: OracleMech, T: float, Y) -> float:
    Y = _f64(Y)
    return lib().or_mixture_enthalpy(om.p, float(T), _ptr(Y))


def evaluate(om: OracleMech, p: float, y, jac: bool = False):
    """RHS f(y), wdot, kf, kr (and the Jacobian) at one state y = [T, Y]."""
    y = _f64(y)
    f = np.zeros(om.n)
    w = np.zeros(om.K)
    kf = np.zeros(om.R)
    kr = np.zeros(om.R)
    J = np.zeros((om.n, om.n)) if jac else None
    lib().or_eval(om.p, float(p), _ptr(y), _ptr(f), _ptr(w), _ptr(kf), _ptr(kr), _ptr(J))
    out = dict(f=f, wdot=w, kf=kf, kr=kr)
    if jac:
        out["J"] = J
    return out


def rhs(om, p, y):
    return evaluate(om, p, y)["f"]


def jacobian(om, p, y):
    return evaluate(om, p, y, jac=True)["J"]


def chem_rates(om: OracleMech, T, p, Y, want_k: bool = False):
    T, p, Y = _f64(T), _f64(p), _f64(Y)
    N = T.size
    w = np.zeros((om.K, N))
    dT = np.zeros(N)
    kf = np.zeros((om.R, N)) if want_k else None
    kr = np.zeros((om.R, N)) if want_k else None
    lib().or_chem_rates(om.p, N, N, _ptr(T), _ptr(p), _ptr(Y), _ptr(w), _ptr(dT), _ptr(kf),
                        _ptr(kr))
    return (w, dT, kf, kr) if want_k else (w, dT)


def lu(a):
    a = _f64(a).copy()
    n = a.shape[0]
    order = np.zeros(n, dtype=np.int32)
    st = lib().or_lu(n, _ptr(a), _ptr(order))
    return st, a, order


def lu_solve(a, order, b):
    b = _f64(b).copy()
    lib().or_lu_solve(a.shape[0], _ptr(a), _ptr(order), _ptr(b))
    return b


def tableau():
    g = C.c_double()
    A, Cc = np.zeros(16), np.zeros(16)
    M, E = np.zeros(4), np.zeros(4)
    nf = np.zeros(4, dtype=np.int32)
    lib().or_ros_tableau(C.byref(g), _ptr(A), _ptr(Cc), _ptr(M), _ptr(E), _ptr(nf))
    return dict(gamma=g.value, A=A.reshape(4, 4), C=Cc.reshape(4, 4), m=M, e=E, newf=nf)


def ros_step_generic(n, f, jac, y, h):
    """One fixed RODAS3 step on y' = f(y) (numpy callables).  Returns
    (y_new, y_embedded)."""
    def _rhs(ctx, yp, fp):
        yy = np.ctypeslib.as_array(yp, (n,)).copy()
        np.ctypeslib.as_array(fp, (n,))[:] = f(yy)

    def _jac(ctx, yp, fp, Jp):
        yy = np.ctypeslib.as_array(yp, (n,)).copy()
        np.ctypeslib.as_array(fp, (n,))[:] = f(yy)
        np.ctypeslib.as_array(Jp, (n * n,))[:] = np.asarray(jac(yy), dtype=np.float64).ravel()

    cr, cj = RHS_CB(_rhs), JAC_CB(_jac)
    y = _f64(y)
    yn, ye = np.zeros(n), np.zeros(n)
    st = lib().or_ros_step_generic(n, cr, cj, None, _ptr(y), float(h), _ptr(yn), _ptr(ye))
    if st:
        raise RuntimeError("singular matrix")
    return yn, ye


def integrate(om: OracleMech, p, y, dt, opts=None, h_hint=0.0):
    """One cell: returns (y_out, status, n_acc, n_rej, h_next)."""
    y = _f64(y).copy()
    h = C.c_double(h_hint)
    na, nr = C.c_int(), C.c_int()
    o = _opts(opts)
    st = lib().or_integrate(om.p, float(p), _ptr(y), float(dt), C.addressof(o), C.byref(h),
                            C.byref(na), C.byref(nr))
    return y, st, na.value, nr.value, h.value


def chem_step(om: OracleMech, dt, T, p, Y, opts=None, dt_cell=None, h_hint=None,
              nthreads: int = 0):
    """Batched plain step.  Returns dict(T, Y, RR, stats, h_hint) (new arrays)."""
    T = _f64(T).copy()
    p = _f64(p)
    Y = _f64(Y).copy()
    N = T.size
    RR = np.zeros((om.K, N))
    stats = np.zeros((3, N), dtype=np.int32)
    hh = None if h_hint is None else _f64(h_hint).copy()
    dtc = None if dt_cell is None else _f64(dt_cell)
    o = _opts(opts)
    lib().or_chem_step(om.p, N, N, float(dt), _ptr(dtc), _ptr(T), _ptr(p), _ptr(Y), _ptr(RR),
                       _ptr(hh), _ptr(stats), C.addressof(o), int(nthreads))
    return dict(T=T, Y=Y, RR=RR, stats=stats, h_hint=hh)


def rk4(om: OracleMech, p, y, dt, nsteps):
    y = _f64(y).copy()
    lib().or_rk4(om.p, float(p), _ptr(y), float(dt), int(nsteps))
    return y


def max_threads() -> int:
    return lib().or_max_threads()
