"""Helpers shared by the GPU tests (no computation of the method here)."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2312_05800_amd as P
    P.lib()  # raises if the library is missing: GPU tests never run without it
    return torch.device("cuda:0")


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def one_way_scale(mech, T, p, Y, kf, kr):
    """Largest one-way rate of progress per cell, the scale of rounding in
    wdot.  kf/kr: [R, N]."""
    RG = 8.314462618
    S = (Y / mech.W[:, None]).sum(axis=0)
    C = (p / (RG * T * S))[None, :] * Y / mech.W[:, None]
    sc = np.zeros(T.size)
    for r in range(mech.R):
        f = kf[r].copy()
        b = kr[r].copy()
        for s in (0, 1):
            k = mech.rsp[r, s]
            if k >= 0:
                f *= C[k] ** mech.rnu[r, s]
        for s in (2, 3):
            k = mech.rsp[r, s]
            if k >= 0:
                b *= C[k] ** mech.rnu[r, s]
        sc = np.maximum(sc, np.maximum(np.abs(f), np.abs(b)))
    return sc


def compare_state(T_g, Y_g, T_o, Y_o, rtol=1e-8, ytiny=1e-10, atol_tiny=1e-16):
    """Parity bar of the plain integrator: T and every Y_k > ytiny within
    rtol relative; smaller Y_k within atol_tiny absolute.  Returns a dict of
    the worst errors."""
    eT = np.abs(T_g - T_o) / np.abs(T_o)
    big = np.abs(Y_o) > ytiny
    eY = np.where(big, np.abs(Y_g - Y_o) / np.maximum(np.abs(Y_o), 1e-300), 0.0)
    eYs = np.where(big, 0.0, np.abs(Y_g - Y_o))
    return dict(T=float(eT.max(initial=0.0)), Y=float(eY.max(initial=0.0)),
                Ytiny=float(eYs.max(initial=0.0)),
                ok=bool(eT.max(initial=0.0) <= rtol and eY.max(initial=0.0) <= rtol
                        and eYs.max(initial=0.0) <= atol_tiny))
