"""Surrogate-form oracle (numpy, FP64) -- TEST INFRASTRUCTURE ONLY.

Follows the paper's ANN model (Sec. 3.2):
* network input  x(t) = {T, p, F(Y(t))} with the Box-Cox transform F;
* network output the change of the mass fractions over one time step,
  u* = Y(t+dt) - Y(t), in physical mass-fraction units (only the inputs are
  Box-Cox transformed);
* inputs and outputs z-score normalised with training-set statistics;
* hidden layers 1600, 800, 400 with GELU; Adam; L1 loss (Eq. Loss), with
  the optional physics terms of Sec. 3.2 (mass-fraction sum, energy, heat
  release rate; formulas are this project's reading, see physics_terms).

Box-Cox (Box & Cox 1964): F(x) = (x^lambda - 1)/lambda with lambda = 0.1,
which maps mass fractions in [0, 1] to [-1/lambda, 0]; negative mass
fractions are clamped to 0 first.

Rounding emulation: ``prec="bf16"`` rounds every layer's input activations and
weights to bfloat16 (round to nearest even) and keeps everything else in FP64;
``prec="fp8"`` additionally quantises the hidden-to-hidden layers' operands to
OCP FP8 E4M3 (saturating, round to nearest even) with per-tensor scales
amax/448.  The GPU accumulates in FP32, so results agree to accumulation
rounding, not bitwise.

The post-processing (de-normalisation, weighted least-squares projection onto
element conservation, clipping, residual and out-of-distribution flags,
enthalpy Newton for T, reaction rates) is not in the paper; it is this
project's reading of how the ANN output becomes a full chemistry step.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from . import OracleMech, mixture_enthalpy, thermo, RGAS

LAMBDA = 0.1
HIDDEN = (1600, 800, 400)

# ----------------------------------------------------------------- rounding


def round_bf16(x):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64.
    First rounds to FP32 (round to nearest even), then to BF16 -- the GPU path
    holds FP32 values when it converts."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) >> 16
    nan = np.isnan(f)
    r = np.where(nan, (u >> 16) | 0x40, r)
    out = (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return out


def round_e4m3(x):
    """Round to OCP FP8 E4M3 (e4m3fn: max 448, no infinities), saturating,
    round to nearest even, via the exact grid of representable values."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), 448.0)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -9)))
    e = np.maximum(e, -6.0)              # subnormals share the 2^-6 binade spacing
    q = 2.0 ** (e - 3.0)                  # 3 mantissa bits
    m = a / q
    r = np.floor(m)
    frac = m - r
    up = (frac > 0.5) | ((frac == 0.5) & (np.mod(r, 2.0) == 1.0))
    r = r + up
    v = np.minimum(r * q, 448.0)
    return np.where(np.isnan(x), np.nan, np.sign(x) * v)


# ------------------------------------------------------------ transforms


def boxcox(Y, lam=LAMBDA):
    return (np.power(np.maximum(Y, 0.0), lam) - 1.0) / lam


def inv_boxcox(z, lam=LAMBDA):
    b = 1.0 + lam * z
    return np.where(b > 0.0, np.power(np.maximum(b, 0.0), 1.0 / lam), 0.0)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def features(T, p, Y, lam=LAMBDA):
    """Raw network features [T, p, F(Y_1..K)] as rows: shape [K+2, N]."""
    return np.vstack([np.atleast_2d(T), np.atleast_2d(p), boxcox(Y, lam)])


def targets(Y0, Y1, lam=LAMBDA):
    """u* = Y(t+dt) - Y(t), shape [K, N] (lam unused: the output is not
    transformed)."""
    return Y1 - Y0


def zstats(A):
    """Training-set mean and standard deviation per row (features x samples),
    with a zero spread replaced by 1."""
    mu = A.mean(axis=1)
    sd = A.std(axis=1)
    sd = np.where(sd < 1e-12 * np.abs(mu) + 1e-30, 1.0, sd)
    return mu, sd


# ------------------------------------------------------------------- MLP


def init_params(sizes, seed):
    """W_l ~ U(+-1/sqrt(fan_in)), b_l ~ U(+-1/sqrt(fan_in)); W_l is [out, in]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        bound = 1.0 / math.sqrt(fi)
        W = rng.uniform(-bound, bound, (fo, fi))
        b = rng.uniform(-bound, bound, fo)
        params.append((W, b))
    return params


def _q(x, prec, layer, nlayers, scale=None):
    if prec == "fp64":
        return x
    if prec == "fp8" and 0 < layer < nlayers - 1:
        return round_e4m3(x / scale) * scale
    return round_bf16(x)


def forward(params, X, prec="fp64", fp8_scales=None, keep=False):
    """X: [N, in] normalised inputs.  Returns the [N, out] output (and the
    pre-activations / layer inputs when keep=True).  fp8_scales: per hidden
    layer l (1..L-2) a pair (act_scale, weight_scale)."""
    L = len(params)
    h = X
    zs, hs = [], []
    for l, (W, b) in enumerate(params):
        if prec == "fp8" and 0 < l < L - 1:
            sa, sw = fp8_scales[l]
            hq = round_e4m3(h / sa) * sa
            Wq = round_e4m3(W / sw) * sw
        else:
            hq = _q(h, prec, l, L)
            Wq = _q(W, prec, l, L)
        hs.append(hq)
        z = hq @ Wq.T + b
        zs.append(z)
        h = gelu(z) if l < L - 1 else z
    if keep:
        return h, zs, hs
    return h


def l1_loss(u, target):
    return np.mean(np.abs(u - target))


def backward(params, X, target, prec="fp64"):
    """Gradients of the L1 loss (mean over samples and outputs) with respect
    to every W_l, b_l.  dL/du = sign(u - u*)/(N * n_out), sign(0) = 0.  With
    prec="bf16" the backward operands are rounded where the GPU rounds them:
    the layer inputs (as in forward), the weights, and each layer's incoming
    gradient dZ before it is multiplied."""
    L = len(params)
    u, zs, hs = forward(params, X, prec=prec, keep=True)
    N, nout = u.shape
    g = np.sign(u - target) / (N * nout)
    grads = [None] * L
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        gq = round_bf16(g) if prec != "fp64" else g
        dW = gq.T @ hs[l]
        db = g.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            Wq = round_bf16(W) if prec != "fp64" else W
            dh = gq @ Wq
            g = dh * gelu_grad(zs[l - 1])
    return grads, l1_loss(u, target)


# ------------------------------------------- per-species ensemble (Sec. 3.2)
#
# Sec. 3.2 trains and runs one network per species: K networks with the same
# inputs and hidden widths, member k predicting the change of species k
# alone.  The ensemble's loss is the mean of the members' L1 losses (which
# equals the L1 mean over samples and species of the single network), so
# member k's gradient is the gradient of its own loss divided by K.


def ensemble_forward(members, X, prec="fp64"):
    """members: K parameter lists with one output each.  Returns [N, K]."""
    return np.concatenate([forward(p, X, prec=prec) for p in members], axis=1)


def ensemble_backward(members, X, target, prec="fp64"):
    """Gradients of the ensemble's loss with respect to every member's
    parameters (a list per member, as backward returns), and the loss."""
    K = len(members)
    grads, losses = [], []
    for k, p in enumerate(members):
        g, loss = backward(p, X, target[:, k:k + 1], prec=prec)
        grads.append([(dW / K, db / K) for dW, db in g])
        losses.append(loss)
    return grads, float(np.mean(losses))


# ------------------------------------------------- physics terms of the loss
#
# Sec. 3.2 adds three physical principles to the loss -- conservation of the
# mass-fraction sum, conservation of energy and the heat release rate --
# without formulas.  Reading used here: each is an L1 penalty on a linear
# functional of the predicted physical change dY_pred = sd u + mu, per
# sample, made dimensionless by the size the functional would have if every
# species were off by one standard deviation of its target:
#   mass    s = sum_k dY_pred,k                    (the sum of Y stays 1)
#   energy  s = sum_k h_k(T1) (dY_pred,k - dY*_k)  (h(T1, Y0 + dY_pred) =
#           h(T1, Y1) = h(T0, Y0): the state keeps the enthalpy of the
#           reference step at its final temperature T1)
#   HRR     s = sum_k h_k(298.15 K) (dY_pred,k - dY*_k)  (the heat released
#           over the step, -rho0/dt sum_k h_f,k dY_k, equals the reference's;
#           the common factor rho0/dt cancels in the scaling)
# with penalty |s| / sum_k |a_k| sd_k (a_k the functional's weights; 1 for
# mass), averaged over the batch and weighted by w = (w_mass, w_energy,
# w_hrr).  h_k in J/kg.

T_REF_HRR = 298.15


def species_enthalpy(om: OracleMech, T):
    """h_k(T) in J/kg of every species at each temperature: [K, N]."""
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    out = np.empty((om.K, T.size))
    for i, t in enumerate(T):
        _, hRT, _ = thermo(om, t)
        out[:, i] = RGAS * t * hRT / om.mech.W
    return out


def physics_terms(u, target, mu_out, sd_out, h_T1, h_ref, w):
    """Physics penalties and their gradient with respect to the network
    output.  u, target: [N, K] z-space; mu_out, sd_out: [K]; h_T1, h_ref:
    [K, N] species enthalpies (J/kg) at the reference step's final
    temperature and at 298.15 K; w: (w_mass, w_energy, w_hrr).  Returns
    (terms, grad): terms = the three batch means of the unweighted
    penalties, grad = d(sum_t w_t terms_t)/du, [N, K]; sign(0) = 0."""
    u = np.asarray(u, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    N, K = u.shape
    sd = np.asarray(sd_out, dtype=np.float64)
    mu = np.asarray(mu_out, dtype=np.float64)
    dY = u * sd[None, :] + mu[None, :]             # predicted change
    e = (u - target) * sd[None, :]                 # its error
    terms = np.zeros(3)
    grad = np.zeros_like(u)
    funcs = [(np.ones((N, K)), dY.sum(axis=1)),
             (h_T1.T, (h_T1.T * e).sum(axis=1)),
             (h_ref.T, (h_ref.T * e).sum(axis=1))]
    for t, (a, s) in enumerate(funcs):
        D = (np.abs(a) * sd[None, :]).sum(axis=1)
        terms[t] = np.mean(np.abs(s) / D)
        grad += w[t] * np.sign(s)[:, None] * a * sd[None, :] / (D[:, None] * N)
    return terms, grad


def backward_phys(params, X, target, mu_out, sd_out, h_T1, h_ref, w, prec="fp64"):
    """backward() for the loss L1 + sum_t w_t terms_t: the same layer
    recursion, started from dL/du = sign(u - u*)/(N K) + the physics
    gradient.  Returns (grads, total loss, L1 loss, terms)."""
    L = len(params)
    u, zs, hs = forward(params, X, prec=prec, keep=True)
    N, nout = u.shape
    terms, gphys = physics_terms(u, target, mu_out, sd_out, h_T1, h_ref, w)
    g = np.sign(u - target) / (N * nout) + gphys
    grads = [None] * L
    for l in range(L - 1, -1, -1):
        W, _ = params[l]
        gq = round_bf16(g) if prec != "fp64" else g
        dW = gq.T @ hs[l]
        db = g.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            Wq = round_bf16(W) if prec != "fp64" else W
            dh = gq @ Wq
            g = dh * gelu_grad(zs[l - 1])
    l1 = l1_loss(u, target)
    return grads, l1 + float(np.dot(w, terms)), l1, terms


def adam_update(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015, Algorithm 1) with bias correction; t >= 1.
    Returns new (params, m, v)."""
    new_p, new_m, new_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for th, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = beta1 * mm + (1 - beta1) * g
            vv = beta2 * vv + (1 - beta2) * g * g
            mh = mm / (1 - beta1 ** t)
            vh = vv / (1 - beta2 ** t)
            th = th - lr * mh / (np.sqrt(vh) + eps)
            out.append((th, mm, vv))
        new_p.append((out[0][0], out[1][0]))
        new_m.append((out[0][1], out[1][1]))
        new_v.append((out[0][2], out[1][2]))
    return new_p, new_m, new_v


# ------------------------------------------------------------------- post


def element_mass_matrix(mech):
    """M[e, k] = (atoms of e in k) * A_e / W_k: element-e mass per unit Y_k."""
    return mech.comp.T.astype(np.float64) * mech.awt[:, None] / mech.W[None, :]


def project(mech, Y0, Yp, sd, floor=1e-10):
    """Weighted least-squares projection of Yp ([K, N]) onto the element
    conservation constraints M Y = M Y0:
    Y = Yp + D M^T (M D M^T)^-1 (M Y0 - M Yp), the minimiser of
    sum_k (Y_k - Yp_k)^2 / d_k under the constraints.  The weight of species k
    is the expected variance of the network's error in its change, sd_k^2
    (sd = the training targets' standard deviations), tapered to zero as the
    species' own mass fraction Y+ = max(Yp, 0) vanishes:
    d_k = sd_k^2 (Y+_k + floor) / (Y+_k + sd_k).  The paper has no
    projection; this weighting is the project's reading (a correction spread
    in proportion to Y itself moved most of an element's residual onto the
    most abundant species, whatever the accuracy of its predicted change)."""
    M = element_mass_matrix(mech)
    sd = np.asarray(sd, dtype=np.float64)
    out = np.empty_like(Yp)
    for i in range(Yp.shape[1]):
        yp = np.maximum(Yp[:, i], 0.0)
        d = sd * sd * (yp + floor) / (yp + sd)
        A = (M * d[None, :]) @ M.T
        r = M @ Y0[:, i] - M @ Yp[:, i]
        lam = np.linalg.solve(A, r)
        out[:, i] = Yp[:, i] + d * (M.T @ lam)
    return out


def temperature_newton(om: OracleMech, T0, Y0, Y, tol=1e-9, maxit=20):
    """Solve h(T, Y) = h(T0, Y0) for T by Newton from T0 (FP64)."""
    T = np.array(T0, dtype=np.float64).copy()
    for i in range(T.size):
        h0 = mixture_enthalpy(om, T0[i], Y0[:, i])
        t = T0[i]
        for _ in range(maxit):
            cpR, _, _ = thermo(om, t)
            cp = float(np.sum(Y[:, i] * RGAS * cpR / om.mech.W))
            dT = (mixture_enthalpy(om, t, Y[:, i]) - h0) / cp
            t = t - dT
            if abs(dT) < tol * t:
                break
        T[i] = t
    return T


def density(mech, T, p, Y):
    S = (Y / mech.W[:, None]).sum(axis=0)
    return p / (RGAS * T * S)


def ood_flags(feat, lo, hi, margin=0.05):
    """feat: raw features [F, N]; lo/hi: training-set range per feature.  A
    cell is out of distribution when any feature lies outside [lo - tol,
    hi + tol] with tol = margin * (hi - lo), or, for a feature of zero
    spread, tol = 1e-6 |hi|.  A non-finite feature is outside."""
    span = hi - lo
    tol = np.where(span > 0, margin * span, 1e-6 * np.maximum(np.abs(hi), 1e-30))
    inside = (feat >= (lo - tol)[:, None]) & (feat <= (hi + tol)[:, None])
    return (~inside).any(axis=0)


def post(om: OracleMech, T0, p, Y0, u_z, mu_out, sd_out, dt, lo=None, hi=None,
         residual_tol=1e-6, margin=0.05, lam=LAMBDA):
    """From the z-space network output u_z ([K, N]) to (T, Y, RR, flags).

    Flag bit 1 (value 2) judges the network itself: it is set when the
    element residual of the network's own state Y' = Y0 + dY, max_e
    |(M Y')_e - (M Y0)_e|, exceeds residual_tol, and also when the projected
    and clipped state still misses element conservation by more than that
    (the projection removes the first residual exactly unless clipping at 0
    breaks it).  A non-finite residual counts as exceeding."""
    mech = om.mech
    du = u_z * sd_out[:, None] + mu_out[:, None]
    Yp = Y0 + du
    Y = project(mech, Y0, Yp, sd_out)
    Y = np.maximum(Y, 0.0)
    M = element_mass_matrix(mech)
    res_raw = np.abs(M @ Yp - M @ Y0).max(axis=0)
    res = np.abs(M @ Y - M @ Y0).max(axis=0)
    flags = np.zeros(T0.size, dtype=np.uint8)
    if lo is not None:
        flags |= np.where(ood_flags(features(T0, p, Y0, lam), lo, hi, margin), 1, 0).astype(np.uint8)
    bad = ~((res_raw <= residual_tol) & (res <= residual_tol))
    flags |= np.where(bad, 2, 0).astype(np.uint8)
    T = temperature_newton(om, T0, Y0, Y)
    rho0 = density(mech, T0, p, Y0)
    RR = rho0[None, :] * (Y - Y0) / dt
    return dict(T=T, Y=Y, RR=RR, flags=flags, residual=res, residual_raw=res_raw, Yp=Yp,
                rho0=rho0)
