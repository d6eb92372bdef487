/*
 * chem_oracle.c -- plain, slow, scalar FP64 CPU oracle for the per-cell
 * chemistry step (paper Sec. 3.1: each composition is integrated over one
 * chemistry time step to give an input/output pair; the reaction ODE maps
 * (Y, T, p) to rates).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header or constant table with the HIP library.
 *
 * Everything is written one cell at a time, in the order the definitions are
 * stated, with no blocking or reordering:
 *   - NASA-7 polynomials (McBride, Gordon & Reno, NASA TM-4513);
 *   - mass-action kinetics of reversible elementary reactions, forward rate
 *     constant A T^b exp(-Ea/RT) evaluated in log space, reverse rate constant
 *     k_f / K_c with K_c from the standard Gibbs energies;
 *   - the adiabatic constant-pressure reactor: state y = [T, Y_1..Y_K],
 *     dY_k/dt = W_k wdot_k / rho, dT/dt = -sum_k H_k wdot_k / (rho c_p);
 *   - its exact analytic Jacobian (chain rule through rho, C_k and c_p);
 *   - LU with partial pivoting; pivot = un-eliminated row with the largest
 *     |a_ik|, ties to the lowest row index; rows are not moved;
 *   - the 4-stage L-stable Rosenbrock method RODAS3 (Sandu et al., Atmos.
 *     Environ. 31:3459, 1997) in the transformed form of Hairer & Wanner,
 *     Solving ODEs II, Sec. IV.7, with an embedded order-2 error estimate and
 *     the step-size controller documented at or_integrate();
 *   - classic fixed-step RK4 as a brute-force cross-check.
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_RGAS 8.314462618   /* J/(mol K) */
#define OR_PREF 101325.0      /* standard-state pressure, Pa */
#define OR_KMAX 64
#define OR_RMAX 1024
#define OR_NMAX (OR_KMAX + 1)

enum { OR_OK = 0, OR_MAX_STEPS = 1, OR_H_UNDERFLOW = 2, OR_NONFINITE = 3, OR_SINGULAR = 4 };

typedef struct {
  int K, R;
  const double *W;     /* [K] kg/mol */
  const double *nasa;  /* [K][17]: Tlow, Tmid, Thigh, low a1..a7, high a1..a7 */
  const int *rsp;      /* [R][4]: reactant0, reactant1, product0, product1 (-1 none) */
  const int *rnu;      /* [R][4]: stoichiometric coefficients of those slots */
  const double *A;     /* [R] SI */
  const double *b;     /* [R] */
  const double *Ea;    /* [R] J/mol */
} or_mech;

typedef struct {
  double rtol, atol_Y, atol_T, h0, h_min;
  int max_steps;
} or_opts;

/* ---------------------------------------------------------------- thermo */

/* c_p/R, h/(RT), s/R and d(c_p/R)/dT of species k at temperature T. */
void or_species_thermo(const or_mech *m, int k, double T, double *cpR, double *hRT,
                       double *sR, double *dcpR) {
  const double *c = m->nasa + 17 * k;
  const double *a = (T <= c[1]) ? c + 3 : c + 10;
  double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
  *cpR = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
  *hRT = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
  *sR = a[0] * log(T) + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
  *dcpR = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T2 + 4.0 * a[4] * T3;
}

/* all species at one T (arrays of length K) */
void or_thermo(const or_mech *m, double T, double *cpR, double *hRT, double *sR) {
  for (int k = 0; k < m->K; ++k) {
    double d;
    or_species_thermo(m, k, T, &cpR[k], &hRT[k], &sR[k], &d);
  }
}

/* mixture specific enthalpy (J/kg) */
double or_mixture_enthalpy(const or_mech *m, double T, const double *Y) {
  double h = 0.0;
  for (int k = 0; k < m->K; ++k) {
    double cpR, hRT, sR, d;
    or_species_thermo(m, k, T, &cpR, &hRT, &sR, &d);
    h += Y[k] * OR_RGAS * T * hRT / m->W[k];
  }
  return h;
}

/* ------------------------------------------------------- kinetics + RHS */

/* Right-hand side of the constant-pressure adiabatic reactor at state
 * y = [T, Y_1..Y_K] and pressure p.  Optional outputs: wdot[K] (mol/m^3/s),
 * kf[R], kr[R] (SI), and the Jacobian J[n*n] (row i = d f_i / d y_j). */
void or_eval(const or_mech *m, double p, const double *y, double *f, double *wdot_out,
             double *kf_out, double *kr_out, double *J) {
  const int K = m->K, R = m->R, n = K + 1;
  const double T = y[0];
  const double *Y = y + 1;
  double cpR[OR_KMAX], hRT[OR_KMAX], sR[OR_KMAX], dcpR[OR_KMAX], gRT[OR_KMAX];
  double C[OR_KMAX], wdot[OR_KMAX], H[OR_KMAX];

  double S = 0.0;
  for (int k = 0; k < K; ++k) S += Y[k] / m->W[k];
  const double rho = p / (OR_RGAS * T * S);
  double cp = 0.0, dcpdT = 0.0;
  for (int k = 0; k < K; ++k) {
    or_species_thermo(m, k, T, &cpR[k], &hRT[k], &sR[k], &dcpR[k]);
    gRT[k] = hRT[k] - sR[k];
    H[k] = OR_RGAS * T * hRT[k];
    C[k] = rho * Y[k] / m->W[k];
    cp += Y[k] * OR_RGAS * cpR[k] / m->W[k];
    dcpdT += Y[k] * OR_RGAS * dcpR[k] / m->W[k];
    wdot[k] = 0.0;
  }

  double *dwdC = NULL, *dwdT = NULL;
  if (J) {
    dwdC = (double *)calloc((size_t)K * K, sizeof(double));
    dwdT = (double *)calloc((size_t)K, sizeof(double));
  }

  const double lnT = log(T);
  const double ln_pref_RT = log(OR_PREF / (OR_RGAS * T));
  for (int r = 0; r < R; ++r) {
    const int *sp = m->rsp + 4 * r;
    const int *nu = m->rnu + 4 * r;
    double dG = 0.0, dH = 0.0;
    int dn = 0;
    for (int s = 0; s < 4; ++s) {
      if (sp[s] < 0) continue;
      double sign = (s < 2) ? -1.0 : 1.0;
      dG += sign * nu[s] * gRT[sp[s]];
      dH += sign * nu[s] * hRT[sp[s]];
      dn += (s < 2) ? -nu[s] : nu[s];
    }
    const double lnkf = log(m->A[r]) + m->b[r] * lnT - m->Ea[r] / (OR_RGAS * T);
    const double lnKc = -dG + dn * ln_pref_RT;
    const double kf = exp(lnkf);
    const double kr = exp(lnkf - lnKc);
    if (kf_out) kf_out[r] = kf;
    if (kr_out) kr_out[r] = kr;
    /* concentration factors C^nu of each slot (1 for an empty slot) */
    double fac[4];
    for (int s = 0; s < 4; ++s) {
      if (sp[s] < 0) fac[s] = 1.0;
      else fac[s] = (nu[s] == 2) ? C[sp[s]] * C[sp[s]] : C[sp[s]];
    }
    const double fwd = kf * fac[0] * fac[1];
    const double rev = kr * fac[2] * fac[3];
    const double q = fwd - rev;
    for (int s = 0; s < 4; ++s) {
      if (sp[s] < 0) continue;
      if (s < 2) wdot[sp[s]] -= nu[s] * q;
      else wdot[sp[s]] += nu[s] * q;
    }
    if (J) {
      /* dq/dC_j of each participating species (slots are distinct species) */
      double dq[4];
      for (int s = 0; s < 4; ++s) {
        if (sp[s] < 0) { dq[s] = 0.0; continue; }
        double dfac = (nu[s] == 2) ? 2.0 * C[sp[s]] : 1.0;
        if (s == 0) dq[s] = kf * dfac * fac[1];
        else if (s == 1) dq[s] = kf * fac[0] * dfac;
        else if (s == 2) dq[s] = -kr * dfac * fac[3];
        else dq[s] = -kr * fac[2] * dfac;
      }
      /* dq/dT at fixed concentrations: d ln kf/dT = b/T + Ea/(R T^2);
         d ln Kc/dT = dH_r/(R T^2) - dn/T  (van 't Hoff) */
      const double dlnkf = m->b[r] / T + m->Ea[r] / (OR_RGAS * T * T);
      const double dlnKc = dH / T - dn / T;
      const double dqdT = fwd * dlnkf - rev * (dlnkf - dlnKc);
      for (int s = 0; s < 4; ++s) {
        if (sp[s] < 0) continue;
        const int k = sp[s];
        const double nuk = (s < 2) ? -(double)nu[s] : (double)nu[s];
        for (int t = 0; t < 4; ++t) {
          if (sp[t] < 0) continue;
          dwdC[k * K + sp[t]] += nuk * dq[t];
        }
        dwdT[k] += nuk * dqdT;
      }
    }
  }

  double Q = 0.0;
  for (int k = 0; k < K; ++k) Q += H[k] * wdot[k];
  f[0] = -Q / (rho * cp);
  for (int k = 0; k < K; ++k) f[1 + k] = m->W[k] * wdot[k] / rho;
  if (wdot_out)
    for (int k = 0; k < K; ++k) wdot_out[k] = wdot[k];

  if (J) {
    const double fT = f[0];
    /* d wdot_k / d Y_i and d wdot_k / d T through C_j(rho(T, Y), Y):
       dC_j/dY_i = rho delta_ij / W_j - C_j / (S W_i),  dC_j/dT = -C_j / T */
    double *dwdY = (double *)calloc((size_t)K * K, sizeof(double));
    double dwdTt[OR_KMAX];
    for (int k = 0; k < K; ++k) {
      double a = 0.0;
      for (int j = 0; j < K; ++j) a += dwdC[k * K + j] * C[j];
      for (int i = 0; i < K; ++i) dwdY[k * K + i] = (rho * dwdC[k * K + i] - a / S) / m->W[i];
      dwdTt[k] = dwdT[k] - a / T;
    }
    /* species rows */
    for (int k = 0; k < K; ++k) {
      J[(1 + k) * n + 0] = (m->W[k] / rho) * dwdTt[k] + m->W[k] * wdot[k] / (rho * T);
      for (int i = 0; i < K; ++i)
        J[(1 + k) * n + 1 + i] =
            (m->W[k] / rho) * dwdY[k * K + i] + m->W[k] * wdot[k] / (rho * S * m->W[i]);
    }
    /* temperature row */
    double sT = 0.0;
    for (int k = 0; k < K; ++k) sT += OR_RGAS * cpR[k] * wdot[k] + H[k] * dwdTt[k];
    J[0] = -sT / (rho * cp) - fT * (-1.0 / T + dcpdT / cp);
    for (int i = 0; i < K; ++i) {
      double s = 0.0;
      for (int k = 0; k < K; ++k) s += H[k] * dwdY[k * K + i];
      J[1 + i] = -s / (rho * cp) - fT * (-1.0 / (S * m->W[i]) + OR_RGAS * cpR[i] / (m->W[i] * cp));
    }
    free(dwdY);
    free(dwdC);
    free(dwdT);
  }
}

void or_rhs(const or_mech *m, double p, const double *y, double *f) {
  or_eval(m, p, y, f, NULL, NULL, NULL, NULL);
}

void or_jacobian(const or_mech *m, double p, const double *y, double *J) {
  double f[OR_NMAX];
  or_eval(m, p, y, f, NULL, NULL, NULL, J);
}

/* Instantaneous rates for N cells (SoA, leading dimension ld). */
void or_chem_rates(const or_mech *m, long N, long ld, const double *T, const double *p,
                   const double *Y, double *wdot, double *dTdt, double *kf, double *kr) {
  const int K = m->K, R = m->R;
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < N; ++i) {
    double y[OR_NMAX], f[OR_NMAX], w[OR_KMAX], kfl[OR_RMAX], krl[OR_RMAX];
    y[0] = T[i];
    for (int k = 0; k < K; ++k) y[1 + k] = Y[k * ld + i];
    or_eval(m, p[i], y, f, w, kfl, krl, NULL);
    for (int k = 0; k < K; ++k) wdot[k * ld + i] = w[k];
    if (dTdt) dTdt[i] = f[0];
    if (kf)
      for (int r = 0; r < R; ++r) kf[r * ld + i] = kfl[r];
    if (kr)
      for (int r = 0; r < R; ++r) kr[r * ld + i] = krl[r];
  }
}

/* ------------------------------------------------------------------- LU */

/* In-place LU of the row-major n x n matrix a.  At step k the pivot is the
 * not-yet-eliminated row with the largest |a[i][k]| (ties: lowest row index;
 * NaN counts as larger than any number); order[k] records it.  Rows stay where they are: the multiplier of row i at
 * step k is stored in a[i][k].  Returns 0, or 1 if a pivot is zero/non-finite. */
int or_lu(int n, double *a, int *order) {
  int done[OR_NMAX];
  for (int i = 0; i < n; ++i) done[i] = 0;
  for (int k = 0; k < n; ++k) {
    int best = -1;
    double bestv = 0.0;
    for (int i = 0; i < n; ++i) {
      if (done[i]) continue;
      double v = fabs(a[i * n + k]);
      if (isnan(v)) v = INFINITY; /* a NaN candidate wins and then fails the check below */
      if (best < 0 || v > bestv) { best = i; bestv = v; }
    }
    if (!(bestv > 0.0) || !isfinite(bestv)) return 1;
    order[k] = best;
    done[best] = 1;
    const double piv = a[best * n + k];
    for (int i = 0; i < n; ++i) {
      if (done[i]) continue;
      const double l = a[i * n + k] / piv;
      a[i * n + k] = l;
      for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[best * n + j];
    }
  }
  return 0;
}

/* Solve A x = b with the factors from or_lu; b is overwritten by x. */
void or_lu_solve(int n, const double *a, const int *order, double *b) {
  double z[OR_NMAX];
  for (int k = 0; k < n; ++k) {
    const int i = order[k];
    double s = b[i];
    for (int j = 0; j < k; ++j) s -= a[i * n + j] * z[j];
    z[k] = s;
  }
  for (int k = n - 1; k >= 0; --k) {
    const int i = order[k];
    double s = z[k];
    for (int j = k + 1; j < n; ++j) s -= a[i * n + j] * b[j];
    b[k] = s / a[i * n + k];
  }
}

/* ------------------------------------------------------------ Rosenbrock */

/* RODAS3 in the transformed form: for stage i,
 *   (I/(gamma h) - J) K_i = f(y + sum_{j<i} a_ij K_j) + (1/h) sum_{j<i} c_ij K_j,
 *   y_new = y + sum_i m_i K_i,   error estimate = sum_i e_i K_i.
 * Stage 2 has the same argument as stage 1 (a_21 = 0) and reuses its f. */
#define ROS_S 4
static const double ROS_GAMMA = 0.5;
static const double ROS_A[ROS_S][ROS_S] = {
    {0, 0, 0, 0}, {0, 0, 0, 0}, {2.0, 0, 0, 0}, {2.0, 0, 1.0, 0}};
static const double ROS_C[ROS_S][ROS_S] = {
    {0, 0, 0, 0}, {4.0, 0, 0, 0}, {1.0, -1.0, 0, 0}, {1.0, -1.0, -8.0 / 3.0, 0}};
static const int ROS_NEWF[ROS_S] = {1, 0, 1, 1};
static const double ROS_M[ROS_S] = {2.0, 0.0, 1.0, 1.0};
static const double ROS_E[ROS_S] = {0.0, 0.0, 0.0, 1.0};

/* copy out the tableau (tests check its order conditions) */
void or_ros_tableau(double *gamma, double *A, double *Cc, double *Mv, double *Ev, int *newf) {
  *gamma = ROS_GAMMA;
  for (int i = 0; i < ROS_S; ++i) {
    for (int j = 0; j < ROS_S; ++j) {
      A[i * ROS_S + j] = ROS_A[i][j];
      Cc[i * ROS_S + j] = ROS_C[i][j];
    }
    Mv[i] = ROS_M[i];
    Ev[i] = ROS_E[i];
    newf[i] = ROS_NEWF[i];
  }
}

typedef void (*or_rhs_fn)(void *ctx, const double *y, double *f);
typedef void (*or_jac_fn)(void *ctx, const double *y, double *f, double *J);

/* One Rosenbrock step of size h from y (size n), writing the new solution and
 * the error vector.  f0/J are evaluated at y by jac().  Returns 0 or 1 (LU
 * failed). */
static int ros_step(int n, or_rhs_fn rhs, or_jac_fn jac, void *ctx, const double *y, double h,
                    double *ynew, double *errv) {
  double Mx[OR_NMAX * OR_NMAX];
  int order[OR_NMAX];
  double Kst[ROS_S][OR_NMAX], F[OR_NMAX], Ys[OR_NMAX], rhsv[OR_NMAX];
  jac(ctx, y, F, Mx);
  const double dg = 1.0 / (ROS_GAMMA * h);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) Mx[i * n + j] = -Mx[i * n + j];
    Mx[i * n + i] += dg;
  }
  if (or_lu(n, Mx, order)) return 1;
  for (int s = 0; s < ROS_S; ++s) {
    if (s > 0 && ROS_NEWF[s]) {
      for (int i = 0; i < n; ++i) {
        double v = y[i];
        for (int j = 0; j < s; ++j) v += ROS_A[s][j] * Kst[j][i];
        Ys[i] = v;
      }
      rhs(ctx, Ys, F);
    }
    for (int i = 0; i < n; ++i) {
      double c = 0.0;
      for (int j = 0; j < s; ++j) c += ROS_C[s][j] * Kst[j][i];
      rhsv[i] = F[i] + c / h;
    }
    or_lu_solve(n, Mx, order, rhsv);
    for (int i = 0; i < n; ++i) Kst[s][i] = rhsv[i];
  }
  for (int i = 0; i < n; ++i) {
    double v = y[i], e = 0.0;
    for (int s = 0; s < ROS_S; ++s) {
      v += ROS_M[s] * Kst[s][i];
      e += ROS_E[s] * Kst[s][i];
    }
    ynew[i] = v;
    errv[i] = e;
  }
  return 0;
}

/* Fixed-size single step on an arbitrary problem given by callbacks (tests of
 * the method's order).  yemb receives the embedded solution ynew - errv. */
int or_ros_step_generic(int n, or_rhs_fn rhs, or_jac_fn jac, void *ctx, const double *y,
                        double h, double *ynew, double *yemb) {
  double e[OR_NMAX];
  int st = ros_step(n, rhs, jac, ctx, y, h, ynew, e);
  for (int i = 0; i < n; ++i) yemb[i] = ynew[i] - e[i];
  return st;
}

typedef struct {
  const or_mech *m;
  double p;
} chem_ctx;

static void chem_rhs_cb(void *c, const double *y, double *f) {
  chem_ctx *x = (chem_ctx *)c;
  or_eval(x->m, x->p, y, f, NULL, NULL, NULL, NULL);
}
static void chem_jac_cb(void *c, const double *y, double *f, double *J) {
  chem_ctx *x = (chem_ctx *)c;
  or_eval(x->m, x->p, y, f, NULL, NULL, NULL, J);
}

/* Adaptive integration of one cell over [0, dt].
 *   weights  sc_i = atol_i + rtol * max(|y_i|, |ynew_i|)  (atol_T for T, atol_Y else)
 *   err      = sqrt( (1/n) sum_i (errv_i / sc_i)^2 )
 *   accept   if err <= 1; a non-finite err is a rejection with factor 0.2
 *   factor   fac = 0.9 err^(-1/3) (fac_max if err == 0), clamped to [0.2, fac_max];
 *            fac_max = 6, or 1 for the step right after a rejection
 *   start    h = min(dt, h_hint) if a hint > 0 is given, else min(dt, h0)
 *   last     the step is cut to dt - t when h >= dt - t; accepting it sets t = dt
 *   failure  more than max_steps attempts -> MAX_STEPS; h < h_min -> H_UNDERFLOW;
 *            non-finite input, T <= 0, p <= 0 or dt <= 0 -> NONFINITE;
 *            zero or non-finite pivot -> SINGULAR
 * No clipping of negative mass fractions.  On return y holds the result (or is
 * unchanged on failure), *h_io the proposed next step size. */
int or_integrate(const or_mech *m, double p, double *y, double dt, const or_opts *o,
                 double *h_io, int *nacc_out, int *nrej_out) {
  const int n = m->K + 1;
  int nacc = 0, nrej = 0;
  *nacc_out = 0;
  *nrej_out = 0;
  for (int i = 0; i < n; ++i)
    if (!isfinite(y[i])) return OR_NONFINITE;
  if (!(y[0] > 0.0) || !isfinite(p) || !(p > 0.0) || !(dt > 0.0) || !isfinite(dt))
    return OR_NONFINITE;
  chem_ctx ctx = {m, p};
  double yw[OR_NMAX], ynew[OR_NMAX], errv[OR_NMAX];
  for (int i = 0; i < n; ++i) yw[i] = y[i];
  double h = (h_io && *h_io > 0.0) ? *h_io : o->h0;
  if (h > dt) h = dt;
  double t = 0.0, fac_max = 6.0;
  int status = OR_OK;
  while (t < dt) {
    if (nacc + nrej >= o->max_steps) { status = OR_MAX_STEPS; break; }
    int last = 0;
    if (h >= dt - t) { h = dt - t; last = 1; }
    if (h < o->h_min) { status = OR_H_UNDERFLOW; break; }
    if (ros_step(n, chem_rhs_cb, chem_jac_cb, &ctx, yw, h, ynew, errv)) {
      status = OR_SINGULAR;
      break;
    }
    double ss = 0.0;
    for (int i = 0; i < n; ++i) {
      const double atol = (i == 0) ? o->atol_T : o->atol_Y;
      const double sc = atol + o->rtol * fmax(fabs(yw[i]), fabs(ynew[i]));
      const double r = errv[i] / sc;
      ss += r * r;
    }
    const double err = sqrt(ss / n);
    if (isfinite(err) && err <= 1.0) {
      for (int i = 0; i < n; ++i) yw[i] = ynew[i];
      t = last ? dt : t + h;
      ++nacc;
      double fac = (err > 0.0) ? 0.9 * pow(err, -1.0 / 3.0) : fac_max;
      fac = fmin(fac_max, fmax(0.2, fac));
      h *= fac;
      fac_max = 6.0;
    } else {
      ++nrej;
      double fac = isfinite(err) ? 0.9 * pow(err, -1.0 / 3.0) : 0.2;
      fac = fmin(1.0, fmax(0.2, fac));
      h *= fac;
      fac_max = 1.0;
    }
  }
  *nacc_out = nacc;
  *nrej_out = nrej;
  if (status == OR_OK) {
    for (int i = 0; i < n; ++i) y[i] = yw[i];
    if (h_io) *h_io = h;
  }
  return status;
}

/* Batched chemistry step over N cells (SoA, leading dimension ld).
 * dt_cell (nullable) overrides dt per cell.  T and Y are updated in place;
 * RR (nullable, [K][ld]) receives rho(T0, Y0) (Y - Y0) / dt in kg/m^3/s;
 * h_hint (nullable) is read and written; stats (nullable, [3][ld]) receives
 * n_acc, n_rej, status.  Failed cells keep their input state and get RR = 0. */
void or_chem_step(const or_mech *m, long N, long ld, double dt, const double *dt_cell,
                  double *T, const double *p, double *Y, double *RR, double *h_hint,
                  int *stats, const or_opts *o, int nthreads) {
  const int K = m->K;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < N; ++i) {
    double y[OR_NMAX], y0[OR_NMAX];
    y[0] = T[i];
    for (int k = 0; k < K; ++k) y[1 + k] = Y[k * ld + i];
    for (int j = 0; j <= K; ++j) y0[j] = y[j];
    const double dti = dt_cell ? dt_cell[i] : dt;
    double h = h_hint ? h_hint[i] : 0.0;
    int nacc = 0, nrej = 0;
    int st = or_integrate(m, p[i], y, dti, o, &h, &nacc, &nrej);
    if (st == OR_OK) {
      T[i] = y[0];
      for (int k = 0; k < K; ++k) Y[k * ld + i] = y[1 + k];
      if (h_hint) h_hint[i] = h;
    }
    if (RR) {
      double S = 0.0;
      for (int k = 0; k < K; ++k) S += y0[1 + k] / m->W[k];
      const double rho0 = p[i] / (OR_RGAS * y0[0] * S);
      for (int k = 0; k < K; ++k)
        RR[k * ld + i] = (st == OR_OK) ? rho0 * (y[1 + k] - y0[1 + k]) / dti : 0.0;
    }
    if (stats) {
      stats[0 * ld + i] = nacc;
      stats[1 * ld + i] = nrej;
      stats[2 * ld + i] = st;
    }
  }
}

/* Classic RK4 with nsteps fixed steps over [0, dt] (brute-force check). */
void or_rk4(const or_mech *m, double p, double *y, double dt, long nsteps) {
  const int n = m->K + 1;
  const double h = dt / (double)nsteps;
  double k1[OR_NMAX], k2[OR_NMAX], k3[OR_NMAX], k4[OR_NMAX], yt[OR_NMAX];
  for (long s = 0; s < nsteps; ++s) {
    or_rhs(m, p, y, k1);
    for (int i = 0; i < n; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
    or_rhs(m, p, yt, k2);
    for (int i = 0; i < n; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
    or_rhs(m, p, yt, k3);
    for (int i = 0; i < n; ++i) yt[i] = y[i] + h * k3[i];
    or_rhs(m, p, yt, k4);
    for (int i = 0; i < n; ++i) y[i] += h * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]) / 6.0;
  }
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
