// FP64 chemistry kernels for gfx950: instantaneous rates and the adaptive
// RODAS3 step of the adiabatic constant-pressure reactor.
//
// Mapping.  A cell is handled by a group of G lanes (G = 16, 32 or 64, the
// smallest power of two >= n = K + 1), so a 64-wide wavefront carries 64/G
// cells.  Lane l of a group owns component l of the state y = [T, Y_1..Y_K]
// (lane 0 is T) and, during the linear algebra, row l of the Newton matrix
// M = I/(gamma h) - J, held in registers.  Reactions are spread over the
// lanes of the group (lane l takes r = l, l+G, ...); species lanes gather
// their net production rate from the per-reaction rates of progress in LDS
// through a fixed per-species reaction list in ascending reaction order.
// Every cross-lane exchange stays inside one wavefront (DS permutes for
// broadcasts and butterflies, LDS for gathers), so no workgroup barrier is
// needed and groups may diverge freely.
//
// Scheduling.  The step kernel is persistent: every group takes a cell from a
// device-wide atomic counter, integrates it with per-cell adaptive substeps,
// writes it back and takes the next one, so cells that need many substeps do
// not hold up the lanes of cheap ones.  The wave ends when the counter runs
// past the last cell; every group reaches that exit.
#include <math.h>

#include "chem_internal.h"

namespace chem {
namespace {

constexpr double RG = 8.314462618;  // J/(mol K)
constexpr double PREF = 101325.0;   // Pa

// RODAS3 (Sandu et al. 1997), transformed form (Hairer & Wanner IV.7):
// (I/(gamma h) - J) K_i = f(y + sum_j a_ij K_j) + (1/h) sum_j c_ij K_j.
constexpr double GAMMA = 0.5;
constexpr double TA[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {2.0, 0, 0, 0}, {2.0, 0, 1.0, 0}};
constexpr double TC[4][4] = {{0, 0, 0, 0}, {4.0, 0, 0, 0}, {1.0, -1.0, 0, 0},
                             {1.0, -1.0, -8.0 / 3.0, 0}};
constexpr bool TNEWF[4] = {true, false, true, true};
constexpr double TM[4] = {2.0, 0.0, 1.0, 1.0};
constexpr double TE[4] = {0.0, 0.0, 0.0, 1.0};

enum { CELL_OK = 0, CELL_MAX_STEPS = 1, CELL_H_UNDERFLOW = 2, CELL_NONFINITE = 3,
       CELL_SINGULAR = 4 };

// Orders LDS accesses between lanes of one wavefront.  DS instructions of a
// wave execute in issue order, so this only has to stop the compiler from
// moving accesses across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ __forceinline__ double grp_sum(double v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

template <int G>
__device__ __forceinline__ bool grp_any(bool b) {
  int v = b ? 1 : 0;
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v |= __shfl_xor(v, off, G);
  return v != 0;
}

// Per-group LDS scratch (doubles).
template <int G>
struct GLds {
  double *C, *hs, *gs, *qs, *dHs, *kfs, *krs, *dqdTs, *J;
  __device__ GLds(double *base, int R) {
    C = base;
    hs = C + G;
    gs = hs + G;
    qs = gs + G;
    dHs = qs + R;
    kfs = dHs + R;
    krs = kfs + R;
    dqdTs = krs + R;
    J = dqdTs + R;
  }
  static constexpr int JS = G + 1;  // row stride of J (odd, spreads banks)
  __host__ __device__ static size_t doubles(int R) {
    return 3 * G + 5 * (size_t)R + (size_t)G * JS;
  }
};

__device__ __forceinline__ double slot_fac(int s, int nu, const double *C) {
  if (s < 0) return 1.0;
  const double c = C[s];
  return nu == 2 ? c * c : c;
}

// Right-hand side (and optionally the Jacobian) of one cell.  Lane l holds
// y_l in yl.  On return lane l holds f_l; species lanes hold wdot_k in wdl.
// With JAC, lane l < n holds row l of M = I*dg - J in m[0..G-1]; lanes >= n
// hold identity rows.  With KOUT the rate constants stay in L.kfs / L.krs.
template <int G, bool JAC, bool KOUT>
__device__ __forceinline__ void eval_cell(const DevMech &M, const GLds<G> &L, int l, double p,
                                          double yl, double &f, double &wdl, double (&m)[G],
                                          double dg) {
  const int K = M.K, R = M.R, n = M.n;
  const double T = __shfl(yl, 0, G);
  const double lnT = log(T);
  const bool isSp = (l >= 1) && (l <= K);
  const int k = isSp ? l - 1 : 0;
  double cpR = 0.0, hRT = 0.0, sR = 0.0, dcpR = 0.0, Wk = 1.0, Yk = 0.0;
  if (isSp) {
    Wk = M.W[k];
    Yk = yl;
    const double *a = (T <= M.Tmid[k]) ? M.nasa_lo + 7 * k : M.nasa_hi + 7 * k;
    const double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    cpR = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
    hRT = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
    sR = a[0] * lnT + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
    if (JAC) dcpR = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T2 + 4.0 * a[4] * T3;
  }
  const double S = grp_sum<G>(Yk / Wk);
  const double rho = p / (RG * T * S);
  const double Ck = rho * Yk / Wk;
  const double cp = grp_sum<G>(Yk * RG * cpR / Wk);
  if (isSp) {
    L.C[k] = Ck;
    L.hs[k] = hRT;
    L.gs[k] = hRT - sR;
  }
  wave_sync();

  const double lnPRT = log(PREF / (RG * T));
  double sumHq = 0.0;
  for (int r = l; r < R; r += G) {
    const int4 sp = M.sp[r];
    const int4 nu = M.nu[r];
    double dG = 0.0, dH = 0.0;
    if (sp.x >= 0) { dG -= nu.x * L.gs[sp.x]; dH -= nu.x * L.hs[sp.x]; }
    if (sp.y >= 0) { dG -= nu.y * L.gs[sp.y]; dH -= nu.y * L.hs[sp.y]; }
    if (sp.z >= 0) { dG += nu.z * L.gs[sp.z]; dH += nu.z * L.hs[sp.z]; }
    if (sp.w >= 0) { dG += nu.w * L.gs[sp.w]; dH += nu.w * L.hs[sp.w]; }
    const double dn = M.dn[r];
    const double lnkf = M.lnA[r] + M.b[r] * lnT - M.EaR[r] / T;
    const double lnKc = -dG + dn * lnPRT;
    const double kf = exp(lnkf);
    const double kr = exp(lnkf - lnKc);
    const double fwd = kf * slot_fac(sp.x, nu.x, L.C) * slot_fac(sp.y, nu.y, L.C);
    const double rev = kr * slot_fac(sp.z, nu.z, L.C) * slot_fac(sp.w, nu.w, L.C);
    L.qs[r] = fwd - rev;
    if (JAC || KOUT) {
      L.kfs[r] = kf;
      L.krs[r] = kr;
    }
    if (JAC) {
      const double dlnkf = M.b[r] / T + M.EaR[r] / (T * T);
      const double dlnKc = dH / T - dn / T;
      const double dqdT = fwd * dlnkf - rev * (dlnkf - dlnKc);
      L.dqdTs[r] = dqdT;
      L.dHs[r] = dH;
      sumHq += RG * T * dH * dqdT;
    }
  }
  wave_sync();

  double wd = 0.0;
  if (isSp) {
    const int e1 = M.csr_off[k + 1];
    for (int e = M.csr_off[k]; e < e1; ++e) wd += M.csr_nu[e] * L.qs[M.csr_r[e]];
  }
  wdl = wd;
  const double Q = grp_sum<G>(isSp ? RG * T * hRT * wd : 0.0);
  const double fT = -Q / (rho * cp);
  f = (l == 0) ? fT : (isSp ? Wk * wd / rho : 0.0);
  if (!JAC) return;

  // ---- analytic Jacobian ----
  const double dcpdT = grp_sum<G>(Yk * RG * dcpR / Wk);
  const double sumCpW = grp_sum<G>(isSp ? RG * cpR * wd : 0.0);
  const double sumHqT = grp_sum<G>(sumHq);
  double *Jrow = L.J + l * GLds<G>::JS;
  if (l < n)
    for (int j = 0; j < n; ++j) Jrow[j] = 0.0;
  wave_sync();
  double dwdTC = 0.0, JwT = 0.0;
  if (isSp) {
    // row k of d wdot / d C (scattered into LDS row l) and sum_r dH_r dq_r/dC_k
    const int e1 = M.csr_off[k + 1];
    for (int e = M.csr_off[k]; e < e1; ++e) {
      const int r = M.csr_r[e];
      const double nuk = M.csr_nu[e];
      const int slot = M.csr_slot[e];
      const int4 sp = M.sp[r];
      const int4 nu = M.nu[r];
      const double kf = L.kfs[r], kr = L.krs[r];
      const double f0 = slot_fac(sp.x, nu.x, L.C), f1 = slot_fac(sp.y, nu.y, L.C);
      const double f2 = slot_fac(sp.z, nu.z, L.C), f3 = slot_fac(sp.w, nu.w, L.C);
      double dq0 = 0.0, dq1 = 0.0, dq2 = 0.0, dq3 = 0.0;
      if (sp.x >= 0) dq0 = kf * (nu.x == 2 ? 2.0 * L.C[sp.x] : 1.0) * f1;
      if (sp.y >= 0) dq1 = kf * f0 * (nu.y == 2 ? 2.0 * L.C[sp.y] : 1.0);
      if (sp.z >= 0) dq2 = -kr * (nu.z == 2 ? 2.0 * L.C[sp.z] : 1.0) * f3;
      if (sp.w >= 0) dq3 = -kr * f2 * (nu.w == 2 ? 2.0 * L.C[sp.w] : 1.0);
      if (sp.x >= 0) Jrow[1 + sp.x] += nuk * dq0;
      if (sp.y >= 0) Jrow[1 + sp.y] += nuk * dq1;
      if (sp.z >= 0) Jrow[1 + sp.z] += nuk * dq2;
      if (sp.w >= 0) Jrow[1 + sp.w] += nuk * dq3;
      dwdTC += nuk * L.dqdTs[r];
      const double dqk = slot == 0 ? dq0 : (slot == 1 ? dq1 : (slot == 2 ? dq2 : dq3));
      JwT += RG * T * L.dHs[r] * dqk;
    }
  }
  double a = 0.0;
  if (isSp)
    for (int j = 0; j < K; ++j) a += Jrow[1 + j] * L.C[j];
  const double aT = grp_sum<G>(isSp ? JwT * Ck : 0.0);
  if (isSp) {
    // chain rule through C_j(rho(T, Y), Y): dC_j/dY_i = rho d_ij/W_j - C_j/(S W_i), dC_j/dT = -C_j/T
    for (int i = 0; i < K; ++i) {
      const double Wi = M.W[i];
      Jrow[1 + i] = (Wk / rho) * ((rho * Jrow[1 + i] - a / S) / Wi) + Wk * wd / (rho * S * Wi);
    }
    Jrow[0] = (Wk / rho) * (dwdTC - a / T) + Wk * wd / (rho * T);
    L.J[1 + k] = -((rho * JwT - aT / S) / Wk) / (rho * cp) -
                 fT * (-1.0 / (S * Wk) + RG * cpR / (Wk * cp));
  }
  if (l == 0)
    L.J[0] = -(sumCpW + sumHqT - aT / T) / (rho * cp) - fT * (-1.0 / T + dcpdT / cp);
  wave_sync();
#pragma unroll
  for (int j = 0; j < G; ++j) {
    double v = 0.0;
    if (j < n && l < n) v = -Jrow[j];
    m[j] = v + ((j == l) ? ((l < n) ? dg : 1.0) : 0.0);
  }
  wave_sync();  // LDS J is reused by the next evaluation
}

// Lane that holds pivot step k within the calling lane's group.
template <int G>
__device__ __forceinline__ int pivot_lane(int mystep, int k, int gbase) {
  const unsigned long long mask = __ballot(mystep == k);
  constexpr unsigned long long seg = (G == 64) ? ~0ull : ((1ull << (G & 63)) - 1ull);
  const unsigned long long gm = (G == 64) ? mask : ((mask >> gbase) & seg);
  return __ffsll((long long)gm) - 1;
}

// In-register LU with partial pivoting of the n x n matrix whose row l sits
// in lane l (m[]).  Pivot of step k: the not-yet-eliminated row with the
// largest |m_ik| (NaN counts as largest), ties to the lowest row.  Rows do not
// move: lane l records the step at which it became pivot (mystep) and the
// inverse of its diagonal.  Returns false for a zero or non-finite pivot.
template <int G>
__device__ __forceinline__ bool lu_factor(double (&m)[G], int l, int n, int &mystep,
                                          double &invd) {
  bool done = (l >= n);
  mystep = done ? l : -1;
  invd = 1.0;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < G; ++k) {
    if (k < n) {
      double v = done ? -1.0 : fabs(m[k]);
      if (v != v) v = INFINITY;
      int idx = l;
#pragma unroll
      for (int off = G / 2; off >= 1; off >>= 1) {
        const double v2 = __shfl_xor(v, off, G);
        const int i2 = __shfl_xor(idx, off, G);
        if (v2 > v || (v2 == v && i2 < idx)) {
          v = v2;
          idx = i2;
        }
      }
      const double pv = __shfl(m[k], idx, G);
      if (!(fabs(pv) > 0.0) || !isfinite(pv)) ok = false;
      const double inv = 1.0 / pv;
      if (l == idx) {
        done = true;
        mystep = k;
        invd = inv;
      }
      const bool upd = !done;
      const double mult = m[k] * inv;
      if (upd) m[k] = mult;
#pragma unroll
      for (int j = k + 1; j < G; ++j) {
        if (j < n) {
          const double pj = __shfl(m[j], idx, G);
          if (upd) m[j] = fma(-mult, pj, m[j]);
        }
      }
    }
  }
  return ok;
}

// Solve M x = b with the factors of lu_factor.  Lane l passes b_l and gets x_l.
template <int G>
__device__ __forceinline__ double lu_solve(const double (&m)[G], int l, int n, int mystep,
                                           double invd, int gbase, double b) {
#pragma unroll
  for (int k = 0; k < G; ++k) {
    if (k < n) {
      const int src = pivot_lane<G>(mystep, k, gbase);
      const double zk = __shfl(b, src, G);
      if (mystep > k) b = fma(-m[k], zk, b);
    }
  }
  double x = 0.0;
#pragma unroll
  for (int k = G - 1; k >= 0; --k) {
    if (k < n) {
      const int src = pivot_lane<G>(mystep, k, gbase);
      const double xk = __shfl(b * invd, src, G);
      if (mystep < k) b = fma(-m[k], xk, b);
      if (l == k) x = xk;
    }
  }
  return x;
}

struct StepArgs {
  int64_t n, ld;
  double dt;
  const double *dt_cell;
  double *T;
  const double *p;
  double *Y;
  double *RR;
  double *h_hint;
  int32_t *stats;
  const int32_t *index;  // optional cell index list (cell j of the call is index[j])
  StepOpts o;
  unsigned long long *counter;
  const unsigned long long *n_dev;  // optional device-side cell count (overrides n)
  uint8_t *flags;                    // optional: bit 4 set for cells that fail
};

__global__ void k_reset_counter(unsigned long long *c) {
  if (threadIdx.x == 0) c[0] = 0ull;
}

template <int G>
__global__ __launch_bounds__(64) void k_rates(DevMech M, int64_t N, int64_t ld, const double *T,
                                              const double *p, const double *Y, double *wdot,
                                              double *dTdt, double *kfkr) {
  extern __shared__ double lds[];
  constexpr int CPW = 64 / G;
  const int lane = threadIdx.x;
  const int g = lane / G, l = lane % G;
  GLds<G> L(lds + g * GLds<G>::doubles(M.R), M.R);
  double m[G];
  for (int64_t base = (int64_t)blockIdx.x * CPW; base < N; base += (int64_t)gridDim.x * CPW) {
    const int64_t cell = base + g;
    if (cell >= N) break;  // group-uniform
    double yl = 0.0;
    if (l == 0) yl = T[cell];
    else if (l <= M.K) yl = Y[(int64_t)(l - 1) * ld + cell];
    const double pc = p[cell];
    double f, wd;
    if (kfkr)
      eval_cell<G, false, true>(M, L, l, pc, yl, f, wd, m, 0.0);
    else
      eval_cell<G, false, false>(M, L, l, pc, yl, f, wd, m, 0.0);
    if (l >= 1 && l <= M.K) wdot[(int64_t)(l - 1) * ld + cell] = wd;
    if (l == 0 && dTdt) dTdt[cell] = f;
    if (kfkr) {
      for (int r = l; r < M.R; r += G) {
        kfkr[(int64_t)r * ld + cell] = L.kfs[r];
        kfkr[(int64_t)(M.R + r) * ld + cell] = L.krs[r];
      }
    }
    wave_sync();
  }
}

template <int G>
__global__ __launch_bounds__(64) void k_step(DevMech M, StepArgs A) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int g = lane / G, l = lane % G, gbase = g * G;
  const int n = M.n;
  GLds<G> L(lds + g * GLds<G>::doubles(M.R), M.R);
  const StepOpts &o = A.o;
  double m[G];

  // per-cell state (group-uniform scalars are replicated in every lane)
  int64_t cell = 0, gcell = 0;
  bool active = false;
  double yl = 0.0, y0 = 0.0, p = 0.0, dt = 0.0, t = 0.0, h = 0.0, fac_max = 6.0, rho0 = 0.0;
  int nacc = 0, nrej = 0, status = CELL_OK;

  const int64_t ncell = A.n_dev ? (int64_t)*A.n_dev : A.n;
  auto fetch = [&]() {
    unsigned long long c = 0;
    if (l == 0) c = atomicAdd(A.counter, 1ull);
    c = __shfl(c, 0, G);
    cell = (int64_t)c;
    active = cell < ncell;
    if (!active) return;
    gcell = A.index ? (int64_t)A.index[cell] : cell;
    yl = 0.0;
    if (l == 0) yl = A.T[gcell];
    else if (l < n) yl = A.Y[(int64_t)(l - 1) * A.ld + gcell];
    y0 = yl;
    p = A.p[gcell];
    dt = A.dt_cell ? A.dt_cell[gcell] : A.dt;
    const double hh = A.h_hint ? A.h_hint[gcell] : 0.0;
    h = (hh > 0.0) ? hh : o.h0;
    if (h > dt) h = dt;
    t = 0.0;
    fac_max = 6.0;
    nacc = 0;
    nrej = 0;
    status = CELL_OK;
    const bool bad = grp_any<G>(l < n && !isfinite(yl));
    const double T0 = __shfl(yl, 0, G);
    if (bad || !(T0 > 0.0) || !isfinite(p) || !(p > 0.0) || !(dt > 0.0) || !isfinite(dt))
      status = CELL_NONFINITE;
    // density at the initial state, for the rates output
    const double s = grp_sum<G>((l >= 1 && l < n) ? yl / M.W[l - 1] : 0.0);
    rho0 = p / (RG * T0 * s);
  };

  auto finish = [&]() {
    const bool ok = (status == CELL_OK);
    if (ok && l < n) {
      if (l == 0) A.T[gcell] = yl;
      else A.Y[(int64_t)(l - 1) * A.ld + gcell] = yl;
    }
    if (A.RR && l >= 1 && l < n)
      A.RR[(int64_t)(l - 1) * A.ld + gcell] = ok ? rho0 * (yl - y0) / dt : 0.0;
    if (l == 0) {
      if (A.h_hint && ok) A.h_hint[gcell] = h;
      if (A.stats) {
        A.stats[gcell] = nacc;
        A.stats[A.ld + gcell] = nrej;
        A.stats[2 * A.ld + gcell] = status;
      }
      if (A.flags && !ok) A.flags[gcell] |= 4;
    }
  };

  fetch();
  while (__any(active)) {
    if (active) {
      bool end = (status != CELL_OK) || !(t < dt);
      if (!end) {
        if (nacc + nrej >= o.max_steps) {
          status = CELL_MAX_STEPS;
          end = true;
        }
      }
      bool last = false;
      if (!end) {
        if (h >= dt - t) {
          h = dt - t;
          last = true;
        }
        if (h < o.h_min) {
          status = CELL_H_UNDERFLOW;
          end = true;
        }
      }
      if (!end) {
        // ---- one RODAS3 attempt of size h from yl ----
        double F, wd;
        eval_cell<G, true, false>(M, L, l, p, yl, F, wd, m, 1.0 / (GAMMA * h));
        int mystep;
        double invd;
        const bool ok = lu_factor<G>(m, l, n, mystep, invd);
        if (!ok) {
          status = CELL_SINGULAR;
          end = true;
        } else {
          double Ks[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            if (s > 0 && TNEWF[s]) {
              double v = yl;
#pragma unroll
              for (int j = 0; j < s; ++j) v += TA[s][j] * Ks[j];
              eval_cell<G, false, false>(M, L, l, p, v, F, wd, m, 0.0);
            }
            double c = 0.0;
#pragma unroll
            for (int j = 0; j < s; ++j) c += TC[s][j] * Ks[j];
            Ks[s] = lu_solve<G>(m, l, n, mystep, invd, gbase, F + c / h);
          }
          double ynew = yl, errv = 0.0;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            ynew += TM[s] * Ks[s];
            errv += TE[s] * Ks[s];
          }
          double r2 = 0.0;
          if (l < n) {
            const double atol = (l == 0) ? o.atol_T : o.atol_Y;
            const double sc = atol + o.rtol * fmax(fabs(yl), fabs(ynew));
            const double rr = errv / sc;
            r2 = rr * rr;
          }
          const double err = sqrt(grp_sum<G>(r2) / n);
          if (isfinite(err) && err <= 1.0) {
            yl = ynew;
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
          end = !(t < dt);
        }
      }
      if (end) {
        if (status != CELL_OK) yl = y0;
        finish();
        fetch();
      }
    }
  }
}

template <int G>
size_t lds_bytes(int R, int cpw) {
  return (size_t)cpw * GLds<G>::doubles(R) * sizeof(double);
}

int group_size(int n) { return n <= 16 ? 16 : (n <= 32 ? 32 : 64); }

chem_status check_lds(size_t sh, int *cus) {
  int dev = 0, maxsh = 0;
  CHEM_HIP(hipGetDevice(&dev));
  CHEM_HIP(hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (cus) {
    CHEM_HIP(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (*cus < 1) *cus = 1;
  }
  if (sh > (size_t)maxsh) {
    set_error("mechanism needs %zu bytes of LDS per wave, the device allows %d", sh, maxsh);
    return CHEM_EUNSUPPORTED;
  }
  return CHEM_OK;
}

}  // namespace

chem_status launch_rates(const chem_mech *m, int64_t N, int64_t ld, const double *T,
                         const double *p, const double *Y, double *wdot, double *dTdt,
                         double *kfkr, hipStream_t s) {
  const int G = group_size(m->d.n);
  const int cpw = 64 / G;
  int64_t blocks = (N + cpw - 1) / cpw;
  if (blocks > 65536) blocks = 65536;
  size_t sh = G == 16 ? lds_bytes<16>(m->R, cpw)
                      : (G == 32 ? lds_bytes<32>(m->R, cpw) : lds_bytes<64>(m->R, cpw));
  chem_status st = check_lds(sh, nullptr);
  if (st != CHEM_OK) return st;
  ProfScope prof("chem_rates", s);
  switch (G) {
    case 16:
      hipLaunchKernelGGL(k_rates<16>, dim3((unsigned)blocks), dim3(64), sh, s, m->d, N, ld, T, p,
                         Y, wdot, dTdt, kfkr);
      break;
    case 32:
      hipLaunchKernelGGL(k_rates<32>, dim3((unsigned)blocks), dim3(64), sh, s, m->d, N, ld, T, p,
                         Y, wdot, dTdt, kfkr);
      break;
    default:
      hipLaunchKernelGGL(k_rates<64>, dim3((unsigned)blocks), dim3(64), sh, s, m->d, N, ld, T, p,
                         Y, wdot, dTdt, kfkr);
      break;
  }
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status launch_step(const chem_mech *m, int64_t N, int64_t ld, double dt,
                        const double *dt_cell, double *T, const double *p, double *Y, double *RR,
                        double *h_hint, int32_t *stats, const StepOpts &o, const int32_t *index,
                        hipStream_t s, const unsigned long long *n_dev, uint8_t *flags) {
  StepArgs A{N, ld, dt, dt_cell, T, p, Y, RR, h_hint, stats, index, o, m->counters, n_dev, flags};
  const int G = group_size(m->d.n);
  const int cpw = 64 / G;
  size_t sh = G == 16 ? lds_bytes<16>(m->R, cpw)
                      : (G == 32 ? lds_bytes<32>(m->R, cpw) : lds_bytes<64>(m->R, cpw));
  int cus = 0;
  chem_status st = check_lds(sh, &cus);
  if (st != CHEM_OK) return st;
  // persistent grid: enough single-wave blocks to fill every CU's LDS
  int per_cu = (int)((160 * 1024) / (sh > 0 ? sh : 1));
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 32) per_cu = 32;
  int64_t want = (N + cpw - 1) / cpw;  // with n_dev, N is an upper bound
  int64_t blocks = (int64_t)cus * per_cu;
  if (blocks > want) blocks = want;
  if (blocks < 1) return CHEM_OK;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, m->counters);
  ProfScope prof(index ? "chem_step_fallback" : "chem_step", s);
  switch (G) {
    case 16:
      hipLaunchKernelGGL(k_step<16>, dim3((unsigned)blocks), dim3(64), sh, s, m->d, A);
      break;
    case 32:
      hipLaunchKernelGGL(k_step<32>, dim3((unsigned)blocks), dim3(64), sh, s, m->d, A);
      break;
    default:
      hipLaunchKernelGGL(k_step<64>, dim3((unsigned)blocks), dim3(64), sh, s, m->d, A);
      break;
  }
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

}  // namespace chem
