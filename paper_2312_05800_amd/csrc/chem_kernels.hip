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
#include <stdlib.h>

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

// Tableau entries for a run-time stage index (selects, no memory access).
__device__ __forceinline__ double TA_S(int s, int j) {
  return s == 2 ? (j == 0 ? TA[2][0] : (j == 1 ? TA[2][1] : TA[2][2]))
       : (s == 3 ? (j == 0 ? TA[3][0] : (j == 1 ? TA[3][1] : TA[3][2])) : 0.0);
}
__device__ __forceinline__ double TC_S(int s, int j) {
  return s == 1 ? (j == 0 ? TC[1][0] : 0.0)
       : (s == 2 ? (j == 0 ? TC[2][0] : (j == 1 ? TC[2][1] : 0.0))
                 : (s == 3 ? (j == 0 ? TC[3][0] : (j == 1 ? TC[3][1] : TC[3][2])) : 0.0));
}
__device__ __forceinline__ bool TNEWF_S(int s) { return s == 2 || s == 3; }
// stage 0's f(y_n) is evaluated once per attempt, before the stage loop
static_assert(TNEWF[0] && !TNEWF[1] && TNEWF[2] && TNEWF[3],
              "TNEWF_S: stage 1 reuses f(y_n), stages 2 and 3 evaluate f at a new point");

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

// FP64 add to LDS (ds_add_f64); no return value.
__device__ __forceinline__ void lds_add(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Cross-lane exchanges inside a group of G lanes without the LDS crossbar:
// DPP patterns pair lanes within 16-lane rows (quad_perm [1,0,3,2] and
// [2,3,0,1], row_half_mirror, row_mirror), v_permlane16_swap pairs rows 0/1
// and 2/3, v_permlane32_swap the two halves of the wave.  After each stage of
// an all-reduce every lane of the merged set holds the same bits (the
// combining operations are commutative).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ double mk_f64(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// the value of the paired row (16-lane rows 0/1, 2/3) or half (32 lanes)
__device__ __forceinline__ void swap16(double v, double &a, double &b) {
  const long long x = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(x >> 32),
                                                   false, false);
  a = mk_f64(lo[0], hi[0]);  // the even row's value, in both rows of the pair
  b = mk_f64(lo[1], hi[1]);  // the odd row's value
}
__device__ __forceinline__ void swap32(double v, double &a, double &b) {
  const long long x = __double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(x >> 32),
                                                   false, false);
  a = mk_f64(lo[0], hi[0]);
  b = mk_f64(lo[1], hi[1]);
}
__device__ __forceinline__ int swap16_min(int v) {
  const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  return min((int)r[0], (int)r[1]);
}
__device__ __forceinline__ int swap32_min(int v) {
  const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return min((int)r[0], (int)r[1]);
}

template <int G>
__device__ __forceinline__ double grp_sum(double v) {
  static_assert(G == 16 || G == 32 || G == 64, "lane groups of 16, 32 or 64");
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  if (G >= 32) {
    double a, b;
    swap16(v, a, b);
    v = a + b;
  }
  if (G == 64) {
    double a, b;
    swap32(v, a, b);
    v = a + b;
  }
  return v;
}

template <int G>
__device__ __forceinline__ double grp_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  if (G >= 32) {
    double a, b;
    swap16(v, a, b);
    v = fmax(a, b);
  }
  if (G == 64) {
    double a, b;
    swap32(v, a, b);
    v = fmax(a, b);
  }
  return v;
}

template <int G>
__device__ __forceinline__ int grp_min(int v) {
  v = min(v, dpp_i32<0xB1>(v));
  v = min(v, dpp_i32<0x4E>(v));
  v = min(v, dpp_i32<0x141>(v));
  v = min(v, dpp_i32<0x140>(v));
  if (G >= 32) v = swap16_min(v);
  if (G == 64) v = swap32_min(v);
  return v;
}

template <int G>
__device__ __forceinline__ bool grp_any(bool b) {
  const unsigned long long m = __ballot(b);
  if (G == 64) return m != 0ull;
  const int gbase = ((int)threadIdx.x & 63) & ~(G - 1);
  return ((m >> gbase) & ((1ull << (G & 63)) - 1ull)) != 0ull;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)x, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), lane);
  return mk_f64(lo, hi);
}

// v of lane 0 of the caller's group.
template <int G>
__device__ __forceinline__ double grp_first(double v) {
  const int g = ((int)threadIdx.x & 63) / G;
  double out = 0.0;
#pragma unroll
  for (int gg = 0; gg < 64 / G; ++gg) {
    const double x = readlane_f64(v, gg * G);
    out = (g == gg) ? x : out;
  }
  return out;
}

// Per-group LDS scratch (doubles): concentrations, (g/RT, h/RT) pairs of the
// species (one 16-byte gather per reaction slot), the net production rates
// being accumulated, and the Jacobian / Newton matrix (n rows of odd
// stride).  In chem_rates the matrix region holds k_f, k_r instead; in the
// solves the concentration slots hold the permuted right-hand side.
template <int G>
struct GLds {
  double *C;
  double2 *gh;  // 16-byte aligned: the slice starts so, and C holds G doubles
  double *wa, *J;
  int js;  // row stride of J
  __device__ GLds(double *base, int R, int n) {
    C = base;
    gh = (double2 *)(C + G);
    wa = C + 3 * G;
    J = wa + G;
    js = stride(n);
  }
  // odd row stride (2 js banks apart: lanes reading one column hit distinct
  // banks) and only the n rows of the n x n matrix
  __host__ __device__ static int stride(int n) { return n | 1; }
  // even, so that every group's slice starts 16-byte aligned
  __host__ __device__ static size_t doubles(int R, int n) {
    const size_t j = (size_t)n * stride(n), k = 2 * (size_t)R;
    return (4 * G + (j > k ? j : k) + 1) & ~(size_t)1;
  }
};

// C^nu of a reaction slot (nu = 1 or 2; an empty slot names the dummy
// species, whose C is 1)
__device__ __forceinline__ double slot_fac(int s, int nu, const double *C) {
  const double c = C[s];
  return nu == 2 ? c * c : c;
}

// Rate constants and one-way rates of progress of reaction r from the
// species data in LDS: ln k_f = ln A + b ln T - E_a/(R T),
// ln K_c = -dG/RT + dn ln(p_ref/RT), k_r = exp(ln k_f - ln K_c).
struct Rxn {
  int4 sp, nu;
  double kf, kr, fwd, rev, dH, dn;
};

template <int G>
__device__ __forceinline__ Rxn rxn_eval(const DevMech &M, const GLds<G> &L, int r, double lnT,
                                        double invT, double lnPRT) {
  Rxn x;
  x.sp = M.sp[r];
  x.nu = M.nu[r];
  // empty slots gather the dummy species (g = h = 0, coefficient 0): no branches,
  // so the eight LDS reads of a reaction (four (g, h) pairs, four
  // concentrations) issue together
  double dG = 0.0, dH = 0.0;
  const double2 a0 = L.gh[x.sp.x], a1 = L.gh[x.sp.y], a2 = L.gh[x.sp.z], a3 = L.gh[x.sp.w];
  dG -= x.nu.x * a0.x;
  dH -= x.nu.x * a0.y;
  dG -= x.nu.y * a1.x;
  dH -= x.nu.y * a1.y;
  dG += x.nu.z * a2.x;
  dH += x.nu.z * a2.y;
  dG += x.nu.w * a3.x;
  dH += x.nu.w * a3.y;
  x.dH = dH;
  x.dn = M.dn[r];
  const double lnkf = M.lnA[r] + M.b[r] * lnT - M.EaR[r] * invT;
  const double lnKc = -dG + x.dn * lnPRT;
  x.kf = exp(lnkf);
  x.kr = exp(lnkf - lnKc);
  x.fwd = x.kf * slot_fac(x.sp.x, x.nu.x, L.C) * slot_fac(x.sp.y, x.nu.y, L.C);
  x.rev = x.kr * slot_fac(x.sp.z, x.nu.z, L.C) * slot_fac(x.sp.w, x.nu.w, L.C);
  return x;
}

// Adds reaction x's terms of the Jacobian to the LDS matrix (atomic FP64
// adds: lanes of the group process different reactions that share species).
// q = k_f prod C^nu' - k_r prod C^nu'', so dq/dC of a slot species is the
// product of the other factors times the derivative of its own factor.  Per
// slot species k_a (net coefficient nu_a: - for reactants, + for products)
// and slot species k_b: row 1 + k_a, column 1 + k_b gets nu_a dq/dC_kb and
// column 0 gets nu_a dq/dT; row 0, column 1 + k_b gets dH_r dq/dC_kb.
template <int G>
__device__ __forceinline__ void jac_scatter(const GLds<G> &L, const Rxn &x, double dqT,
                                            double dHr) {
  const double f0 = slot_fac(x.sp.x, x.nu.x, L.C), f1 = slot_fac(x.sp.y, x.nu.y, L.C);
  const double f2 = slot_fac(x.sp.z, x.nu.z, L.C), f3 = slot_fac(x.sp.w, x.nu.w, L.C);
  // empty slots (coefficient 0) name the dummy species, which has no row or
  // column in the matrix: they are skipped
  const int sp[4] = {x.sp.x, x.sp.y, x.sp.z, x.sp.w};
  const bool has[4] = {x.nu.x > 0, x.nu.y > 0, x.nu.z > 0, x.nu.w > 0};
  double dq[4];
  dq[0] = x.kf * (x.nu.x == 2 ? 2.0 * L.C[sp[0]] : 1.0) * f1;
  dq[1] = x.kf * f0 * (x.nu.y == 2 ? 2.0 * L.C[sp[1]] : 1.0);
  dq[2] = -x.kr * (x.nu.z == 2 ? 2.0 * L.C[sp[2]] : 1.0) * f3;
  dq[3] = -x.kr * f2 * (x.nu.w == 2 ? 2.0 * L.C[sp[3]] : 1.0);
  const double nu[4] = {-(double)x.nu.x, -(double)x.nu.y, (double)x.nu.z, (double)x.nu.w};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (!has[a]) continue;
    double *row = L.J + (1 + sp[a]) * L.js;
    lds_add(row, nu[a] * dqT);
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (has[b]) lds_add(row + 1 + sp[b], nu[a] * dq[b]);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
    if (has[b]) lds_add(L.J + 1 + sp[b], dHr * dq[b]);
}

// sum_j x[j] y[j] over j < n (LDS arrays), one FMA per term in index order.
// The operands are read eight at a time, so a chunk costs one LDS round trip
// instead of one per term; the last chunk reads with its indices clamped to
// n - 1 and adds only its terms below n.
__device__ __forceinline__ double dot_lds(const double *x, const double *y, int n) {
  double acc = 0.0;
  int j0 = 0;
  for (; j0 + 8 <= n; j0 += 8) {
    double a[8], c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = x[j0 + u];
      c[u] = y[j0 + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(a[u], c[u], acc);
  }
  if (j0 < n) {
    double a[8], c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = min(j0 + u, n - 1);
      a[u] = x[j];
      c[u] = y[j];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j0 + u < n) acc = fma(a[u], c[u], acc);
  }
  return acc;
}

// Right-hand side (and optionally the Jacobian) of one cell.  Lane l holds
// y_l in yl.  On return lane l holds f_l; species lanes hold wdot_k in wdl.
// With JAC, LDS row l (l < n) of L.J holds row l of M = I*dg - J.  With KOUT
// the rate constants are left in L.J (k_f at [r], k_r at [R + r]).
template <int G, bool JAC, bool KOUT>
__device__ __forceinline__ void eval_cell(const DevMech &M, const GLds<G> &L, int l, double p,
                                          double yl, double &f, double &wdl, double dg) {
  const int K = M.K, R = M.R, n = M.n;
  const double T = grp_first<G>(yl);
  const double lnT = log(T), invT = 1.0 / T;
  const bool isSp = (l >= 1) && (l <= K);
  const int k = isSp ? l - 1 : 0;
  double cpR = 0.0, hRT = 0.0, sR = 0.0, dcpR = 0.0, Wk = 1.0, iWk = 1.0, Yk = 0.0;
  if (isSp) {
    Wk = M.W[k];
    iWk = M.invW[k];
    Yk = yl;
    // coefficient i of species k in the range T selects: [i * K] from here
    const int o = (T <= M.Tmid[k] ? 0 : 7 * K) + k;
    const double *a = M.cpT + o, *hc = M.hT + o, *sc = M.sT + o;
    cpR = a[0] + T * (a[K] + T * (a[2 * K] + T * (a[3 * K] + T * a[4 * K])));
    hRT = hc[0] + T * (hc[K] + T * (hc[2 * K] + T * (hc[3 * K] + T * hc[4 * K]))) +
          hc[5 * K] * invT;
    sR = sc[0] * lnT + T * (sc[K] + T * (sc[2 * K] + T * (sc[3 * K] + T * sc[4 * K]))) +
         sc[5 * K];
    if (JAC) dcpR = a[K] + T * (2.0 * a[2 * K] + T * (3.0 * a[3 * K] + T * (4.0 * a[4 * K])));
  }
  const double S = grp_sum<G>(Yk * iWk);
  const double rho = p / (RG * T * S);
  const double irho = 1.0 / rho;
  const double Ck = rho * Yk * iWk;
  const double cp = grp_sum<G>(Yk * RG * cpR * iWk);
  if (isSp) {
    L.C[k] = Ck;
    L.gh[k] = make_double2(hRT - sR, hRT);
  }
  if (l == 0) {  // the dummy species of empty reaction slots
    L.C[K] = 1.0;
    L.gh[K] = make_double2(0.0, 0.0);
  }
  L.wa[l] = 0.0;
  double *Jrow = L.J + l * L.js;
  if (JAC && l < n)
    for (int j = 0; j < n; ++j) Jrow[j] = 0.0;
  wave_sync();

  const double lnPRT = log(PREF / (RG * T));
  double sumHq = 0.0;
  // two reactions per pass: their loads and gathers are independent and
  // issue together before the adds to LDS
  auto finish_rxn = [&](const Rxn &x, int r) {
    // wdot_k = sum_r (nu''_kr - nu'_kr) q_r, added from the reaction's lane
    // (the dummy species of empty slots takes the zero terms)
    const double q = x.fwd - x.rev;
    lds_add(L.wa + x.sp.x, -x.nu.x * q);
    lds_add(L.wa + x.sp.y, -x.nu.y * q);
    lds_add(L.wa + x.sp.z, x.nu.z * q);
    lds_add(L.wa + x.sp.w, x.nu.w * q);
    if (KOUT) {
      L.J[r] = x.kf;
      L.J[R + r] = x.kr;
    }
    if (JAC) {
      // dq/dT at fixed C: d ln kf/dT = b/T + Ea/(R T^2), d ln Kc/dT = dH_r/(R T^2) - dn/T
      const double dlnkf = M.b[r] * invT + M.EaR[r] * invT * invT;
      const double dlnKc = (x.dH - x.dn) * invT;
      const double dqT = x.fwd * dlnkf - x.rev * (dlnkf - dlnKc);
      sumHq += RG * T * x.dH * dqT;
      jac_scatter<G>(L, x, dqT, RG * T * x.dH);
    }
  };
  for (int r0 = l; r0 < R; r0 += 2 * G) {
    const int r1 = r0 + G;
    const bool two = r1 < R;
    const Rxn x0 = rxn_eval<G>(M, L, r0, lnT, invT, lnPRT);
    const Rxn x1 = rxn_eval<G>(M, L, two ? r1 : r0, lnT, invT, lnPRT);
    finish_rxn(x0, r0);
    if (two) finish_rxn(x1, r1);
  }
  wave_sync();

  const double wd = isSp ? L.wa[k] : 0.0;
  wdl = wd;
  const double Q = grp_sum<G>(isSp ? RG * T * hRT * wd : 0.0);
  const double fT = -Q * irho / cp;
  f = (l == 0) ? fT : (isSp ? Wk * wd * irho : 0.0);
  if (!JAC) return;

  // ---- analytic Jacobian ----
  // The reaction loop left, per species row k (LDS row 1 + k): d wdot_k/dC_j
  // at column 1 + j and sum_r nu_kr dq_r/dT at column 0; and in row 0,
  // column 1 + j: sum_r dH_r dq_r/dC_j.
  const double dcpdT = grp_sum<G>(Yk * RG * dcpR * iWk);
  const double sumCpW = grp_sum<G>(isSp ? RG * cpR * wd : 0.0);
  const double sumHqT = grp_sum<G>(sumHq);
  double a = 0.0, dwdTC = 0.0, JwT = 0.0;
  if (isSp) {
    a = dot_lds(Jrow + 1, L.C, K);
    dwdTC = Jrow[0];
    JwT = L.J[1 + k];
  }
  const double aT = grp_sum<G>(isSp ? JwT * Ck : 0.0);
  wave_sync();
  // chain rule through C_j(rho(T, Y), Y): dC_j/dY_i = rho d_ij/W_j - C_j/(S W_i),
  // dC_j/dT = -C_j/T; each entry is written once, as the Newton matrix
  // M = I/(gamma h) - J
  const double irhocp = irho / cp;
  if (isSp) {
    const double c2 = Wk * (wd - a) * irho / S;
    // eight entries of the row read, then eight written: one LDS round trip
    // per chunk (the last chunk reads with its indices clamped to K - 1)
    for (int i0 = 0; i0 < K; i0 += 8) {
      double jr[8], iw[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = min(i0 + u, K - 1);
        jr[u] = Jrow[1 + i];
        iw[u] = M.invW[i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u;
        if (i < K) {
          const double Jki = (Wk * jr[u] + c2) * iw[u];
          Jrow[1 + i] = ((i == k) ? dg : 0.0) - Jki;
        }
      }
    }
    Jrow[0] = -(Wk * irho * (dwdTC + (wd - a) * invT));
    L.J[1 + k] = ((rho * JwT - aT / S) * iWk) * irhocp + fT * (-iWk / S + RG * cpR * iWk / cp);
  }
  if (l == 0) L.J[0] = dg - (-(sumCpW + sumHqT - aT * invT) * irhocp - fT * (-invT + dcpdT / cp));
  wave_sync();
}

// Gauss-Jordan elimination with partial pivoting of the n x n matrix held in
// LDS, row l owned by lane l (odd row stride).  Pivot of step k: the
// not-yet-eliminated row with the largest |a_ik| (NaN counts as largest), ties
// to the lowest row, as in an LU with partial pivoting.  Rows do not move and
// pivot rows are not scaled: with p_k the pivot row of step k and
// m_i = a_ik / a_{p_k k}, every other row i becomes a_i. - m_i a_{p_k}. and
// its column k holds -m_i, the pivot row's column k holds 1.  Afterwards row
// p_k holds a_{p_k k} times row k of the inverse with its columns in pivot
// order (column j belongs to unknown p_j): each solve is then one
// matrix-vector product instead of two triangular sweeps of n dependent
// steps.  Lane l records its step (mystep) and 1/a_{l,mystep}.  Returns false
// for a zero or non-finite pivot.
template <int G>
__device__ __forceinline__ bool gj_factor(double *A, int l, int n, int &mystep, double &invd) {
  const int JS = GLds<G>::stride(n);
  double *row = A + l * JS;
  bool done = (l >= n);
  mystep = done ? l : -1;
  invd = 1.0;
  bool ok = true;
  for (int k = 0; k < n; ++k) {
    double v = done ? -1.0 : fabs(row[k]);
    if (v != v) v = INFINITY;
    const double vmax = grp_max<G>(v);
    const int idx = grp_min<G>(v == vmax ? l : G);
    const double *prow = A + idx * JS;
    const double pv = prow[k];
    if (!(fabs(pv) > 0.0) || !isfinite(pv)) ok = false;
    const double inv = 1.0 / pv;
    const bool isp = (l == idx);
    if (isp) {
      done = true;
      mystep = k;
      invd = inv;
    }
    if (l < n) {
      // the pivot row itself takes m = 0 and stays unchanged, so lanes
      // reading it see the same values whatever the order of the stores.
      // Eight entries are loaded before any is stored (the stores may alias
      // the pivot row as far as the compiler knows, which would otherwise
      // cost one LDS round trip per entry).
      const double m = isp ? 0.0 : row[k] * inv;
      for (int j0 = 0; j0 < n; j0 += 8) {
        double pr[8], rr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (j0 + u < n) {
            pr[u] = prow[j0 + u];
            rr[u] = row[j0 + u];
          }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (j0 + u < n) row[j0 + u] = fma(-m, pr[u], rr[u]);
      }
      row[k] = isp ? 1.0 : -m;
    }
    wave_sync();
  }
  return ok;
}

// Largest of 32-bit integer values over the caller's group (one DPP max per
// stage, as in grp_max).
template <int G>
__device__ __forceinline__ int grp_max_i32(int v) {
  v = max(v, dpp_i32<0xB1>(v));
  v = max(v, dpp_i32<0x4E>(v));
  v = max(v, dpp_i32<0x141>(v));
  v = max(v, dpp_i32<0x140>(v));
  if (G >= 32) {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    v = max((int)r[0], (int)r[1]);
  }
  if (G == 64) {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    v = max((int)r[0], (int)r[1]);
  }
  return v;
}
template <int G>
__device__ __forceinline__ unsigned grp_max_u32(unsigned v) {
  v = max(v, (unsigned)dpp_i32<0xB1>((int)v));
  v = max(v, (unsigned)dpp_i32<0x4E>((int)v));
  v = max(v, (unsigned)dpp_i32<0x141>((int)v));
  v = max(v, (unsigned)dpp_i32<0x140>((int)v));
  if (G >= 32) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = max((unsigned)r[0], (unsigned)r[1]);
  }
  if (G == 64) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    v = max((unsigned)r[0], (unsigned)r[1]);
  }
  return v;
}

// Lowest lane (index within the caller's group) whose b is set; G if none.
template <int G>
__device__ __forceinline__ int grp_first_lane(bool b) {
  const unsigned long long m = __ballot(b);
  if (G == 64) return m ? __builtin_ctzll(m) : G;
  const int g = ((int)threadIdx.x & 63) / G;
  int out = G;
#pragma unroll
  for (int gg = 0; gg < 64 / G; ++gg) {
    // bit G stands in for "no lane"
    const unsigned long long part =
        ((m >> (gg * G)) & ((1ull << (G & 63)) - 1ull)) | (1ull << (G & 63));
    const int f = __builtin_ctzll(part);
    out = (g == gg) ? f : out;
  }
  return out;
}

// Pivot lane of an elimination step: the lane with the largest v in the
// group, the lowest lane among equal values.  v is +0 ... +inf (a candidate
// row's |entry|) or -1 (a row already used), never NaN; on these values the
// order of the doubles is the order of the pair (high word as a signed
// integer, low word as an unsigned one), so the search runs on 32-bit words
// and ends in a ballot of the lanes holding the maximum.
template <int G>
__device__ __forceinline__ bool grp_is_max(double v) {
  const long long b = __double_as_longlong(v);
  const int hi = (int)(b >> 32);
  const unsigned lo = (unsigned)b;
  const int mh = grp_max_i32<G>(hi);
  const unsigned ml = grp_max_u32<G>(hi == mh ? lo : 0u);
  return hi == mh && lo == ml;
}
template <int G>
__device__ __forceinline__ int grp_argmax(double v) {
  return grp_first_lane<G>(grp_is_max<G>(v));
}
// the wave's ballot of the lanes holding their group's maximum
template <int G>
__device__ __forceinline__ unsigned long long grp_argmax_mask(double v) {
  return __ballot(grp_is_max<G>(v));
}

// c - m a as a three-address FMA: its result may go to another register than
// c, so the rotation of the register row below costs no copies.
__device__ __forceinline__ double fma_nm(double m, double a, double c) {
  double d;
  asm("v_fma_f64 %0, -%1, %2, %3" : "=v"(d) : "v"(m), "v"(a), "v"(c));
  return d;
}

// pairs of the pivot row broadcast by v_readlane instead of LDS (G = 32)
constexpr int GJ_RL = 2;

// gj_factor with each lane's row held in registers (groups of up to 32
// lanes): slot 0 always holds the column being eliminated (the row is
// rotated by one slot per step, so every index is a compile-time constant),
// and the pivot row reaches the other lanes through pbuf (G doubles of LDS)
// as one broadcast per step; the only LDS round trip left on a step's
// dependency chain.  Every lane forms the reciprocal of its own candidate
// pivot while the pivot is searched for, and the pivot lane sends its
// reciprocal in place of the pivot (slot 0): the division leaves the chain.
// Same arithmetic, in the same order, as gj_factor; the factors are written
// back to the LDS rows at the end.
template <int G>
__device__ __forceinline__ bool gj_factor_reg(double *A, double *pbuf, int l, int n, int &mystep,
                                              double &invd) {
  static_assert(G <= 32, "the register row holds G doubles");
  const int JS = GLds<G>::stride(n);
  double *rowp = A + l * JS;
  const bool real = l < n;
  double r[G];
#pragma unroll
  for (int i = 0; i < G; ++i) r[i] = (real && i < n) ? rowp[i] : 0.0;
  bool done = !real;
  mystep = done ? l : -1;
  invd = 1.0;
  bool ok = true;  // this lane's pivot (if it was one) is finite and non-zero
  // the reciprocal of slot 0, formed as soon as the slot is (at the end of
  // the previous step)
  double rinv = 1.0 / r[0];
  for (int k = 0; k < n; ++k) {
    double v = done ? -1.0 : fabs(r[0]);
    if (v != v) v = INFINITY;
    // the first GJ_RL pairs of the pivot row (slot 0 carrying the
    // reciprocal) reach the other lanes by v_readlane from the pivot lanes of
    // the wave's two groups, the rest through LDS: the LDS pipe, shared by
    // every wave of the CU, is the integrator's busiest unit, and moving two
    // of the sixteen pairs to the VALU was the fastest split measured
    constexpr int RP = (G == 32) ? GJ_RL : 0;
    int idx, q0 = 0, q1 = 0;
    if constexpr (RP > 0) {
      const unsigned long long bm = grp_argmax_mask<G>(v);
      q0 = __builtin_ctzll((bm & 0xffffffffull) | (1ull << 32));
      q1 = __builtin_ctzll((bm >> 32) | (1ull << 32));
      idx = (((int)threadIdx.x & 63) < 32) ? q0 : q1;
      q0 &= 31;
      q1 = 32 + (q1 & 31);
    } else {
      idx = grp_argmax<G>(v);
    }
    const bool isp = (l == idx);
    // pbuf is 16-byte aligned: the row moves as G / 2 pairs (b128 accesses)
    double2 *const pb2 = (double2 *)pbuf;
    if (isp) {
      if (RP == 0) pb2[0] = make_double2(rinv, r[1]);
#pragma unroll
      for (int i = (RP > 0 ? RP : 1); i < G / 2; ++i)
        pb2[i] = make_double2(r[2 * i], r[2 * i + 1]);
      if (!(fabs(r[0]) > 0.0) || !isfinite(r[0])) ok = false;
      done = true;
      mystep = k;
      invd = rinv;
    }
    wave_sync();
    double2 q[G / 2];
#pragma unroll
    for (int i = RP; i < G / 2; ++i) q[i] = pb2[i];
    if constexpr (RP > 0) {
      const bool g0 = ((int)threadIdx.x & 63) < 32;
#pragma unroll
      for (int i = 0; i < RP; ++i) {
        const double e0 = (i == 0) ? rinv : r[2 * i], e1 = r[2 * i + 1];
        const double a0 = readlane_f64(e0, q0), b0 = readlane_f64(e0, q1);
        const double a1 = readlane_f64(e1, q0), b1 = readlane_f64(e1, q1);
        q[i] = make_double2(g0 ? a0 : b0, g0 ? a1 : b1);
      }
    }
    const double inv = q[0].x;
    const double m = isp ? 0.0 : r[0] * inv;
    double pr[G];
#pragma unroll
    for (int i = 1; i < G; ++i) pr[i] = (i & 1) ? q[i / 2].y : q[i / 2].x;
    const double c0 = isp ? 1.0 : -m;
    // the next step's column first, so that its reciprocal (formed here by
    // every lane, not sunk into the pivot's branch) overlaps the other updates
    r[0] = fma_nm(m, pr[1], r[1]);
    rinv = 1.0 / r[0];
    asm volatile("" : "+v"(rinv));
#pragma unroll
    for (int i = 1; i < G - 1; ++i) r[i] = fma_nm(m, pr[i + 1], r[i + 1]);
    r[G - 1] = c0;
    wave_sync();  // every lane has read pbuf before the next pivot row goes there
  }
  // after n rotations slot i holds column (n + i) mod G: G - n more put
  // column i back in slot i, so the stores take constant offsets
  for (int t = n; t < G; ++t) {
    const double c0 = r[0];
#pragma unroll
    for (int i = 0; i < G - 1; ++i) r[i] = r[i + 1];
    r[G - 1] = c0;
  }
  if (real) {
#pragma unroll
    for (int i = 0; i < G; ++i)
      if (i < n) rowp[i] = r[i];
  }
  wave_sync();
  return !grp_any<G>(!ok);
}

// Solve M x = b with the factors of gj_factor.  Lane l passes b_l, gets x_l.
// v (G doubles of LDS) carries b in pivot order, then x.
template <int G>
__device__ __forceinline__ double gj_solve(const double *A, double *v, int l, int n, int mystep,
                                           double invd, double b) {
  const int JS = GLds<G>::stride(n);
  const double *row = A + l * JS;
  const bool real = l < n;  // lanes past n own no row (none is stored for them)
  if (real) v[mystep] = b;
  wave_sync();
  const double acc = real ? dot_lds(row, v, n) : 0.0;
  wave_sync();
  if (real) v[mystep] = acc * invd;
  wave_sync();
  const double x = real ? v[l] : 0.0;
  wave_sync();
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
  const chem_set *sets;              // optional set table (device): queue index q is cell
  const int64_t *set_off;            //   q - set_off[s] of the set s with set_off[s] <= q
  int n_sets;
};

// Arrays of the cell a group is working on.
struct CellRef {
  double *T;
  const double *p;
  double *Y;
  double *RR;
  double *hh;
  int32_t *stats;
  int64_t ld, i;
  double dt;
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
  GLds<G> L(lds + g * GLds<G>::doubles(M.R, M.n), M.R, M.n);
  for (int64_t base = (int64_t)blockIdx.x * CPW; base < N; base += (int64_t)gridDim.x * CPW) {
    const int64_t cell = base + g;
    if (cell >= N) break;  // group-uniform
    double yl = 0.0;
    if (l == 0) yl = T[cell];
    else if (l <= M.K) yl = Y[(int64_t)(l - 1) * ld + cell];
    const double pc = p[cell];
    double f, wd;
    if (kfkr)
      eval_cell<G, false, true>(M, L, l, pc, yl, f, wd, 0.0);
    else
      eval_cell<G, false, false>(M, L, l, pc, yl, f, wd, 0.0);
    if (l >= 1 && l <= M.K) wdot[(int64_t)(l - 1) * ld + cell] = wd;
    if (l == 0 && dTdt) dTdt[cell] = f;
    if (kfkr) {
      for (int r = l; r < M.R; r += G) {
        kfkr[(int64_t)r * ld + cell] = L.J[r];
        kfkr[(int64_t)(M.R + r) * ld + cell] = L.J[M.R + r];
      }
    }
    wave_sync();
  }
}

template <int G>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_step(DevMech M, StepArgs A) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x;
  const int g = lane / G, l = lane % G;
  const int n = M.n;
  GLds<G> L(lds + g * GLds<G>::doubles(M.R, M.n), M.R, M.n);
  const StepOpts &o = A.o;

  // per-cell state (group-uniform scalars are replicated in every lane)
  int64_t cell = 0, gcell = 0;
  bool active = false;
  double yl = 0.0, y0 = 0.0, p = 0.0, dt = 0.0, t = 0.0, h = 0.0, fac_max = 6.0, rho0 = 0.0;
  int nacc = 0, nrej = 0, status = CELL_OK;

  const int64_t ncell = A.n_dev ? (int64_t)*A.n_dev : A.n;
  // an empty device-side list (no cell fell back) ends every wave here,
  // without a round of atomics on the queue counter
  if (ncell <= 0) return;
  CellRef cr{};
  auto fetch = [&]() {
    unsigned long long c = 0;
    if (l == 0) c = atomicAdd(A.counter, 1ull);
    c = __shfl(c, 0, G);
    cell = (int64_t)c;
    active = cell < ncell;
    if (!active) return;
    if (A.n_sets > 0) {
      int lo = 0, hi = A.n_sets;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (A.set_off[mid] <= cell) lo = mid;
        else hi = mid;
      }
      const chem_set &st = A.sets[lo];
      cr = CellRef{st.T, st.p, st.Y, st.RR, st.h_hint, st.stats, st.ld, cell - A.set_off[lo],
                   st.dt};
    } else {
      const int64_t gc = A.index ? (int64_t)A.index[cell] : cell;
      cr = CellRef{A.T, A.p, A.Y, A.RR, A.h_hint, A.stats, A.ld, gc,
                   A.dt_cell ? A.dt_cell[gc] : A.dt};
    }
    gcell = cr.i;
    yl = 0.0;
    if (l == 0) yl = cr.T[gcell];
    else if (l < n) yl = cr.Y[(int64_t)(l - 1) * cr.ld + gcell];
    y0 = yl;
    p = cr.p[gcell];
    dt = cr.dt;
    const double hh = cr.hh ? cr.hh[gcell] : 0.0;
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
      if (l == 0) cr.T[gcell] = yl;
      else cr.Y[(int64_t)(l - 1) * cr.ld + gcell] = yl;
    }
    if (cr.RR && l >= 1 && l < n)
      cr.RR[(int64_t)(l - 1) * cr.ld + gcell] = ok ? rho0 * (yl - y0) / dt : 0.0;
    if (l == 0) {
      if (cr.hh && ok) cr.hh[gcell] = h;
      if (cr.stats) {
        cr.stats[gcell] = nacc;
        cr.stats[cr.ld + gcell] = nrej;
        cr.stats[2 * cr.ld + gcell] = status;
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
        eval_cell<G, true, false>(M, L, l, p, yl, F, wd, 1.0 / (GAMMA * h));
        int mystep;
        double invd;
        bool ok;
        if constexpr (G <= 32)
          ok = gj_factor_reg<G>(L.J, L.wa, l, n, mystep, invd);
        else
          ok = gj_factor<G>(L.J, l, n, mystep, invd);
        if (!ok) {
          status = CELL_SINGULAR;
          end = true;
        } else {
          // Stage loop kept rolled so that one copy of the right-hand side and
          // of the triangular solve is emitted (the unrolled form overflows the
          // instruction cache).  Terms with j >= s add exact zeros, so the
          // sums equal the oracle's sums over j < s.
          double K0 = 0.0, K1 = 0.0, K2 = 0.0, K3 = 0.0;
#pragma nounroll
          for (int s = 0; s < 4; ++s) {
            if (TNEWF_S(s)) {
              const double v = yl + TA_S(s, 0) * K0 + TA_S(s, 1) * K1 + TA_S(s, 2) * K2;
              eval_cell<G, false, false>(M, L, l, p, v, F, wd, 0.0);
            }
            const double c = TC_S(s, 0) * K0 + TC_S(s, 1) * K1 + TC_S(s, 2) * K2;
            const double x = gj_solve<G>(L.J, L.C, l, n, mystep, invd, F + c / h);
            K0 = (s == 0) ? x : K0;
            K1 = (s == 1) ? x : K1;
            K2 = (s == 2) ? x : K2;
            K3 = (s == 3) ? x : K3;
          }
          double ynew = yl, errv = 0.0;
          ynew += TM[0] * K0;
          errv += TE[0] * K0;
          ynew += TM[1] * K1;
          errv += TE[1] * K1;
          ynew += TM[2] * K2;
          errv += TE[2] * K2;
          ynew += TM[3] * K3;
          errv += TE[3] * K3;
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
size_t lds_bytes(int R, int n, int cpw) {
  return (size_t)cpw * GLds<G>::doubles(R, n) * sizeof(double);
}

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

int group_size(int n) { return n <= 16 ? 16 : (n <= 32 ? 32 : 64); }

size_t step_lds_bytes(const chem_mech *m, int G) {
  const int cpw = 64 / G;
  return G == 16 ? lds_bytes<16>(m->R, m->d.n, cpw)
                 : (G == 32 ? lds_bytes<32>(m->R, m->d.n, cpw) : lds_bytes<64>(m->R, m->d.n, cpw));
}

int max_waves_per_cu(size_t sh) {
  const int w = (int)((160 * 1024) / (sh > 0 ? sh : 1));
  return w < 1 ? 1 : (w > 32 ? 32 : w);
}

chem_status launch_rates(const chem_mech *m, int64_t N, int64_t ld, const double *T,
                         const double *p, const double *Y, double *wdot, double *dTdt,
                         double *kfkr, hipStream_t s) {
  const int G = group_size(m->d.n);
  const int cpw = 64 / G;
  int64_t blocks = (N + cpw - 1) / cpw;
  if (blocks > 65536) blocks = 65536;
  size_t sh = G == 16 ? lds_bytes<16>(m->R, m->d.n, cpw)
                      : (G == 32 ? lds_bytes<32>(m->R, m->d.n, cpw) : lds_bytes<64>(m->R, m->d.n, cpw));
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

// Offsets of a device set table: off[s] = cells of the valid sets before s,
// off[n_sets] and *total = all of them; a set with bad sizes, null arrays or
// a bad dt counts as empty and is counted in *n_bad.  One block: each thread
// sums a contiguous run of sets, a scan over the runs, then each thread
// writes its run's offsets.
constexpr int SETOFF_THREADS = 1024;

__device__ __forceinline__ int64_t valid_cells(const chem_set &c, int *bad) {
  const bool ok = c.n >= 0 && c.ld >= c.n &&
                  (c.n == 0 || (c.T && c.p && c.Y && c.dt > 0.0 && isfinite(c.dt)));
  *bad = ok ? 0 : 1;
  return ok ? c.n : 0;
}

__global__ __launch_bounds__(SETOFF_THREADS) void k_set_offsets(const chem_set *sets, int n_sets,
                                                                 int64_t *off,
                                                                 unsigned long long *total,
                                                                 int32_t *n_bad) {
  __shared__ int64_t run[SETOFF_THREADS];
  __shared__ int bads[SETOFF_THREADS];
  const int t = threadIdx.x;
  const int per = (n_sets + SETOFF_THREADS - 1) / SETOFF_THREADS;
  const int s0 = t * per, s1 = s0 + per < n_sets ? s0 + per : n_sets;
  int64_t sum = 0;
  int nb = 0;
  for (int i = s0; i < s1; ++i) {
    int b = 0;
    sum += valid_cells(sets[i], &b);
    nb += b;
  }
  run[t] = sum;
  bads[t] = nb;
  __syncthreads();
  if (t == 0) {  // exclusive scan of the runs, in order
    int64_t acc = 0;
    int nbad = 0;
    for (int q = 0; q < SETOFF_THREADS; ++q) {
      const int64_t v = run[q];
      run[q] = acc;
      acc += v;
      nbad += bads[q];
    }
    off[n_sets] = acc;
    *total = (unsigned long long)acc;
    if (n_bad) *n_bad = nbad;
  }
  __syncthreads();
  int64_t acc = run[t];
  for (int i = s0; i < s1; ++i) {
    off[i] = acc;
    int b = 0;
    acc += valid_cells(sets[i], &b);
  }
}

chem_status launch_set_offsets(const chem_set *sets, int n_sets, int64_t *off,
                               unsigned long long *total, int32_t *n_bad, hipStream_t s) {
  hipLaunchKernelGGL(k_set_offsets, dim3(1), dim3(SETOFF_THREADS), 0, s, sets, n_sets, off,
                     total, n_bad);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status launch_step(const chem_mech *m, int64_t N, int64_t ld, double dt,
                        const double *dt_cell, double *T, const double *p, double *Y, double *RR,
                        double *h_hint, int32_t *stats, const StepOpts &o, const int32_t *index,
                        hipStream_t s, const unsigned long long *n_dev, uint8_t *flags,
                        const chem_set *sets, const int64_t *set_off, int n_sets) {
  StepArgs A{N,       ld,    dt,          dt_cell, T,     p,    Y,       RR,     h_hint,
             stats,   index, o,           m->counters, n_dev, flags, sets, set_off, n_sets};
  const int G = m->tune_G ? m->tune_G : group_size(m->d.n);
  const int cpw = 64 / G;
  const size_t sh = step_lds_bytes(m, G);
  int cus = 0;
  chem_status st = check_lds(sh, &cus);
  if (st != CHEM_OK) return st;
  // persistent grid: enough single-wave blocks to fill every CU's LDS, or
  // the tuned number of waves per CU
  int per_cu = max_waves_per_cu(sh);
  if (m->tune_waves > 0 && m->tune_waves < per_cu) per_cu = m->tune_waves;
  int64_t want = (N + cpw - 1) / cpw;  // with n_dev, N is an upper bound
  int64_t blocks = (int64_t)cus * per_cu;
  if (blocks > want) blocks = want;
  if (blocks < 1) return CHEM_OK;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, m->counters);
  ProfScope prof(index ? "chem_step_fallback" : (sets ? "chem_step_sets" : "chem_step"), s);
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
