// Partially stirred reactor closure of the chemistry source (Sec. 4.1): each
// cell's step rates are multiplied by its reacting fraction
// kappa = tau_c / (tau_c + tau_mix), with the mixing time the geometric mean
// of the flow's Taylor and Kolmogorov times and the chemical time set by the
// slowest formation rate among the species that take part in the step.
//
// One thread per cell.  The kernel streams Y and RR once (SoA: one species of
// 64 consecutive cells is one 512-byte wavefront load), keeps both in
// registers for the two passes over the species and writes the scaled rates
// back in place: 3K + 6 doubles of HBM traffic per cell, nothing re-read.
#include <math.h>

#include "chem_internal.h"

namespace chem {
namespace {

constexpr double RG = 8.314462618;  // J/(mol K)
constexpr int PASR_THREADS = 256;

struct PasrArgs {
  int64_t n, ld;
  const double *T, *p, *Y;
  double *RR;                       // [K][ld] in/out
  const double *tau_t, *tau_k;      // [n] Taylor and Kolmogorov times, s
  double *kappa, *tau_c;            // [n] out, nullable
  double eta;
};

// KC: register slots per array (K <= KC); species beyond K are never touched.
// The cells of a block are addressed from a block-uniform base (one scalar
// pointer per species row) plus the lane's 32-bit offset, so the loads and
// the in-place stores share one address register.
template <int KC>
__device__ __forceinline__ void pasr_block(const DevMech &M, const PasrArgs &a, int64_t c0) {
  const int K = M.K;
  const int64_t ld = a.ld;
  const unsigned t = threadIdx.x;
  if (c0 + t >= a.n) return;
  const double *Yb = a.Y + c0;
  double *Rb = a.RR + c0;
  double y[KC], r[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    if (k < K) {
      const double *yrow = Yb + (int64_t)k * ld;
      const double *rrow = Rb + (int64_t)k * ld;
      y[k] = yrow[t];
      r[k] = rrow[t];
    }
  }
  const double T = a.T[c0 + t], p = a.p[c0 + t];
  const double tT = a.tau_t[c0 + t], tK = a.tau_k[c0 + t];
  // ideal-gas density of the state and the largest rate magnitude
  double s = 0.0, amax = 0.0;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    if (k < K) {
      s += y[k] / M.W[k];
      amax = fmax(amax, fabs(r[k]));
    }
  }
  const double rho = p / (RG * T * s);
  // the slowest time rho Y_k / |RR_k| among species with |RR_k| >= eta max
  const double thr = a.eta * amax;
  double tc = -INFINITY;
  bool any = false;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    if (k < K) {
      const double m = fabs(r[k]);
      if (m > 0.0 && m >= thr) {
        any = true;
        tc = fmax(tc, rho * fmax(y[k], 0.0) / m);
      }
    }
  }
  if (!any) tc = INFINITY;
  const double tmix = sqrt(tT * tK);
  const double den = tc + tmix;
  const double kap = (isinf(tc) && tc > 0.0) || den == 0.0 ? 1.0 : tc / den;
#pragma unroll
  for (int k = 0; k < KC; ++k)
    if (k < K) {
      double *rrow = Rb + (int64_t)k * ld;
      rrow[t] = kap * r[k];
    }
  if (a.kappa) a.kappa[c0 + t] = kap;
  if (a.tau_c) a.tau_c[c0 + t] = tc;
}

template <int KC>
__global__ __launch_bounds__(PASR_THREADS) void k_pasr(DevMech M, PasrArgs a) {
  for (int64_t c0 = (int64_t)blockIdx.x * PASR_THREADS; c0 < a.n;
       c0 += (int64_t)gridDim.x * PASR_THREADS)
    pasr_block<KC>(M, a, c0);
}

}  // namespace
}  // namespace chem

using namespace chem;

extern "C" chem_status chem_pasr_scale(const chem_mech *m, chem_batch batch, const double *T,
                                       const double *p, const double *Y, double *RR,
                                       const double *tau_taylor, const double *tau_kolmogorov,
                                       const chem_pasr_opts *opts, double *kappa,
                                       double *tau_c, void *stream) {
  if (!m) {
    set_error("chem_pasr_scale: null mechanism");
    return CHEM_EINVAL;
  }
  const int64_t n = batch.n;
  if (n < 0 || batch.ld < n || n > ((int64_t)1 << 40)) {
    set_error("chem_pasr_scale: bad batch n=%lld ld=%lld", (long long)n, (long long)batch.ld);
    return CHEM_EINVAL;
  }
  const double eta = opts ? opts->eta : 1e-3;
  if (!(eta >= 0.0 && eta <= 1.0)) {
    set_error("chem_pasr_scale: eta=%g outside [0, 1]", eta);
    return CHEM_EINVAL;
  }
  if (n == 0) return CHEM_OK;
  if (!T || !p || !Y || !RR || !tau_taylor || !tau_kolmogorov) {
    set_error("chem_pasr_scale: null array");
    return CHEM_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  PasrArgs a{n, batch.ld, T, p, Y, RR, tau_taylor, tau_kolmogorov, kappa, tau_c, eta};
  int64_t blocks = (n + PASR_THREADS - 1) / PASR_THREADS;
  if (blocks > (1 << 20)) blocks = 1 << 20;  // larger batches loop over the grid
  const dim3 grid((unsigned)blocks);
  ProfScope prof("pasr_scale", st);
  const int K = m->d.K;
  if (K <= 16)
    hipLaunchKernelGGL(k_pasr<16>, grid, dim3(PASR_THREADS), 0, st, m->d, a);
  else if (K <= 32)
    hipLaunchKernelGGL(k_pasr<32>, grid, dim3(PASR_THREADS), 0, st, m->d, a);
  else
    hipLaunchKernelGGL(k_pasr<64>, grid, dim3(PASR_THREADS), 0, st, m->d, a);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}
