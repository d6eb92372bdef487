// Partially stirred reactor closure of the chemistry source (Sec. 4.1): each
// cell's step rates are multiplied by its reacting fraction
// kappa = tau_c / (tau_c + tau_mix), with the mixing time the geometric mean
// of the flow's Taylor and Kolmogorov times and the chemical time set by the
// slowest formation rate among the species that take part in the step.
//
// A block of four waves owns 64 consecutive cells, one per lane; wave w holds
// species w, w + 4, w + 8, ... of them in registers (Y and RR), so every load
// or store instruction moves one species row of 64 cells: 512 contiguous
// bytes from a wave-uniform base.  Rows are addressed through buffer
// resources whose size is the block's live cells, so the ragged last block
// needs no per-lane branch (reads past the end return 0, writes are dropped).
// The four waves' partial density sums, largest rates and slowest times meet
// in LDS.  The kernel streams Y and RR once and writes the scaled rates back
// in place: 3K + 6 doubles of HBM traffic per cell, nothing re-read.
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

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int BUF_DWORD3 = 0x00020000;  // raw buffer access, 32-bit data format

// a row of `cells` doubles starting at p, as a bounds-checked buffer
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const double *p, int cells) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, cells * 8, BUF_DWORD3);
}
__device__ __forceinline__ double row_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void row_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

constexpr int PASR_CELLS = 64;
constexpr int PASR_WAVES = PASR_THREADS / 64;

// KC: species slots per cell (K <= KC); wave w holds slots w, w + 4, ...
template <int KC>
__device__ __forceinline__ void pasr_cells(const DevMech &M, const PasrArgs &a, int64_t c0,
                                           double (*red)[PASR_CELLS]) {
  constexpr int J = KC / PASR_WAVES;
  const int K = M.K;
  const int64_t ld = a.ld;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const unsigned t = threadIdx.x & 63u;
  const unsigned off = t * 8u;
  const int live = (int)(a.n - c0 < PASR_CELLS ? a.n - c0 : PASR_CELLS);
  // every load of the cells goes out first: the per-cell inputs do not
  // wait behind the block's two reductions
  const double T = row_load(row_rsrc(a.T + c0, live), off);
  const double p = row_load(row_rsrc(a.p + c0, live), off);
  const double tT = row_load(row_rsrc(a.tau_t + c0, live), off);
  const double tK = row_load(row_rsrc(a.tau_k + c0, live), off);
  double y[J], r[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k = w + PASR_WAVES * j;
    y[j] = 0.0;
    r[j] = 0.0;
    if (k < K) {
      y[j] = row_load(row_rsrc(a.Y + (int64_t)k * ld + c0, live), off);
      r[j] = row_load(row_rsrc(a.RR + (int64_t)k * ld + c0, live), off);
    }
  }
  // partial density sums and largest rate magnitudes of this wave's species
  double s = 0.0, amax = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k = w + PASR_WAVES * j;
    if (k < K) {
      s += y[j] / M.W[k];
      amax = fmax(amax, fabs(r[j]));
    }
  }
  red[w][t] = s;
  red[PASR_WAVES + w][t] = amax;
  __syncthreads();
  s = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
  amax = fmax(fmax(red[4][t], red[5][t]), fmax(red[6][t], red[7][t]));
  const double rho = p / (RG * T * s);
  // the slowest time rho Y_k / |RR_k| among species with |RR_k| >= eta max
  // (-inf while none qualifies)
  const double thr = a.eta * amax;
  double tc = -INFINITY;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const double m = fabs(r[j]);
    if (m > 0.0 && m >= thr) tc = fmax(tc, rho * fmax(y[j], 0.0) / m);
  }
  red[2 * PASR_WAVES + w][t] = tc;
  __syncthreads();
  tc = fmax(fmax(red[8][t], red[9][t]), fmax(red[10][t], red[11][t]));
  if (tc == -INFINITY) tc = INFINITY;  // no reacting species
  const double tmix = sqrt(tT * tK);
  const double den = tc + tmix;
  const double kap = tc == INFINITY || den == 0.0 ? 1.0 : tc / den;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k = w + PASR_WAVES * j;
    if (k < K) row_store(row_rsrc(a.RR + (int64_t)k * ld + c0, live), off, kap * r[j]);
  }
  if (w == 0) {
    if (a.kappa) row_store(row_rsrc(a.kappa + c0, live), off, kap);
    if (a.tau_c) row_store(row_rsrc(a.tau_c + c0, live), off, tc);
  }
}

template <int KC>
__global__ __launch_bounds__(PASR_THREADS) void k_pasr(DevMech M, PasrArgs a) {
  __shared__ double red[3 * PASR_WAVES][PASR_CELLS];
  for (int64_t c0 = (int64_t)blockIdx.x * PASR_CELLS; c0 < a.n;
       c0 += (int64_t)gridDim.x * PASR_CELLS) {
    pasr_cells<KC>(M, a, c0, red);
    __syncthreads();  // red is reused by the block's next cells
  }
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
  int64_t blocks = (n + PASR_CELLS - 1) / PASR_CELLS;
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
