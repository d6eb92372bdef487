// Training-set sampler (the random-data generation of Sec. 3.1) on the GPU:
// every seed state is perturbed by Eqs. (Trand)-(Yrand) with the seed set's
// ranges and renormalised with N2 held at its perturbed value, or replaced by
// a state on the line between two given end states; each sample is then
// tested against the temperature threshold and the element-ratio limits of
// Table 1.  One thread per sample; the ranges come from an exact min/max
// reduction over the seeds first.
#include <math.h>

#include "chem_internal.h"

namespace chem {
namespace {

constexpr int RANGE_BLOCKS = 512;
constexpr int RANGE_THREADS = 256;

// partial min/max of T, p and y_N2 per block: part[b][6] =
// (min T, max T, min p, max p, min y_N2, max y_N2)
__global__ void k_ranges_part(int64_t n, int64_t ld, const double *T, const double *p,
                              const double *Y, int n2, double *part) {
  __shared__ double red[6][RANGE_THREADS];
  double v[6] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double t = T[i], q = p[i], y = Y[(int64_t)n2 * ld + i];
    v[0] = fmin(v[0], t);
    v[1] = fmax(v[1], t);
    v[2] = fmin(v[2], q);
    v[3] = fmax(v[3], q);
    v[4] = fmin(v[4], y);
    v[5] = fmax(v[5], y);
  }
  for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int off = RANGE_THREADS / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int q = 0; q < 6; ++q) {
        const double a = red[q][threadIdx.x], b = red[q][threadIdx.x + off];
        red[q][threadIdx.x] = (q & 1) ? fmax(a, b) : fmin(a, b);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_ranges_fin(const double *part, int nparts, double *out) {
  if (threadIdx.x >= 6) return;
  const int q = threadIdx.x;
  double v = part[q];
  for (int b = 1; b < nparts; ++b) {
    const double x = part[b * 6 + q];
    v = (q & 1) ? fmax(v, x) : fmin(v, x);
  }
  out[q] = v;
}

struct SampleArgs {
  int64_t n, ld;
  const double *T, *p, *Y;   // seeds
  const double *c;           // [K + 3][ld] uniform in [-1, 1]
  const double *s;           // [ld] mixing fraction (< 0: perturb), nullable
  const double *end_eq, *end_air;  // [K + 2]: T, p, Y_1..K
  const double *ranges;      // [6] from k_ranges_fin
  double *To, *po, *Yo;
  uint8_t *keep;
  chem_sample_opts o;
};

__device__ void sample_one(const DevMech &M, const SampleArgs &a, int64_t i) {
  const int K = M.K, n2 = a.o.n2;
  const int64_t ld = a.ld;
  const double s = a.s ? a.s[i] : -1.0;
  double T, p;
  if (s >= 0.0) {
    // the mixing line between the two end states
    T = (1.0 - s) * a.end_eq[0] + s * a.end_air[0];
    p = (1.0 - s) * a.end_eq[1] + s * a.end_air[1];
    for (int k = 0; k < K; ++k)
      a.Yo[(int64_t)k * ld + i] = (1.0 - s) * a.end_eq[2 + k] + s * a.end_air[2 + k];
  } else {
    // Eqs. (Trand), (Prand), (N2rand), (Yrand)
    const double *r = a.ranges;
    T = a.T[i] + a.o.alpha * a.c[i] * (r[1] - r[0]);
    p = a.p[i] + a.o.beta * a.c[ld + i] * (r[3] - r[2]);
    const double yn2 = a.Y[(int64_t)n2 * ld + i] + a.o.alpha * a.c[2 * ld + i] * (r[5] - r[4]);
    double sum = 0.0;
    for (int k = 0; k < K; ++k) {
      if (k == n2) continue;
      const double y = a.Y[(int64_t)k * ld + i];
      const double yp = y > 0.0 ? pow(y, 1.0 + a.o.gamma * a.c[(int64_t)(3 + k) * ld + i]) : 0.0;
      a.Yo[(int64_t)k * ld + i] = yp;
      sum += yp;
    }
    // every species but N2 rescaled so that the mass fractions sum to one
    const double scale = (1.0 - yn2) / sum;
    for (int k = 0; k < K; ++k) {
      if (k == n2) continue;
      a.Yo[(int64_t)k * ld + i] *= scale;
    }
    a.Yo[(int64_t)n2 * ld + i] = yn2;
  }
  a.To[i] = T;
  a.po[i] = p;
  // element moles per kg, the ratios of Table 1 and the equivalence ratio
  // (2 n_C + n_H / 2) / n_O
  double nC = 0.0, nH = 0.0, nO = 0.0, nN = 0.0;
  bool ok = isfinite(T) && T >= a.o.T_min;
  for (int k = 0; k < K; ++k) {
    const double y = a.Yo[(int64_t)k * ld + i];
    ok = ok && isfinite(y) && y >= 0.0;
    const double cC = M.compd[a.o.el_C * K + k], cH = M.compd[a.o.el_H * K + k];
    const double cO = M.compd[a.o.el_O * K + k], cN = M.compd[a.o.el_N * K + k];
    if (cC != 0.0) nC += cC * y / M.W[k];
    if (cH != 0.0) nH += cH * y / M.W[k];
    if (cO != 0.0) nO += cO * y / M.W[k];
    if (cN != 0.0) nN += cN * y / M.W[k];
  }
  const double yn2o = a.Yo[(int64_t)n2 * ld + i];
  ok = ok && yn2o >= 0.0 && yn2o < 1.0;
  const double hc = nH / nC, on = nO / nN, phi = (2.0 * nC + 0.5 * nH) / nO;
  ok = ok && isfinite(hc) && hc >= a.o.hc_min && hc <= a.o.hc_max;
  ok = ok && isfinite(on) && on >= a.o.on_min && on <= a.o.on_max;
  ok = ok && isfinite(phi) && phi >= a.o.phi_min && phi <= a.o.phi_max;
  a.keep[i] = ok ? 1 : 0;
}

__global__ void k_sample(DevMech M, SampleArgs a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x)
    sample_one(M, a, i);
}

}  // namespace
}  // namespace chem

using namespace chem;

extern "C" chem_status chem_sample_states(const chem_mech *m, chem_batch seeds, const double *T,
                                          const double *p, const double *Y, const double *c,
                                          const double *s, const double *end_eq,
                                          const double *end_air, const chem_sample_opts *opts,
                                          double *T_out, double *p_out, double *Y_out,
                                          uint8_t *keep, void *stream) {
  if (!m || !opts) {
    set_error("chem_sample_states: null mechanism or options");
    return CHEM_EINVAL;
  }
  const int64_t n = seeds.n;
  if (n < 0 || seeds.ld < n || n > ((int64_t)1 << 40)) {
    set_error("chem_sample_states: bad batch n=%lld ld=%lld", (long long)n, (long long)seeds.ld);
    return CHEM_EINVAL;
  }
  const chem_sample_opts &o = *opts;
  if (o.n2 < 0 || o.n2 >= m->K) {
    set_error("chem_sample_states: N2 index %d outside the %d species", o.n2, m->K);
    return CHEM_EINVAL;
  }
  const int el[4] = {o.el_C, o.el_H, o.el_O, o.el_N};
  for (int a = 0; a < 4; ++a) {
    if (el[a] < 0 || el[a] >= m->E) {
      set_error("chem_sample_states: element index %d outside the %d elements", el[a], m->E);
      return CHEM_EINVAL;
    }
    for (int b = 0; b < a; ++b)
      if (el[a] == el[b]) {
        set_error("chem_sample_states: the C, H, O and N element indices must differ");
        return CHEM_EINVAL;
      }
  }
  if (!(o.alpha >= 0.0) || !(o.beta >= 0.0) || !(o.gamma >= 0.0) || !isfinite(o.T_min)) {
    set_error("chem_sample_states: alpha, beta, gamma must be >= 0 and T_min finite");
    return CHEM_EINVAL;
  }
  if (n == 0) return CHEM_OK;
  if (!T || !p || !Y || !c || !T_out || !p_out || !Y_out || !keep ||
      (s && (!end_eq || !end_air))) {
    set_error("chem_sample_states: null array (the end states are needed with s)");
    return CHEM_EINVAL;
  }
  if (!m->sample_buf) {
    const hipError_t e = hipMalloc((void **)&((chem_mech *)m)->sample_buf,
                                   (size_t)(RANGE_BLOCKS * 6 + 8) * sizeof(double));
    if (e != hipSuccess) {
      set_error("chem_sample_states: cannot allocate the range buffer");
      return CHEM_ENOMEM;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  double *part = m->sample_buf, *ranges = m->sample_buf + RANGE_BLOCKS * 6;
  ProfScope prof("sample_states", st);
  hipLaunchKernelGGL(k_ranges_part, dim3(RANGE_BLOCKS), dim3(RANGE_THREADS), 0, st, n, seeds.ld,
                     T, p, Y, o.n2, part);
  hipLaunchKernelGGL(k_ranges_fin, dim3(1), dim3(64), 0, st, part, RANGE_BLOCKS, ranges);
  SampleArgs a{n, seeds.ld, T, p, Y, c, s, end_eq, end_air, ranges, T_out, p_out, Y_out,
               keep, o};
  int64_t blocks = (n + 255) / 256;
  if (blocks > (1 << 20)) blocks = 1 << 20;  // larger batches loop over the grid
  hipLaunchKernelGGL(k_sample, dim3((unsigned)blocks), dim3(256), 0, st, m->d, a);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}
