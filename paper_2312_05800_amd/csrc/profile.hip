// Opt-in launch timing: when enabled, every library launch is bracketed by a
// pair of HIP events recorded on the launch's own stream; chem_profile_read
// synchronises and returns per-label launch counts and total milliseconds.
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "chem_internal.h"

namespace chem {
namespace {

struct Rec {
  const char *label;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
bool g_suspended = false;  // during graph capture
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

void profile_suspend(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_suspended = on;
}

ProfScope::ProfScope(const char *label, hipStream_t s) : label_(label), s_(s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || g_suspended) return;
  a_ = get_event();
  b_ = get_event();
  if (a_ && b_) {
    (void)hipEventRecord((hipEvent_t)a_, s);
    on_ = true;
  }
}

ProfScope::~ProfScope() {
  if (!on_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord((hipEvent_t)b_, s_);
  g_recs.push_back(Rec{label_, (hipEvent_t)a_, (hipEvent_t)b_});
}

}  // namespace chem

extern "C" void chem_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(chem::g_mu);
  chem::g_on = on != 0;
}

extern "C" int32_t chem_profile_read(char (*names)[48], int64_t *launches, double *total_ms,
                                     int32_t cap) {
  std::vector<chem::Rec> recs;
  {
    std::lock_guard<std::mutex> lk(chem::g_mu);
    recs.swap(chem::g_recs);
  }
  std::vector<std::string> lab;
  std::vector<int64_t> cnt;
  std::vector<double> tot;
  for (auto &r : recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      size_t i = 0;
      for (; i < lab.size(); ++i)
        if (lab[i] == r.label) break;
      if (i == lab.size()) {
        lab.emplace_back(r.label);
        cnt.push_back(0);
        tot.push_back(0.0);
      }
      cnt[i] += 1;
      tot[i] += ms;
    }
    std::lock_guard<std::mutex> lk(chem::g_mu);
    chem::g_pool.push_back(r.a);
    chem::g_pool.push_back(r.b);
  }
  int32_t n = 0;
  for (size_t i = 0; i < lab.size() && n < cap; ++i, ++n) {
    if (names) {
      strncpy(names[n], lab[i].c_str(), 47);
      names[n][47] = 0;
    }
    if (launches) launches[n] = cnt[i];
    if (total_ms) total_ms[n] = tot[i];
  }
  return n;
}

// ------------------------------------------------ attainable peaks
//
// Throughput probes for the three units the step's kernels are priced
// against: dense BF16 and FP8 MFMA (v_mfma_f32_16x16x32_bf16 and
// v_mfma_scale_f32_16x16x128_f8f6f4 with unit block scales), and FP64 vector
// FMA.  Every wave runs eight independent accumulator chains so that issue,
// not latency, bounds it; the result feeds a comparison that the compiler
// cannot decide, so no work is removed.

namespace chem {
namespace {

typedef __bf16 pk_bf16x8 __attribute__((ext_vector_type(8)));
typedef float pk_f32x4 __attribute__((ext_vector_type(4)));
typedef int pk_i32x8 __attribute__((ext_vector_type(8)));

constexpr int PEAK_CHAINS = 8;
constexpr int PEAK_BLOCKS = 2048;  // 256 threads each: 32 waves per CU over 256 CUs
constexpr int PEAK_THREADS = 256;

__global__ __launch_bounds__(256) void k_peak_bf16(float *sink, int iters) {
  const float v = 1e-3f * (float)(threadIdx.x & 7);
  pk_bf16x8 a, b;
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(v + 1e-3f * i);
    b[i] = (__bf16)(v - 1e-3f * i);
  }
  pk_f32x4 acc[PEAK_CHAINS] = {};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < PEAK_CHAINS; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
  for (int c = 0; c < PEAK_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 1234.5f) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_fp8(float *sink, int iters) {
  // E4M3 bytes of small magnitude (exponent field 1..3) in every lane
  const int byte = 0x08 + (int)(threadIdx.x & 15);
  const int w = byte | (byte << 8) | (byte << 16) | (byte << 24);
  pk_i32x8 a, b;
  for (int i = 0; i < 8; ++i) {
    a[i] = w;
    b[i] = w ^ (i << 1);
  }
  pk_f32x4 acc[PEAK_CHAINS] = {};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < PEAK_CHAINS; ++c)
      acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[c], 0, 0, 0, 127, 0,
                                                                127);
  }
  float s = 0.0f;
  for (int c = 0; c < PEAK_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 1234.5f) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_fp64(double *sink, int iters) {
  double x[PEAK_CHAINS];
  for (int c = 0; c < PEAK_CHAINS; ++c) x[c] = 1.0 + 1e-3 * (double)(threadIdx.x + c);
  const double m = 0.9999999, a = 1e-7;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < PEAK_CHAINS; ++c) x[c] = fma(x[c], m, a);
  }
  double s = 0.0;
  for (int c = 0; c < PEAK_CHAINS; ++c) s += x[c];
  if (s == 1234.5) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <typename F>
chem_status time_launch(F &&launch, hipStream_t s, double *ms) {
  hipEvent_t a = nullptr, b = nullptr;
  CHEM_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return hip_fail(hipErrorOutOfMemory, "chem_measure_peaks: hipEventCreate");
  }
  launch();  // warm-up (clocks, code object)
  (void)hipEventRecord(a, s);
  launch();
  (void)hipEventRecord(b, s);
  hipError_t e = hipEventSynchronize(b);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "chem_measure_peaks: timing");
  *ms = t;
  return CHEM_OK;
}

}  // namespace
}  // namespace chem

extern "C" chem_status chem_measure_peaks(double *tflops, void *stream) {
  using namespace chem;
  if (!tflops) {
    set_error("chem_measure_peaks: null output");
    return CHEM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  void *sink = nullptr;
  CHEM_HIP(hipMalloc(&sink, (size_t)PEAK_BLOCKS * PEAK_THREADS * sizeof(double)));
  const double waves = (double)PEAK_BLOCKS * PEAK_THREADS / 64.0;
  const double threads = (double)PEAK_BLOCKS * PEAK_THREADS;
  const int it_mfma = 2048, it_f64 = 4096;
  double ms[3] = {0, 0, 0};
  chem_status st = time_launch(
      [&] {
        hipLaunchKernelGGL(k_peak_bf16, dim3(PEAK_BLOCKS), dim3(PEAK_THREADS), 0, s,
                           (float *)sink, it_mfma);
      },
      s, &ms[0]);
  if (st == CHEM_OK)
    st = time_launch(
        [&] {
          hipLaunchKernelGGL(k_peak_fp8, dim3(PEAK_BLOCKS), dim3(PEAK_THREADS), 0, s,
                             (float *)sink, it_mfma);
        },
        s, &ms[1]);
  if (st == CHEM_OK)
    st = time_launch(
        [&] {
          hipLaunchKernelGGL(k_peak_fp64, dim3(PEAK_BLOCKS), dim3(PEAK_THREADS), 0, s,
                             (double *)sink, it_f64);
        },
        s, &ms[2]);
  (void)hipFree(sink);
  if (st != CHEM_OK) return st;
  const double f_bf16 = waves * it_mfma * PEAK_CHAINS * (16.0 * 16.0 * 32.0 * 2.0);
  const double f_fp8 = waves * it_mfma * PEAK_CHAINS * (16.0 * 16.0 * 128.0 * 2.0);
  const double f_fp64 = threads * it_f64 * PEAK_CHAINS * 2.0;
  tflops[0] = f_bf16 / (ms[0] * 1e-3) / 1e12;
  tflops[1] = f_fp8 / (ms[1] * 1e-3) / 1e12;
  tflops[2] = f_fp64 / (ms[2] * 1e-3) / 1e12;
  return CHEM_OK;
}
