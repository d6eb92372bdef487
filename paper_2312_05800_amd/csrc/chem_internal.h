// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "chemstep.h"

namespace chem {

constexpr int KMAX = 63;  // species limit: n = K + 1 <= 64 lanes per cell

// Device-resident mechanism constants (one allocation, see chem_api.hip).
struct DevMech {
  int K, R, E, n;
  const double *W;        // [K] kg/mol
  const double *invW;     // [K]
  const double *Tmid;     // [K]
  const double *nasa_lo;  // [K][7]
  const double *nasa_hi;  // [K][7]
  const double *lnA;      // [R]
  const double *b;        // [R]
  const double *EaR;      // [R] Ea / R_gas, K
  const double *dn;       // [R] sum of product minus reactant coefficients
  const int4 *sp;         // [R] species of slots reactant0, reactant1, product0, product1;
                          //   an empty slot names the dummy species K (the kernels keep
                          //   C = 1 and h = g = 0 for it, so it drops out of every product
                          //   and sum without a branch)
  const int4 *nu;         // [R] their coefficients (0 for empty slots)
  const double *Mel;      // [E][K] element mass per unit mass fraction, A_e a_ek / W_k
  const double *nasa_h;   // [K][7] low-range h/RT polynomial: a1, a2/2, a3/3, a4/4, a5/5, a6, 0
  const double *nasa_hh;  // [K][7] same for the high range
  const double *nasa_s;   // [K][7] low-range s/R: a1, a2, a3/2, a4/3, a5/4, a7, 0
  const double *nasa_sh;  // [K][7] same for the high range
  const double *compd;    // [E][K] atoms of element e in species k
  const double *cpT;      // [2][7][K] the c_p/R, h/RT and s/R polynomials above,
  const double *hT;       //   low range then high range, coefficient-major
  const double *sT;
};

struct StepOpts {
  double rtol, atol_Y, atol_T, h0, h_min;
  int max_steps;
};

}  // namespace chem

struct chem_mech {
  chem::DevMech d;
  void *blob;                      // device allocation behind d
  unsigned long long *counters;    // device work-queue counters
  void *set_buf = nullptr;         // device copy of the last chem_step_sets table
  size_t set_cap = 0;
  void *dset_buf = nullptr;        // offsets and count of chem_step_sets_device's table
  size_t dset_cap = 0;
  double *sample_buf = nullptr;    // training-set sampler: range partials and ranges
  int device;
  int K, R, E;
  // integrator launch shape (0 = default heuristic), set by chem_autotune or
  // chem_set_tuning
  int tune_G = 0, tune_waves = 0;
  double tune_cps = 0.0;
  uint64_t digest = 0;  // FNV-1a of the packed tables (keys the tuning cache)
};

// A captured step: the graph, its executable and the stream it was captured
// on; `release` (if set) runs at destruction (returns the model's workspace
// to growable).
struct chem_graph {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  hipStream_t s = nullptr;
  void (*release)(void *) = nullptr;
  void *owner = nullptr;
};

namespace chem {

// Brackets the launches issued during its lifetime with HIP events on stream
// s when launch timing is enabled (chem_profile_enable); no-op otherwise.
class ProfScope {
 public:
  ProfScope(const char *label, hipStream_t s);
  ~ProfScope();
  ProfScope(const ProfScope &) = delete;
  ProfScope &operator=(const ProfScope &) = delete;

 private:
  const char *label_;
  hipStream_t s_;
  void *a_ = nullptr, *b_ = nullptr;
  bool on_ = false;
};

void set_error(const char *fmt, ...);

// Tuning results kept between runs in the text file named by the environment
// variable CHEM_AUTOTUNE_CACHE (no file: nothing is kept): one line
// "key = value" per tuned problem, the last write of a key winning.
bool tune_cache_get(const std::string &key, std::string *value);
void tune_cache_put(const std::string &key, const std::string &value);
// The current device's architecture name and compute-unit count, for keys.
std::string tune_device_key();
uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull);

// ProfScope is a no-op while suspended (graph capture).
void profile_suspend(bool on);

chem_status hip_fail(hipError_t e, const char *what);

// Records body(stream) on a fresh stream (default priority) into a HIP graph
// and instantiates it; launch timing is suspended meanwhile.  On failure
// nothing is left behind.
template <typename F>
chem_status capture_graph(F &&body, chem_graph **out) {
  if (!out) {
    set_error("graph: null output handle");
    return CHEM_EINVAL;
  }
  *out = nullptr;
  chem_graph *cg = new chem_graph();
  hipError_t e = hipStreamCreateWithFlags(&cg->s, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete cg;
    return hip_fail(e, "graph: hipStreamCreateWithFlags");
  }
  chem_status st = CHEM_OK;
  profile_suspend(true);
  e = hipStreamBeginCapture(cg->s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = body(cg->s);
    const hipError_t e2 = hipStreamEndCapture(cg->s, &cg->g);
    if (st == CHEM_OK && e2 != hipSuccess) st = hip_fail(e2, "graph: hipStreamEndCapture");
    if (st == CHEM_OK) {
      const hipError_t e3 = hipGraphInstantiate(&cg->e, cg->g, nullptr, nullptr, 0);
      if (e3 != hipSuccess) st = hip_fail(e3, "graph: hipGraphInstantiate");
    }
  } else {
    st = hip_fail(e, "graph: hipStreamBeginCapture");
  }
  profile_suspend(false);
  if (st != CHEM_OK) {
    if (cg->e) (void)hipGraphExecDestroy(cg->e);
    if (cg->g) (void)hipGraphDestroy(cg->g);
    (void)hipStreamDestroy(cg->s);
    delete cg;
    return st;
  }
  *out = cg;
  return CHEM_OK;
}

#define CHEM_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return chem::hip_fail(e_, #call); \
  } while (0)

StepOpts resolve_opts(const chem_step_opts *o);

// launchers (chem_kernels.hip)
chem_status launch_rates(const chem_mech *m, int64_t n, int64_t ld, const double *T,
                         const double *p, const double *Y, double *wdot, double *dTdt,
                         double *kfkr, hipStream_t s);
// smallest lane group (16, 32 or 64) that holds n = K + 1 components
int group_size(int n);
// LDS bytes of one integrator wavefront with G lanes per cell
size_t step_lds_bytes(const chem_mech *m, int G);
// resident integrator wavefronts per CU that the LDS allows (1..32)
int max_waves_per_cu(size_t sh);
chem_status launch_step(const chem_mech *m, int64_t n, int64_t ld, double dt,
                        const double *dt_cell, double *T, const double *p, double *Y,
                        double *RR, double *h_hint, int32_t *stats, const StepOpts &o,
                        const int32_t *index, hipStream_t s,
                        const unsigned long long *n_dev = nullptr, uint8_t *flags = nullptr,
                        const chem_set *sets = nullptr, const int64_t *set_off = nullptr,
                        int n_sets = 0);
// Offsets and total cell count of a device set table (see k_set_offsets).
chem_status launch_set_offsets(const chem_set *sets, int n_sets, int64_t *off,
                               unsigned long long *total, int32_t *n_bad, hipStream_t s);

}  // namespace chem
