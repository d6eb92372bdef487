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
