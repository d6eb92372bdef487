// Host side of the C ABI: status strings, error reporting, mechanism upload
// and argument validation for chem_rates / chem_step.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <mutex>
#include <sstream>
#include <utility>
#include <vector>
#include <vector>

#include "chem_internal.h"

namespace chem {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

chem_status hip_fail(hipError_t e, const char *what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return CHEM_EHIP;
}

StepOpts resolve_opts(const chem_step_opts *o) {
  StepOpts r{1e-6, 1e-12, 1e-6, 1e-8, 1e-20, 100000};
  if (o) {
    r.rtol = o->rtol;
    r.atol_Y = o->atol_Y;
    r.atol_T = o->atol_T;
    r.h0 = o->h0;
    r.h_min = o->h_min;
    r.max_steps = o->max_steps;
  }
  return r;
}

}  // namespace chem

using namespace chem;

extern "C" const char *chem_status_string(chem_status s) {
  switch (s) {
    case CHEM_OK: return "CHEM_OK";
    case CHEM_EINVAL: return "CHEM_EINVAL";
    case CHEM_ENOMEM: return "CHEM_ENOMEM";
    case CHEM_EHIP: return "CHEM_EHIP";
    case CHEM_EMECH: return "CHEM_EMECH";
    case CHEM_EMODEL: return "CHEM_EMODEL";
    case CHEM_EUNSUPPORTED: return "CHEM_EUNSUPPORTED";
  }
  return "CHEM_UNKNOWN";
}

extern "C" const char *chem_last_error(void) { return g_err; }

namespace {

// Packs host arrays into one byte blob with 256-byte aligned sections.
struct Packer {
  std::vector<unsigned char> buf;
  size_t add(const void *p, size_t bytes) {
    size_t off = (buf.size() + 255) & ~size_t(255);
    buf.resize(off + bytes);
    if (bytes) memcpy(buf.data() + off, p, bytes);
    return off;
  }
};

}  // namespace

extern "C" chem_status chem_mech_create(const chem_mech_desc *d, chem_mech **out) {
  if (!d || !out) {
    set_error("chem_mech_create: null argument");
    return CHEM_EINVAL;
  }
  *out = nullptr;
  const int K = d->K, R = d->R, E = d->E;
  if (K < 1 || R < 0 || E < 1 || !d->W || !d->comp || !d->awt || !d->nasa ||
      (R > 0 && (!d->rsp || !d->rnu || !d->A || !d->b || !d->Ea))) {
    set_error("chem_mech_create: bad sizes or null arrays (K=%d R=%d E=%d)", K, R, E);
    return CHEM_EINVAL;
  }
  if (K > KMAX) {
    set_error("chem_mech_create: K=%d exceeds the limit of %d species", K, KMAX);
    return CHEM_EUNSUPPORTED;
  }
  for (int k = 0; k < K; ++k) {
    if (!(d->W[k] > 0.0) || !isfinite(d->W[k])) {
      set_error("chem_mech_create: W[%d] must be finite and positive", k);
      return CHEM_EMECH;
    }
    const double *c = d->nasa + 17 * k;
    for (int j = 0; j < 17; ++j)
      if (!isfinite(c[j])) {
        set_error("chem_mech_create: non-finite NASA coefficient of species %d", k);
        return CHEM_EMECH;
      }
  }
  for (int r = 0; r < R; ++r) {
    const int32_t *sp = d->rsp + 4 * r, *nu = d->rnu + 4 * r;
    if (!(d->A[r] > 0.0) || !isfinite(d->A[r]) || !isfinite(d->b[r]) || !isfinite(d->Ea[r])) {
      set_error("chem_mech_create: reaction %d has a non-positive or non-finite A/b/Ea", r);
      return CHEM_EMECH;
    }
    std::vector<long> bal(E, 0);
    int nreac = 0, nprod = 0;
    for (int s = 0; s < 4; ++s) {
      if (sp[s] < 0) continue;
      if (sp[s] >= K || nu[s] < 1 || nu[s] > 2) {
        set_error("chem_mech_create: reaction %d slot %d: species %d / coefficient %d invalid", r,
                  s, sp[s], nu[s]);
        return CHEM_EMECH;
      }
      for (int t = 0; t < s; ++t)
        if (sp[t] == sp[s]) {
          set_error("chem_mech_create: reaction %d lists species %d twice", r, sp[s]);
          return CHEM_EMECH;
        }
      (s < 2 ? nreac : nprod)++;
      for (int e = 0; e < E; ++e) bal[e] += (s < 2 ? -1 : 1) * (long)nu[s] * d->comp[sp[s] * E + e];
    }
    if (nreac == 0 || nprod == 0) {
      set_error("chem_mech_create: reaction %d needs at least one reactant and one product", r);
      return CHEM_EMECH;
    }
    for (int e = 0; e < E; ++e)
      if (bal[e] != 0) {
        set_error("chem_mech_create: reaction %d does not conserve element %d", r, e);
        return CHEM_EMECH;
      }
  }

  // host-side tables
  std::vector<double> W(K), invW(K), Tmid(K), lo(7 * K), hi(7 * K);
  for (int k = 0; k < K; ++k) {
    W[k] = d->W[k];
    invW[k] = 1.0 / d->W[k];
    Tmid[k] = d->nasa[17 * k + 1];
    for (int j = 0; j < 7; ++j) {
      lo[7 * k + j] = d->nasa[17 * k + 3 + j];
      hi[7 * k + j] = d->nasa[17 * k + 10 + j];
    }
  }
  std::vector<double> lnA(R), bb(R), EaR(R), dn(R);
  std::vector<int4> sp4(R), nu4(R);
  const double RGAS = 8.314462618;
  for (int r = 0; r < R; ++r) {
    const int32_t *sp = d->rsp + 4 * r, *nu = d->rnu + 4 * r;
    lnA[r] = log(d->A[r]);
    bb[r] = d->b[r];
    EaR[r] = d->Ea[r] / RGAS;
    int dnn = 0;
    int s4[4], n4[4];
    for (int s = 0; s < 4; ++s) {
      s4[s] = sp[s] < 0 ? K : sp[s];  // empty slot: the dummy species K (see DevMech::sp)
      n4[s] = sp[s] < 0 ? 0 : nu[s];
      dnn += (s < 2 ? -1 : 1) * n4[s];
    }
    dn[r] = dnn;
    sp4[r] = make_int4(s4[0], s4[1], s4[2], s4[3]);
    nu4[r] = make_int4(n4[0], n4[1], n4[2], n4[3]);
  }
  std::vector<double> compd((size_t)E * K);
  for (int e = 0; e < E; ++e)
    for (int k = 0; k < K; ++k) compd[(size_t)e * K + k] = d->comp[k * E + e];
  std::vector<double> Mel((size_t)E * K);
  for (int e = 0; e < E; ++e)
    for (int k = 0; k < K; ++k) Mel[(size_t)e * K + k] = d->comp[k * E + e] * d->awt[e] / d->W[k];

  // thermo polynomials with the constant divisors folded in
  std::vector<double> nh(7 * K), nhh(7 * K), ns(7 * K), nsh(7 * K);
  for (int k = 0; k < K; ++k)
    for (int r = 0; r < 2; ++r) {
      const double *a = d->nasa + 17 * k + (r == 0 ? 3 : 10);
      double *h = (r == 0 ? nh.data() : nhh.data()) + 7 * k;
      double *e = (r == 0 ? ns.data() : nsh.data()) + 7 * k;
      h[0] = a[0]; h[1] = a[1] / 2.0; h[2] = a[2] / 3.0; h[3] = a[3] / 4.0; h[4] = a[4] / 5.0;
      h[5] = a[5]; h[6] = 0.0;
      e[0] = a[0]; e[1] = a[1]; e[2] = a[2] / 2.0; e[3] = a[3] / 3.0; e[4] = a[4] / 4.0;
      e[5] = a[6]; e[6] = 0.0;
    }
  // the same polynomials coefficient-major, [range][coefficient][species], so
  // that one coefficient of consecutive species is one contiguous load
  std::vector<double> cpT(14 * (size_t)K), hT(14 * (size_t)K), sT(14 * (size_t)K);
  for (int r = 0; r < 2; ++r)
    for (int i = 0; i < 7; ++i)
      for (int k = 0; k < K; ++k) {
        const size_t t = ((size_t)r * 7 + i) * K + k;
        cpT[t] = (r == 0 ? lo : hi)[7 * k + i];
        hT[t] = (r == 0 ? nh : nhh)[7 * k + i];
        sT[t] = (r == 0 ? ns : nsh)[7 * k + i];
      }
  if (R >= 65536) {
    set_error("chem_mech_create: at most 65535 reactions");
    return CHEM_EUNSUPPORTED;
  }

  Packer pk;
  size_t oW = pk.add(W.data(), K * 8), oiW = pk.add(invW.data(), K * 8),
         oTm = pk.add(Tmid.data(), K * 8), olo = pk.add(lo.data(), 7 * K * 8),
         ohi = pk.add(hi.data(), 7 * K * 8), olnA = pk.add(lnA.data(), R * 8),
         ob = pk.add(bb.data(), R * 8), oEa = pk.add(EaR.data(), R * 8),
         odn = pk.add(dn.data(), R * 8), osp = pk.add(sp4.data(), R * sizeof(int4)),
         onu = pk.add(nu4.data(), R * sizeof(int4)), oM = pk.add(Mel.data(), Mel.size() * 8),
         onh = pk.add(nh.data(), nh.size() * 8), onhh = pk.add(nhh.data(), nhh.size() * 8),
         ons = pk.add(ns.data(), ns.size() * 8), onsh = pk.add(nsh.data(), nsh.size() * 8),
         ocpT = pk.add(cpT.data(), cpT.size() * 8), ohT = pk.add(hT.data(), hT.size() * 8),
         osT = pk.add(sT.data(), sT.size() * 8), ocd = pk.add(compd.data(), compd.size() * 8);

  chem_mech *m = new chem_mech();
  m->K = K;
  m->R = R;
  m->E = E;
  hipError_t e = hipGetDevice(&m->device);
  if (e == hipSuccess) e = hipMalloc(&m->blob, pk.buf.size());
  if (e != hipSuccess) {
    delete m;
    set_error("chem_mech_create: device allocation: %s", hipGetErrorString(e));
    return CHEM_ENOMEM;
  }
  e = hipMalloc((void **)&m->counters, 64 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    (void)hipFree(m->blob);
    delete m;
    set_error("chem_mech_create: device allocation: %s", hipGetErrorString(e));
    return CHEM_ENOMEM;
  }
  m->digest = fnv1a(pk.buf.data(), pk.buf.size());
  e = hipMemcpy(m->blob, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->counters, 0, 64 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    (void)hipFree(m->blob);
    (void)hipFree(m->counters);
    delete m;
    return hip_fail(e, "chem_mech_create: upload");
  }
  const unsigned char *base = (const unsigned char *)m->blob;
  DevMech &dm = m->d;
  dm.K = K;
  dm.R = R;
  dm.E = E;
  dm.n = K + 1;
  dm.W = (const double *)(base + oW);
  dm.invW = (const double *)(base + oiW);
  dm.Tmid = (const double *)(base + oTm);
  dm.nasa_lo = (const double *)(base + olo);
  dm.nasa_hi = (const double *)(base + ohi);
  dm.lnA = (const double *)(base + olnA);
  dm.b = (const double *)(base + ob);
  dm.EaR = (const double *)(base + oEa);
  dm.dn = (const double *)(base + odn);
  dm.sp = (const int4 *)(base + osp);
  dm.nu = (const int4 *)(base + onu);
  dm.Mel = (const double *)(base + oM);
  dm.nasa_h = (const double *)(base + onh);
  dm.nasa_hh = (const double *)(base + onhh);
  dm.nasa_s = (const double *)(base + ons);
  dm.nasa_sh = (const double *)(base + onsh);
  dm.cpT = (const double *)(base + ocpT);
  dm.hT = (const double *)(base + ohT);
  dm.sT = (const double *)(base + osT);
  dm.compd = (const double *)(base + ocd);
  *out = m;
  return CHEM_OK;
}

extern "C" void chem_mech_destroy(chem_mech *m) {
  if (!m) return;
  if (m->set_buf) (void)hipFree(m->set_buf);
  if (m->dset_buf) (void)hipFree(m->dset_buf);
  if (m->sample_buf) (void)hipFree(m->sample_buf);
  (void)hipFree(m->blob);
  (void)hipFree(m->counters);
  delete m;
}

extern "C" int32_t chem_mech_num_species(const chem_mech *m) { return m ? m->K : -1; }
extern "C" int32_t chem_mech_num_reactions(const chem_mech *m) { return m ? m->R : -1; }

static chem_status check_batch(const char *fn, const chem_mech *m, chem_batch b) {
  if (!m) {
    set_error("%s: null mechanism", fn);
    return CHEM_EINVAL;
  }
  if (b.n < 0 || b.ld < b.n || b.n > (int64_t)1 << 40) {
    set_error("%s: bad batch n=%lld ld=%lld", fn, (long long)b.n, (long long)b.ld);
    return CHEM_EINVAL;
  }
  return CHEM_OK;
}

extern "C" chem_status chem_rates(const chem_mech *m, chem_batch batch, const double *T,
                                  const double *p, const double *Y, double *wdot, double *dTdt,
                                  double *kfkr, void *stream) {
  chem_status st = check_batch("chem_rates", m, batch);
  if (st != CHEM_OK) return st;
  if (batch.n == 0) return CHEM_OK;
  if (!T || !p || !Y || !wdot) {
    set_error("chem_rates: T, p, Y and wdot must be non-null");
    return CHEM_EINVAL;
  }
  return launch_rates(m, batch.n, batch.ld, T, p, Y, wdot, dTdt, kfkr, (hipStream_t)stream);
}

extern "C" chem_status chem_step(const chem_mech *m, chem_batch batch, double dt,
                                 const double *dt_cell, double *T, const double *p, double *Y,
                                 double *RR, double *h_hint, int32_t *stats,
                                 const chem_step_opts *opts, void *stream) {
  chem_status st = check_batch("chem_step", m, batch);
  if (st != CHEM_OK) return st;
  if (batch.n == 0) return CHEM_OK;
  if (!T || !p || !Y) {
    set_error("chem_step: T, p and Y must be non-null");
    return CHEM_EINVAL;
  }
  if (!dt_cell && !(dt > 0.0 && isfinite(dt))) {
    set_error("chem_step: dt must be finite and positive (got %g)", dt);
    return CHEM_EINVAL;
  }
  StepOpts o = resolve_opts(opts);
  if (!(o.rtol > 0.0) || !(o.atol_Y >= 0.0) || !(o.atol_T >= 0.0) || !(o.h0 > 0.0) ||
      !(o.h_min >= 0.0) || o.max_steps < 1) {
    set_error("chem_step: invalid options (rtol>0, atol>=0, h0>0, h_min>=0, max_steps>=1)");
    return CHEM_EINVAL;
  }
  return launch_step(m, batch.n, batch.ld, dt, dt_cell, T, p, Y, RR, h_hint, stats, o, nullptr,
                     (hipStream_t)stream);
}

namespace {
// Validates a set table and lays it out in device memory *buf (grown to
// fit; capacity *cap): the descriptors, then the first queue index of every
// set.  The copy has completed on `s` when this returns (its pageable source
// is a local).
chem_status stage_sets(const char *fn, int32_t n_sets, const chem_set *sets, hipStream_t s,
                       void **buf, size_t *cap, const chem_set **dsets, const int64_t **doff,
                       int64_t *total) {
  std::vector<int64_t> off(n_sets + 1, 0);
  for (int i = 0; i < n_sets; ++i) {
    const chem_set &c = sets[i];
    if (c.n < 0 || c.ld < c.n || (c.n > 0 && (!c.T || !c.p || !c.Y)) ||
        (c.n > 0 && !(c.dt > 0.0 && isfinite(c.dt)))) {
      set_error("%s: set %d has bad sizes, null arrays or dt", fn, i);
      return CHEM_EINVAL;
    }
    off[i + 1] = off[i] + c.n;
  }
  *total = off[n_sets];
  if (*total == 0) return CHEM_OK;
  const size_t tb = (size_t)n_sets * sizeof(chem_set);
  const size_t ob = (tb + 255) & ~size_t(255);
  const size_t need = ob + off.size() * 8;
  if (*cap < need) {
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (hipMalloc(buf, need) != hipSuccess) {
      *buf = nullptr;
      set_error("%s: cannot allocate the set table", fn);
      return CHEM_ENOMEM;
    }
    *cap = need;
  }
  std::vector<unsigned char> host(need);
  memcpy(host.data(), sets, tb);
  memcpy(host.data() + ob, off.data(), off.size() * 8);
  CHEM_HIP(hipMemcpyAsync(*buf, host.data(), need, hipMemcpyHostToDevice, s));
  CHEM_HIP(hipStreamSynchronize(s));
  *dsets = (const chem_set *)*buf;
  *doff = (const int64_t *)((unsigned char *)*buf + ob);
  return CHEM_OK;
}

chem_status check_sets_call(const char *fn, const chem_mech *m, int32_t n_sets,
                            const chem_set *sets, const chem_step_opts *opts, StepOpts *o) {
  if (!m || n_sets < 0 || (n_sets > 0 && !sets)) {
    set_error("%s: null mechanism or set table", fn);
    return CHEM_EINVAL;
  }
  if (n_sets > (1 << 20)) {
    set_error("%s: at most 2^20 sets", fn);
    return CHEM_EINVAL;
  }
  *o = resolve_opts(opts);
  if (!(o->rtol > 0.0) || !(o->atol_Y >= 0.0) || !(o->atol_T >= 0.0) || !(o->h0 > 0.0) ||
      !(o->h_min >= 0.0) || o->max_steps < 1) {
    set_error("%s: invalid options", fn);
    return CHEM_EINVAL;
  }
  return CHEM_OK;
}
}  // namespace

extern "C" chem_status chem_step_sets(const chem_mech *m, int32_t n_sets, const chem_set *sets,
                                      const chem_step_opts *opts, void *stream) {
  StepOpts o;
  chem_status st = check_sets_call("chem_step_sets", m, n_sets, sets, opts, &o);
  if (st != CHEM_OK) return st;
  chem_mech *mm = const_cast<chem_mech *>(m);
  hipStream_t s = (hipStream_t)stream;
  const chem_set *dsets = nullptr;
  const int64_t *doff = nullptr;
  int64_t total = 0;
  st = stage_sets("chem_step_sets", n_sets, sets, s, &mm->set_buf, &mm->set_cap, &dsets, &doff,
                  &total);
  if (st != CHEM_OK || total == 0) return st;
  return launch_step(m, total, 0, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                     nullptr, o, nullptr, s, nullptr, nullptr, dsets, doff, n_sets);
}

// ------------------------------------------------------ launch autotuning

namespace {
bool valid_opts(const StepOpts &o) {
  return o.rtol > 0.0 && o.atol_Y >= 0.0 && o.atol_T >= 0.0 && o.h0 > 0.0 && o.h_min >= 0.0 &&
         o.max_steps >= 1;
}

// the waves-per-CU value a launch with G lanes per cell uses
int resolved_waves(const chem_mech *m, int G) {
  const int wmax = max_waves_per_cu(step_lds_bytes(m, G));
  return (m->tune_waves > 0 && m->tune_waves < wmax) ? m->tune_waves : wmax;
}
}  // namespace

extern "C" chem_status chem_set_tuning(chem_mech *m, const chem_tuning *t) {
  if (!m) {
    set_error("chem_set_tuning: null mechanism");
    return CHEM_EINVAL;
  }
  if (!t) {
    m->tune_G = 0;
    m->tune_waves = 0;
    m->tune_cps = 0.0;
    return CHEM_OK;
  }
  const int g0 = group_size(m->d.n), G = t->lanes_per_cell;
  if (G != 0 && !((G == 16 || G == 32 || G == 64) && G >= g0)) {
    set_error("chem_set_tuning: lanes_per_cell must be 0 or 16/32/64 >= %d", g0);
    return CHEM_EINVAL;
  }
  if (t->waves_per_cu < 0 || t->waves_per_cu > 32) {
    set_error("chem_set_tuning: waves_per_cu must be in [0, 32]");
    return CHEM_EINVAL;
  }
  m->tune_G = G;
  m->tune_waves = t->waves_per_cu;
  m->tune_cps = 0.0;
  return CHEM_OK;
}

extern "C" chem_status chem_get_tuning(const chem_mech *m, chem_tuning *out) {
  if (!m || !out) {
    set_error("chem_get_tuning: null argument");
    return CHEM_EINVAL;
  }
  const int G = m->tune_G ? m->tune_G : group_size(m->d.n);
  out->lanes_per_cell = G;
  out->waves_per_cu = resolved_waves(m, G);
  out->cells_per_s = m->tune_cps;
  return CHEM_OK;
}

extern "C" chem_status chem_autotune(chem_mech *m, chem_batch sample, double dt,
                                     const double *T, const double *p, const double *Y,
                                     const chem_step_opts *opts, void *stream,
                                     chem_tuning *best) {
  chem_status st = check_batch("chem_autotune", m, sample);
  if (st != CHEM_OK) return st;
  if (sample.n < 1 || !T || !p || !Y || !(dt > 0.0 && isfinite(dt))) {
    set_error("chem_autotune: needs a non-empty sample, non-null arrays and a positive dt");
    return CHEM_EINVAL;
  }
  const StepOpts o = resolve_opts(opts);
  if (!valid_opts(o)) {
    set_error("chem_autotune: invalid options");
    return CHEM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = sample.n;
  const int K = m->K;
  // a shape measured before for this device, mechanism, step and controls
  // (CHEM_AUTOTUNE_CACHE) is taken without timing
  char kb[256];
  snprintf(kb, sizeof(kb), "chem_step %s K=%d R=%d mech=%016llx dt=%.6g rtol=%.3g atol=%.3g",
           tune_device_key().c_str(), K, m->R, (unsigned long long)m->digest, dt, o.rtol,
           o.atol_Y);
  std::string cached;
  if (tune_cache_get(kb, &cached)) {
    int cg = 0, cw = 0;
    double ccps = 0.0;
    if (sscanf(cached.c_str(), "%d %d %lf", &cg, &cw, &ccps) == 3 && cg >= group_size(m->d.n) &&
        cg <= 64 && (cg & (cg - 1)) == 0 && cw >= 1 &&
        cw <= max_waves_per_cu(step_lds_bytes(m, cg))) {
      m->tune_G = cg;
      m->tune_waves = cw;
      m->tune_cps = ccps;
      if (best) {
        best->lanes_per_cell = cg;
        best->waves_per_cu = resolved_waves(m, cg);
        best->cells_per_s = ccps;
      }
      return CHEM_OK;
    }
  }
  // candidates: every usable lane group, and 1/4 .. 4/4 of the waves per CU
  // its LDS allows
  struct Cand {
    int G, w;
  };
  std::vector<Cand> cands;
  for (int G = group_size(m->d.n); G <= 64; G *= 2) {
    const int wmax = max_waves_per_cu(step_lds_bytes(m, G));
    int last = 0;
    for (int q = 4; q >= 1; --q) {
      const int w = (wmax * q + 3) / 4;
      if (w >= 1 && w != last) cands.push_back(Cand{G, w});
      last = w;
    }
  }
  double *buf = nullptr;
  hipEvent_t ea = nullptr, eb = nullptr;
  auto cleanup = [&]() {
    if (ea) (void)hipEventDestroy(ea);
    if (eb) (void)hipEventDestroy(eb);
    if (buf) (void)hipFree(buf);
  };
  if (hipMalloc(&buf, (size_t)n * (K + 1) * sizeof(double)) != hipSuccess) {
    set_error("chem_autotune: cannot allocate %lld scratch cells", (long long)n);
    return CHEM_ENOMEM;
  }
  double *const Ts = buf, *const Ys = buf + n;
  if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
    cleanup();
    set_error("chem_autotune: hipEventCreate failed");
    return CHEM_EHIP;
  }
  const int saveG = m->tune_G, saveW = m->tune_waves;
  Cand bc{saveG, saveW};
  float best_ms = INFINITY;
  for (const Cand &c : cands) {
    m->tune_G = c.G;
    m->tune_waves = c.w;
    float ms = INFINITY;
    for (int rep = 0; rep < 2 && st == CHEM_OK; ++rep) {  // the first run warms up
      hipError_t e = hipMemcpyAsync(Ts, T, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(Ys, (size_t)n * 8, Y, (size_t)sample.ld * 8, (size_t)n * 8, K,
                             hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipEventRecord(ea, s);
      if (e != hipSuccess) {
        st = hip_fail(e, "chem_autotune: staging the sample");
        break;
      }
      st = launch_step(m, n, n, dt, nullptr, Ts, p, Ys, nullptr, nullptr, nullptr, o, nullptr, s);
      if (st != CHEM_OK) break;
      e = hipEventRecord(eb, s);
      if (e == hipSuccess) e = hipEventSynchronize(eb);
      float t = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, ea, eb);
      if (e != hipSuccess) {
        st = hip_fail(e, "chem_autotune: timing");
        break;
      }
      ms = fminf(ms, t);
    }
    if (st == CHEM_EUNSUPPORTED) {  // this lane group does not fit the LDS
      st = CHEM_OK;
      continue;
    }
    if (st != CHEM_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      bc = c;
    }
  }
  cleanup();
  if (st != CHEM_OK || !(best_ms < INFINITY)) {
    m->tune_G = saveG;
    m->tune_waves = saveW;
    if (st == CHEM_OK) {
      set_error("chem_autotune: no launch shape could run");
      st = CHEM_EUNSUPPORTED;
    }
    return st;
  }
  m->tune_G = bc.G;
  m->tune_waves = bc.w;
  m->tune_cps = (double)n / (best_ms * 1e-3);
  {
    char vb[96];
    snprintf(vb, sizeof(vb), "%d %d %.17g", bc.G, bc.w, m->tune_cps);
    tune_cache_put(kb, vb);
  }
  if (best) {
    best->lanes_per_cell = bc.G;
    best->waves_per_cu = resolved_waves(m, bc.G);
    best->cells_per_s = m->tune_cps;
  }
  return CHEM_OK;
}

// ------------------------------------------------------- captured steps

extern "C" chem_status chem_step_graph_create(const chem_mech *m, chem_batch batch, double dt,
                                              const double *dt_cell, double *T, const double *p,
                                              double *Y, double *RR, double *h_hint,
                                              int32_t *stats, const chem_step_opts *opts,
                                              void *stream, chem_graph **out) {
  (void)stream;  // nothing runs before the capture
  chem_status st = check_batch("chem_step_graph_create", m, batch);
  if (st != CHEM_OK) return st;
  if (batch.n < 1) {
    set_error("chem_step_graph_create: empty batch");
    return CHEM_EINVAL;
  }
  return capture_graph(
      [&](hipStream_t cs) {
        return chem_step(m, batch, dt, dt_cell, T, p, Y, RR, h_hint, stats, opts, cs);
      },
      out);
}

namespace {
void free_device(void *p) { (void)hipFree(p); }
}  // namespace

extern "C" chem_status chem_step_sets_device(const chem_mech *m, int32_t n_sets,
                                             const chem_set *sets, const chem_step_opts *opts,
                                             int32_t *n_bad, void *stream) {
  StepOpts o;
  chem_status st = check_sets_call("chem_step_sets_device", m, n_sets, sets, opts, &o);
  if (st != CHEM_OK) return st;
  if (n_sets == 0) return CHEM_OK;
  chem_mech *mm = const_cast<chem_mech *>(m);
  hipStream_t s = (hipStream_t)stream;
  // offsets [n_sets + 1] and the total count, in memory the handle owns
  const size_t need = ((size_t)(n_sets + 1) * 8 + 255) / 256 * 256 + 256;
  if (mm->dset_cap < need) {
    if (mm->dset_buf) (void)hipFree(mm->dset_buf);
    mm->dset_buf = nullptr;
    mm->dset_cap = 0;
    if (hipMalloc(&mm->dset_buf, need) != hipSuccess) {
      mm->dset_buf = nullptr;
      set_error("chem_step_sets_device: cannot allocate the set offsets");
      return CHEM_ENOMEM;
    }
    mm->dset_cap = need;
  }
  int64_t *off = (int64_t *)mm->dset_buf;
  unsigned long long *total =
      (unsigned long long *)((unsigned char *)mm->dset_buf + need - 256);
  if ((st = launch_set_offsets(sets, n_sets, off, total, n_bad, s)) != CHEM_OK) return st;
  // the cell count stays on the device: a full persistent grid whose waves
  // stop at the count
  return launch_step(m, INT64_MAX / 4, 0, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr,
                     nullptr, nullptr, o, nullptr, s, total, nullptr, sets, off, n_sets);
}

extern "C" chem_status chem_step_sets_graph_create(const chem_mech *m, int32_t n_sets,
                                                   const chem_set *sets,
                                                   const chem_step_opts *opts, void *stream,
                                                   chem_graph **out) {
  StepOpts o;
  chem_status st = check_sets_call("chem_step_sets_graph_create", m, n_sets, sets, opts, &o);
  if (st != CHEM_OK) return st;
  // the graph owns its own copy of the table
  void *buf = nullptr;
  size_t cap = 0;
  const chem_set *dsets = nullptr;
  const int64_t *doff = nullptr;
  int64_t total = 0;
  st = stage_sets("chem_step_sets_graph_create", n_sets, sets, (hipStream_t)stream, &buf, &cap,
                  &dsets, &doff, &total);
  if (st == CHEM_OK && total == 0) {
    set_error("chem_step_sets_graph_create: no cells");
    st = CHEM_EINVAL;
  }
  if (st == CHEM_OK)
    st = capture_graph(
        [&](hipStream_t cs) {
          return launch_step(m, total, 0, 0.0, nullptr, nullptr, nullptr, nullptr, nullptr,
                             nullptr, nullptr, o, nullptr, cs, nullptr, nullptr, dsets, doff,
                             n_sets);
        },
        out);
  if (st != CHEM_OK) {
    if (buf) (void)hipFree(buf);
    return st;
  }
  (*out)->release = free_device;
  (*out)->owner = buf;
  return CHEM_OK;
}

extern "C" chem_status chem_graph_launch(chem_graph *g, void *stream) {
  if (!g || !g->e) {
    set_error("chem_graph_launch: null graph");
    return CHEM_EINVAL;
  }
  CHEM_HIP(hipGraphLaunch(g->e, (hipStream_t)stream));
  return CHEM_OK;
}

extern "C" void chem_graph_destroy(chem_graph *g) {
  if (!g) return;
  if (g->e) (void)hipGraphExecDestroy(g->e);
  if (g->g) (void)hipGraphDestroy(g->g);
  if (g->s) (void)hipStreamDestroy(g->s);
  if (g->release) g->release(g->owner);
  delete g;
}

// ------------------------------------------------------------ tuning cache
namespace chem {

uint64_t fnv1a(const void *p, size_t n, uint64_t h) {
  const unsigned char *c = (const unsigned char *)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

namespace {
std::mutex g_cache_mu;

const char *cache_path() {
  const char *p = getenv("CHEM_AUTOTUNE_CACHE");
  return p && *p ? p : nullptr;
}

// every "key = value" line of the file, in order
std::vector<std::pair<std::string, std::string>> cache_read(const char *path) {
  std::vector<std::pair<std::string, std::string>> out;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t eq = line.find(" = ");
    if (eq == std::string::npos) continue;
    out.emplace_back(line.substr(0, eq), line.substr(eq + 3));
  }
  return out;
}
}  // namespace

bool tune_cache_get(const std::string &key, std::string *value) {
  const char *path = cache_path();
  if (!path) return false;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  bool found = false;
  for (auto &kv : cache_read(path))
    if (kv.first == key) {
      *value = kv.second;
      found = true;
    }
  return found;
}

void tune_cache_put(const std::string &key, const std::string &value) {
  const char *path = cache_path();
  if (!path) return;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto all = cache_read(path);
  bool replaced = false;
  for (auto &kv : all)
    if (kv.first == key) {
      kv.second = value;
      replaced = true;
    }
  if (!replaced) all.emplace_back(key, value);
  std::ofstream out(path, std::ios::trunc);
  for (auto &kv : all) out << kv.first << " = " << kv.second << "\n";
}

std::string tune_device_key() {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::ostringstream k;
  k << prop.gcnArchName << ":" << prop.multiProcessorCount;
  return k.str();
}

}  // namespace chem
