// Host side of the surrogate (ANN) ABI: the model handle (weights, Adam
// state, normalisation statistics, workspaces), inference with fallback to
// the FP64 integrator, one training step, statistics fitting and save/load.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <iomanip>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "ann_internal.h"

using ann::u16;

namespace {

// Growable device workspace made of named sections.
struct Workspace {
  void *base = nullptr;
  size_t bytes = 0;
  int64_t cap = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// splitmix64 (Steele, Lea & Flood 2014) for the seeded initial weights.
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
};

}  // namespace

struct ann_model {
  int device = 0;
  int n_in = 0, n_out = 0, prec = 0;
  // networks: 1, or n_out for the per-species ensemble (member g predicts
  // species g; every per-layer array holds the members one after another)
  int G = 1;
  ann::Layer L[ann::NLAYER];
  float *Wm[ann::NLAYER] = {}, *bm[ann::NLAYER] = {};  // FP32 master parameters
  u16 *Wb[ann::NLAYER] = {};                           // BF16 copies used by the GEMMs
  u16 *Wt[ann::NLAYER] = {};     // K-blocked BF16 copies for the large-batch forward path
  u16 *W2p = nullptr;            // second layer K-blocked in the fused kernel's K order
  bool wt_stale = true;          // Wt, W2p behind Wb (set on every weight change)
  float *mW[ann::NLAYER] = {}, *vW[ann::NLAYER] = {}, *mb[ann::NLAYER] = {},
        *vb[ann::NLAYER] = {};
  float *gW[ann::NLAYER] = {}, *gb[ann::NLAYER] = {};
  void *params = nullptr;  // one allocation behind all of the above
  int64_t step = 0;
  bool has_norm = false;
  ann::Norm nm{};
  void *norm_buf = nullptr;
  std::vector<float> h_mu_in, h_sd_in, h_lo, h_hi, h_mu_out, h_sd_out;
  // inference workspace (per chunk of cells)
  Workspace wi;
  u16 *X = nullptr, *H[3] = {};
  float *U = nullptr;
  float *Um = nullptr;
  int32_t *fb_index = nullptr;  // fallback cell list (own allocation, fb_cap entries)
  int64_t fb_cap = 0;
  unsigned long long *fb_count = nullptr;
  // training workspace (per batch)
  Workspace wt;
  u16 *tX = nullptr, *tH[3] = {}, *tGb[ann::NLAYER] = {};
  float *tZ[3] = {}, *tU = nullptr, *tUt = nullptr, *tGf[ann::NLAYER] = {};
  double *loss_part = nullptr;
  double *phys_part = nullptr;  // [PHYS_PARTS][3] partial sums of the physics terms
  double *col_part = nullptr;  // [COLSUM_PARTS][max dout] bias-gradient partials
  float *wg_part = nullptr;    // split-K partial weight gradients
  size_t wg_cap = 0;           // floats in wg_part
  // FP8 inference of the hidden-to-hidden layers (L2, L3)
  bool fp8_ready = false, use_fp8 = false;
  float sa[3] = {1, 1, 1}, sw[3] = {1, 1, 1};  // per-tensor scales of layers 1, 2
  void *fp8_buf = nullptr;
  uint8_t *Wq1 = nullptr, *Wq2 = nullptr;  // [n2p][kq1], [L3 outputs][k3p] E4M3
  uint8_t *Wq1t = nullptr, *Wq2t = nullptr;  // the same, K-blocked by 128 bytes
  float *bq1 = nullptr;                    // layer-1 bias padded to N2p
  int n2p = 0, k3p = 0, kq1 = 0;           // FP8 widths: L2 out (x32), L3 in / L2 in (x128)
  uint8_t *H1q = nullptr, *H2q = nullptr;  // inference workspace (E4M3 activations)
  uint8_t *ood = nullptr;                  // per-cell out-of-distribution bits
  int graph_refs = 0;  // live captured steps that use the inference workspace
  // tilings of the eleven training products at batch tt_B, from
  // ann_autotune_train (tt_B = 0: the built-in rules)
  int64_t tt_B = 0;
  int tt_tile[11] = {}, tt_bk[11] = {}, tt_split[4] = {};
  // audit workspace of ann_step: copies of the audited cells of one chunk and
  // a flags row for callers that pass none
  void *aud_buf = nullptr;
  int64_t aud_cells = 0, aud_flag_cap = 0;
  double *aud_T = nullptr, *aud_p = nullptr, *aud_Y = nullptr, *aud_Y0 = nullptr;
  int32_t *aud_stats = nullptr;
  uint8_t *aud_flags = nullptr;
};

using namespace chem;

namespace {

constexpr int64_t CHUNK = 1 << 21;  // cells per inference pass
constexpr int LOSS_PARTS = 256;

int pad32(int x) { return (x + 31) / 32 * 32; }

size_t layer_elems(const ann::Layer &L) { return (size_t)L.doutp * L.dinp; }

// Row width of the network output U (species padded to 32); one network's
// output layer width, the assembled ensemble's otherwise.
int uw(const ann_model *m) { return pad32(m->n_out); }

// E4M3 layout: L2 reads H1q [cells][kq1] and Wq1 [n2p][kq1]; L3 reads H2q
// [cells][k3p] and Wq2 [L3 outputs][k3p]; K widths padded to 128 with zeros.
int fp8_n2p(const ann_model *m) { return (m->L[1].dout + 31) / 32 * 32; }
int fp8_kq1(const ann_model *m) { return (m->L[1].dinp + 127) / 128 * 128; }
int fp8_k3p(const ann_model *m) { return (fp8_n2p(m) + 127) / 128 * 128; }

// The inference workspace of cap cells: input rows, activations, network
// output, out-of-distribution bytes, the fallback count and (no-allocation
// step only) the fallback list.
struct InferWs {
  int64_t cap = 0;  // rows between K-blocks of the K-blocked activations
  u16 *X = nullptr, *H[3] = {};
  float *U = nullptr;
  float *Um = nullptr;  // one ensemble member's output [cap][32] before its column is taken
  uint8_t *ood = nullptr;
  unsigned long long *fb_count = nullptr;
  uint8_t *H1q = nullptr, *H2q = nullptr;  // E4M3 activations, rows padded with zeros
  size_t q_bytes = 0;                      // bytes from H1q to the end of H2q
  int32_t *fb_index = nullptr;
};

// Section offsets of a workspace of cap cells (fb_list: with a fallback list
// of cap entries).  Returns the bytes needed; with base non-null, fills w.
size_t infer_layout(const ann_model *m, int64_t cap, bool fb_list, unsigned char *base,
                    InferWs *w) {
  size_t off = 0;
  auto sect = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t oX = sect((size_t)cap * m->L[0].dinp * 2);
  size_t oH[3];
  for (int l = 0; l < 3; ++l) oH[l] = sect((size_t)cap * m->L[l].doutp * 2);
  const size_t oU = sect((size_t)cap * uw(m) * 4);
  const size_t oUm = m->G > 1 ? sect((size_t)cap * m->L[3].doutp * 4) : 0;
  const size_t oO = sect((size_t)cap);
  const size_t oC = sect(64);
  // E4M3 activations (the FP8 variant exists for single networks only)
  const size_t q1 = m->G > 1 ? 0 : (size_t)cap * fp8_kq1(m);
  const size_t q2 = m->G > 1 ? 0 : (size_t)cap * fp8_k3p(m);
  const size_t oQ1 = sect(q1);
  const size_t oQ2 = sect(q2);
  const size_t oF = fb_list ? sect((size_t)cap * 4) : 0;
  if (base && w) {
    w->cap = cap;
    w->X = (u16 *)(base + oX);
    for (int l = 0; l < 3; ++l) w->H[l] = (u16 *)(base + oH[l]);
    w->U = (float *)(base + oU);
    w->Um = m->G > 1 ? (float *)(base + oUm) : nullptr;
    w->ood = base + oO;
    w->fb_count = (unsigned long long *)(base + oC);
    w->H1q = base + oQ1;
    w->H2q = base + oQ2;
    w->q_bytes = oQ2 - oQ1 + q2;
    w->fb_index = fb_list ? (int32_t *)(base + oF) : nullptr;
  }
  return off;
}

// The model's own (growable) inference workspace as a view.
InferWs model_ws(const ann_model *m) {
  InferWs w;
  w.cap = m->wi.cap;
  w.X = m->X;
  for (int l = 0; l < 3; ++l) w.H[l] = m->H[l];
  w.U = m->U;
  w.Um = m->Um;
  w.ood = m->ood;
  w.fb_count = m->fb_count;
  w.H1q = m->H1q;
  w.H2q = m->H2q;
  w.fb_index = m->fb_index;
  return w;
}

chem_status grow_infer(ann_model *m, int64_t n) {
  const int64_t need = n < CHUNK ? n : CHUNK;
  if (m->wi.cap >= need) return CHEM_OK;
  if (m->graph_refs > 0) {
    set_error("ann: the inference workspace is held by a captured step (destroy its graphs "
              "before a call with more cells)");
    return CHEM_EINVAL;
  }
  const int64_t cap = need;
  const size_t off = infer_layout(m, cap, false, nullptr, nullptr);
  if (m->wi.base) (void)hipFree(m->wi.base);
  m->wi.base = nullptr;
  m->wi.cap = 0;
  if (hipMalloc(&m->wi.base, off) != hipSuccess) {
    set_error("ann: cannot allocate %zu bytes of inference workspace", off);
    return CHEM_ENOMEM;
  }
  InferWs w;
  infer_layout(m, cap, false, (unsigned char *)m->wi.base, &w);
  m->X = w.X;
  for (int l = 0; l < 3; ++l) m->H[l] = w.H[l];
  m->U = w.U;
  m->Um = w.Um;
  m->ood = w.ood;
  m->fb_count = w.fb_count;
  m->H1q = w.H1q;
  m->H2q = w.H2q;
  // the E4M3 activation rows are padded to multiples of 128 bytes; the
  // padding is never written and must read as zero
  if (w.q_bytes && hipMemset(w.H1q, 0, w.q_bytes) != hipSuccess) {
    set_error("ann: cannot clear the E4M3 activation workspace");
    return CHEM_EHIP;
  }
  m->wi.bytes = off;
  m->wi.cap = cap;
  return CHEM_OK;
}

// Split-K factor of a weight-gradient GEMM (M x N output, K = batch rows): a
// power of two that brings the launch to about 1024 blocks of 128 x 128, while
// every split keeps a multiple of 32 rows.
int wgrad_splits(int M, int N, int64_t K, int groups = 1) {
  const long tiles = (long)((M + 127) / 128) * ((N + 127) / 128) * groups;
  int S = 1;
  while (tiles * S < 1024 && S < 16 && K % (64L * S) == 0) S *= 2;
  return S;
}

chem_status grow_train(ann_model *m, int64_t B) {
  if (m->wt.cap >= B) return CHEM_OK;
  size_t off = 0;
  auto sect = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  // the input rows and targets are shared by the members of an ensemble;
  // activations, outputs and gradients are per member
  const size_t G = (size_t)m->G;
  const size_t oX = sect((size_t)B * m->L[0].dinp * 2);
  size_t oH[3], oZ[3], oGb[4], oGf[4];
  for (int l = 0; l < 3; ++l) {
    oH[l] = sect(G * B * m->L[l].doutp * 2);
    oZ[l] = sect(G * B * m->L[l].doutp * 4);
  }
  const size_t oU = sect(G * B * m->L[3].doutp * 4);
  const size_t oUt = sect((size_t)B * uw(m) * 4);
  for (int l = 0; l < 4; ++l) {
    oGb[l] = sect(G * B * m->L[l].doutp * 2);
    oGf[l] = sect(G * B * m->L[l].doutp * 4);
  }
  const size_t oL = sect(LOSS_PARTS * 8);
  const size_t oP = sect(ann::PHYS_PARTS * 3 * 8);
  size_t col_n = 0, wg_n = 0;
  for (int l = 0; l < 4; ++l) {
    const ann::Layer &L = m->L[l];
    col_n = std::max(col_n, G * ann::COLSUM_PARTS * L.doutp);
    // the largest split any batch size can select (K = 2^30 divides by all)
    const int S = wgrad_splits(L.doutp, L.dinp, 1L << 30, m->G);
    if (S > 1) wg_n = std::max(wg_n, (size_t)S * G * L.doutp * L.dinp);
  }
  const size_t oC = sect(col_n * 8);
  const size_t oW = sect(wg_n * 4);
  if (m->wt.base) (void)hipFree(m->wt.base);
  m->wt.base = nullptr;
  m->wt.cap = 0;
  if (hipMalloc(&m->wt.base, off) != hipSuccess) {
    set_error("ann: cannot allocate %zu bytes of training workspace", off);
    return CHEM_ENOMEM;
  }
  unsigned char *b = (unsigned char *)m->wt.base;
  m->phys_part = (double *)(b + oP);
  m->tX = (u16 *)(b + oX);
  for (int l = 0; l < 3; ++l) {
    m->tH[l] = (u16 *)(b + oH[l]);
    m->tZ[l] = (float *)(b + oZ[l]);
  }
  m->tU = (float *)(b + oU);
  m->tUt = (float *)(b + oUt);
  for (int l = 0; l < 4; ++l) {
    m->tGb[l] = (u16 *)(b + oGb[l]);
    m->tGf[l] = (float *)(b + oGf[l]);
  }
  m->loss_part = (double *)(b + oL);
  m->col_part = (double *)(b + oC);
  m->wg_part = (float *)(b + oW);
  m->wg_cap = wg_n;
  m->wt.cap = B;
  m->wt.bytes = off;
  return CHEM_OK;
}

// Uploads logical [dout][din] FP32 weights into the padded device layout.
// Layer index idx = 4 g + l: layer l of member g (g = 0 for one network).
chem_status upload_layer(ann_model *m, int idx, const float *W, const float *b) {
  const int l = idx & 3, g = idx >> 2;
  const ann::Layer &L = m->L[l];
  const size_t ow = (size_t)g * layer_elems(L), ob = (size_t)g * L.doutp;
  std::vector<float> Wp((size_t)L.doutp * L.dinp, 0.0f), bp(L.doutp, 0.0f);
  for (int o = 0; o < L.dout; ++o) {
    for (int i = 0; i < L.din; ++i) Wp[(size_t)o * L.dinp + i] = W[(size_t)o * L.din + i];
    bp[o] = b[o];
  }
  CHEM_HIP(hipMemcpy(m->Wm[l] + ow, Wp.data(), Wp.size() * 4, hipMemcpyHostToDevice));
  CHEM_HIP(hipMemcpy(m->bm[l] + ob, bp.data(), bp.size() * 4, hipMemcpyHostToDevice));
  m->wt_stale = true;
  chem_status st = ann::to_bf16((int64_t)Wp.size(), m->Wm[l] + ow, m->Wb[l] + ow, nullptr);
  if (st != CHEM_OK) return st;
  CHEM_HIP(hipDeviceSynchronize());
  return CHEM_OK;
}

// dW, db: the per-layer arrays of layer idx & 3 (all members); idx = 4 g + l.
chem_status download_pair(const ann_model *m, int idx, const float *dW, const float *db, float *W,
                          float *b) {
  const int l = idx & 3, g = idx >> 2;
  const ann::Layer &L = m->L[l];
  dW += (size_t)g * layer_elems(L);
  db += (size_t)g * L.doutp;
  std::vector<float> Wp((size_t)L.doutp * L.dinp), bp(L.doutp);
  CHEM_HIP(hipDeviceSynchronize());
  CHEM_HIP(hipMemcpy(Wp.data(), dW, Wp.size() * 4, hipMemcpyDeviceToHost));
  CHEM_HIP(hipMemcpy(bp.data(), db, bp.size() * 4, hipMemcpyDeviceToHost));
  if (W)
    for (int o = 0; o < L.dout; ++o)
      for (int i = 0; i < L.din; ++i) W[(size_t)o * L.din + i] = Wp[(size_t)o * L.dinp + i];
  if (b)
    for (int o = 0; o < L.dout; ++o) b[o] = bp[o];
  return CHEM_OK;
}

chem_status check_model(const char *fn, const ann_model *m) {
  if (!m) {
    set_error("%s: null model", fn);
    return CHEM_EINVAL;
  }
  return CHEM_OK;
}

chem_status upload_norm(ann_model *m) {
  const int ni = m->n_in, no = m->n_out;
  if (!m->norm_buf) {
    CHEM_HIP(hipMalloc(&m->norm_buf, (size_t)(4 * ni + 2 * no) * 4));
    float *f = (float *)m->norm_buf;
    m->nm.mu_in = f;
    m->nm.sd_in = f + ni;
    m->nm.lo = f + 2 * ni;
    m->nm.hi = f + 3 * ni;
    m->nm.mu_out = f + 4 * ni;
    m->nm.sd_out = f + 4 * ni + no;
  }
  std::vector<float> all;
  for (auto *v : {&m->h_mu_in, &m->h_sd_in, &m->h_lo, &m->h_hi, &m->h_mu_out, &m->h_sd_out})
    all.insert(all.end(), v->begin(), v->end());
  CHEM_HIP(hipMemcpy(m->norm_buf, all.data(), all.size() * 4, hipMemcpyHostToDevice));
  m->has_norm = true;
  return CHEM_OK;
}

}  // namespace

extern "C" chem_status ann_create(const ann_arch *arch, uint64_t seed, ann_model **out) {
  if (!arch || !out) {
    set_error("ann_create: null argument");
    return CHEM_EINVAL;
  }
  *out = nullptr;
  if (arch->n_in < 1 || arch->n_out < 1 || arch->n_in > 96 || arch->n_out > 96) {
    set_error("ann_create: n_in/n_out must be in 1..96 (got %d, %d)", arch->n_in, arch->n_out);
    return CHEM_EINVAL;
  }
  for (int i = 0; i < 3; ++i)
    if (arch->hidden[i] < 1 || arch->hidden[i] > 8192) {
      set_error("ann_create: hidden sizes must be in 1..8192");
      return CHEM_EINVAL;
    }
  if (arch->prec != 0) {
    set_error("ann_create: only BF16 hidden layers (prec 0) are available in this library");
    return CHEM_EUNSUPPORTED;
  }
  const int G = arch->members <= 1 ? 1 : arch->members;
  if (G > 1 && G != arch->n_out) {
    set_error("ann_create: an ensemble has one member per output (members = n_out = %d, got "
              "%d)", arch->n_out, arch->members);
    return CHEM_EINVAL;
  }
  ann_model *m = new ann_model();
  m->n_in = arch->n_in;
  m->n_out = arch->n_out;
  m->prec = arch->prec;
  m->G = G;
  const int dims[5] = {arch->n_in, arch->hidden[0], arch->hidden[1], arch->hidden[2],
                       G > 1 ? 1 : arch->n_out};
  for (int l = 0; l < 4; ++l) {
    m->L[l].din = dims[l];
    m->L[l].dout = dims[l + 1];
    m->L[l].dinp = pad32(dims[l]);
    m->L[l].doutp = pad32(dims[l + 1]);
  }
  size_t off = 0;
  size_t oW[4], ob[4], oWb[4], oWt[4], omW[4], ovW[4], omb[4], ovb[4], ogW[4], ogb[4];
  auto sect = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t oW2p = sect(G * layer_elems(m->L[1]) * 2);
  for (int l = 0; l < 4; ++l) {
    const size_t e = G * layer_elems(m->L[l]), nb = G * m->L[l].doutp;
    oW[l] = sect(e * 4);
    ob[l] = sect(nb * 4);
    oWb[l] = sect(e * 2);
    oWt[l] = sect(e * 2);
    omW[l] = sect(e * 4);
    ovW[l] = sect(e * 4);
    omb[l] = sect(nb * 4);
    ovb[l] = sect(nb * 4);
    ogW[l] = sect(e * 4);
    ogb[l] = sect(nb * 4);
  }
  hipError_t e = hipGetDevice(&m->device);
  if (e == hipSuccess) e = hipMalloc(&m->params, off);
  if (e != hipSuccess) {
    delete m;
    set_error("ann_create: device allocation of %zu bytes failed", off);
    return CHEM_ENOMEM;
  }
  e = hipMemset(m->params, 0, off);
  if (e != hipSuccess) {
    (void)hipFree(m->params);
    delete m;
    return hip_fail(e, "ann_create: hipMemset");
  }
  unsigned char *b = (unsigned char *)m->params;
  m->W2p = (u16 *)(b + oW2p);
  for (int l = 0; l < 4; ++l) {
    m->Wm[l] = (float *)(b + oW[l]);
    m->bm[l] = (float *)(b + ob[l]);
    m->Wb[l] = (u16 *)(b + oWb[l]);
    m->Wt[l] = (u16 *)(b + oWt[l]);
    m->mW[l] = (float *)(b + omW[l]);
    m->vW[l] = (float *)(b + ovW[l]);
    m->mb[l] = (float *)(b + omb[l]);
    m->vb[l] = (float *)(b + ovb[l]);
    m->gW[l] = (float *)(b + ogW[l]);
    m->gb[l] = (float *)(b + ogb[l]);
  }
  // W, b ~ U(-1/sqrt(fan_in), +1/sqrt(fan_in)), member after member
  SplitMix rng{seed};
  for (int idx = 0; idx < 4 * G; ++idx) {
    const ann::Layer &L = m->L[idx & 3];
    const double bound = 1.0 / sqrt((double)L.din);
    std::vector<float> W((size_t)L.dout * L.din), bb(L.dout);
    for (auto &w : W) w = (float)((2.0 * rng.uniform() - 1.0) * bound);
    for (auto &w : bb) w = (float)((2.0 * rng.uniform() - 1.0) * bound);
    chem_status st = upload_layer(m, idx, W.data(), bb.data());
    if (st != CHEM_OK) {
      ann_destroy(m);
      return st;
    }
  }
  *out = m;
  return CHEM_OK;
}

extern "C" void ann_destroy(ann_model *m) {
  if (!m) return;
  if (m->fp8_buf) (void)hipFree(m->fp8_buf);
  (void)hipFree(m->params);
  if (m->norm_buf) (void)hipFree(m->norm_buf);
  if (m->wi.base) (void)hipFree(m->wi.base);
  if (m->wt.base) (void)hipFree(m->wt.base);
  if (m->fb_index) (void)hipFree(m->fb_index);
  if (m->aud_buf) (void)hipFree(m->aud_buf);
  delete m;
}

extern "C" chem_status ann_set_layer(ann_model *m, int32_t layer, const float *W,
                                     const float *b) {
  chem_status st = check_model("ann_set_layer", m);
  if (st != CHEM_OK) return st;
  if (layer < 0 || layer >= ann::NLAYER * m->G || !W || !b) {
    set_error("ann_set_layer: bad layer index or null array");
    return CHEM_EINVAL;
  }
  return upload_layer(m, layer, W, b);
}

extern "C" chem_status ann_get_layer(const ann_model *m, int32_t layer, float *W, float *b) {
  chem_status st = check_model("ann_get_layer", m);
  if (st != CHEM_OK) return st;
  if (layer < 0 || layer >= ann::NLAYER * m->G) {
    set_error("ann_get_layer: bad layer index");
    return CHEM_EINVAL;
  }
  return download_pair(m, layer, m->Wm[layer & 3], m->bm[layer & 3], W, b);
}

extern "C" chem_status ann_get_grad(const ann_model *m, int32_t layer, float *dW, float *db) {
  chem_status st = check_model("ann_get_grad", m);
  if (st != CHEM_OK) return st;
  if (layer < 0 || layer >= ann::NLAYER * m->G) {
    set_error("ann_get_grad: bad layer index");
    return CHEM_EINVAL;
  }
  return download_pair(m, layer, m->gW[layer & 3], m->gb[layer & 3], dW, db);
}

extern "C" chem_status ann_get_moments(const ann_model *m, int32_t layer, float *mW, float *vW,
                                       float *mb, float *vb) {
  chem_status st = check_model("ann_get_moments", m);
  if (st != CHEM_OK) return st;
  if (layer < 0 || layer >= ann::NLAYER * m->G) {
    set_error("ann_get_moments: bad layer index");
    return CHEM_EINVAL;
  }
  st = download_pair(m, layer, m->mW[layer & 3], m->mb[layer & 3], mW, mb);
  if (st != CHEM_OK) return st;
  return download_pair(m, layer, m->vW[layer & 3], m->vb[layer & 3], vW, vb);
}

extern "C" chem_status ann_set_norm(ann_model *m, const ann_norm *nm) {
  chem_status st = check_model("ann_set_norm", m);
  if (st != CHEM_OK) return st;
  if (!nm || !nm->mu_in || !nm->sd_in || !nm->lo || !nm->hi || !nm->mu_out || !nm->sd_out ||
      !(nm->lambda > 0.0f) || !(nm->dt_model > 0.0)) {
    set_error("ann_set_norm: null array, lambda <= 0 or dt_model <= 0");
    return CHEM_EINVAL;
  }
  for (int j = 0; j < m->n_in; ++j)
    if (!(nm->sd_in[j] > 0.0f)) {
      set_error("ann_set_norm: sd_in[%d] must be positive", j);
      return CHEM_EINVAL;
    }
  for (int j = 0; j < m->n_out; ++j)
    if (!(nm->sd_out[j] > 0.0f)) {
      set_error("ann_set_norm: sd_out[%d] must be positive", j);
      return CHEM_EINVAL;
    }
  m->nm.lambda = nm->lambda;
  m->nm.dt_model = nm->dt_model;
  m->h_mu_in.assign(nm->mu_in, nm->mu_in + m->n_in);
  m->h_sd_in.assign(nm->sd_in, nm->sd_in + m->n_in);
  m->h_lo.assign(nm->lo, nm->lo + m->n_in);
  m->h_hi.assign(nm->hi, nm->hi + m->n_in);
  m->h_mu_out.assign(nm->mu_out, nm->mu_out + m->n_out);
  m->h_sd_out.assign(nm->sd_out, nm->sd_out + m->n_out);
  return upload_norm(m);
}

extern "C" chem_status ann_get_norm(const ann_model *m, float *mu_in, float *sd_in, float *lo,
                                    float *hi, float *mu_out, float *sd_out, float *lambda,
                                    double *dt_model) {
  chem_status st = check_model("ann_get_norm", m);
  if (st != CHEM_OK) return st;
  if (!m->has_norm) {
    set_error("ann_get_norm: no statistics set");
    return CHEM_EMODEL;
  }
  auto cp = [](const std::vector<float> &v, float *o) {
    if (o) memcpy(o, v.data(), v.size() * 4);
  };
  cp(m->h_mu_in, mu_in);
  cp(m->h_sd_in, sd_in);
  cp(m->h_lo, lo);
  cp(m->h_hi, hi);
  cp(m->h_mu_out, mu_out);
  cp(m->h_sd_out, sd_out);
  if (lambda) *lambda = m->nm.lambda;
  if (dt_model) *dt_model = m->nm.dt_model;
  return CHEM_OK;
}

extern "C" chem_status ann_fit_norm(ann_model *m, chem_batch batch, const double *T,
                                    const double *p, const double *Y0, const double *Y1,
                                    float lambda, double dt_model, void *stream) {
  chem_status st = check_model("ann_fit_norm", m);
  if (st != CHEM_OK) return st;
  const int K = m->n_out;
  if (m->n_in != K + 2 || batch.n < 1 || batch.ld < batch.n || !T || !p || !Y0 || !Y1 ||
      !(lambda > 0.0f) || !(dt_model > 0.0)) {
    set_error("ann_fit_norm: needs n_in = n_out + 2, n >= 1, non-null arrays, lambda > 0");
    return CHEM_EINVAL;
  }
  const int F = 2 * K + 2;
  const int nblocks = 256;
  double *part = nullptr;
  CHEM_HIP(hipMalloc(&part, ((size_t)nblocks * F * 4 + F) * sizeof(double)));
  ann::StatArgs a{batch.n, batch.ld, T, p, Y0, Y1, K, lambda, part, nblocks};
  hipStream_t s = (hipStream_t)stream;
  st = ann::stats_partial(a, s);
  // partial sums [nblocks][F][4], then the F shifts they were taken about
  std::vector<double> h((size_t)nblocks * F * 4 + F);
  if (st == CHEM_OK) {
    hipError_t e = hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "ann_fit_norm: read back");
  }
  (void)hipFree(part);
  if (st != CHEM_OK) return st;
  const double *shift = h.data() + (size_t)nblocks * F * 4;
  std::vector<float> mu(F), sd(F), lo(F), hi(F);
  for (int f = 0; f < F; ++f) {
    double s1 = 0, s2 = 0, mn = INFINITY, mx = -INFINITY;
    for (int b = 0; b < nblocks; ++b) {
      const double *o = &h[((size_t)b * F + f) * 4];
      s1 += o[0];
      s2 += o[1];
      mn = fmin(mn, o[2]);
      mx = fmax(mx, o[3]);
    }
    const double dmean = s1 / batch.n;
    const double var = fmax(s2 / batch.n - dmean * dmean, 0.0);
    const double mean = shift[f] + dmean;
    double sdv = sqrt(var);
    if (sdv < 1e-12 * fabs(mean) + 1e-30) sdv = 1.0;
    mu[f] = (float)mean;
    sd[f] = (float)sdv;
    lo[f] = (float)mn;
    hi[f] = (float)mx;
  }
  m->nm.lambda = lambda;
  m->nm.dt_model = dt_model;
  m->h_mu_in.assign(mu.begin(), mu.begin() + K + 2);
  m->h_sd_in.assign(sd.begin(), sd.begin() + K + 2);
  m->h_lo.assign(lo.begin(), lo.begin() + K + 2);
  m->h_hi.assign(hi.begin(), hi.begin() + K + 2);
  m->h_mu_out.assign(mu.begin() + K + 2, mu.end());
  m->h_sd_out.assign(sd.begin() + K + 2, sd.end());
  return upload_norm(m);
}

namespace {

// Network forward for n cells (n <= workspace capacity): features -> X ->
// L1..L3 (bias + GELU, BF16) -> L4 (bias, FP32) -> U [n][ldu] (ldu = n_out,
// or the padded output width, whose extra columns come out zero).  With ood
// non-null the out-of-distribution bit of every cell is written there.
// Large batches of a network whose widths match the direct-to-LDS tilings run
// every hidden layer on those kernels with K-blocked activations and weights
// (rows of one 32-wide K-step contiguous in HBM; 128 bytes for E4M3).
bool tiled_path(const ann_model *m, int64_t n) {
  const ann::Layer &a = m->L[0], &b = m->L[1], &c = m->L[2];
  if (n < (1 << 17) || a.dinp != 32 || a.doutp % 320 != 0) return false;
  if (m->use_fp8) return m->n2p % 160 == 0 && c.doutp % 208 == 0;
  return b.doutp % 400 == 0 && (c.doutp % 416 == 0 || c.doutp % 400 == 0);
}

// The per-species ensemble: the shared input rows once, then each member's
// four layers on the single network's kernels (its weights at the member's
// offset), its one output written to U's column g.  Members run one after
// another: at inference sizes every launch fills the GPU on its own.
chem_status forward_members(ann_model *m, const InferWs &w, int64_t n, float *U, int ldu,
                            hipStream_t s) {
  chem_status st;
  const bool tl = tiled_path(m, n);
  const long cap = (long)w.cap;
  const int G = m->G;
  if (m->wt_stale) {
    for (int g = 0; g < G; ++g) {
      for (int l = 1; l <= 2; ++l) {
        const size_t o = (size_t)g * layer_elems(m->L[l]);
        if ((st = ann::tile_bf16(m->L[l].doutp, m->L[l].dinp, m->Wb[l] + o, m->Wt[l] + o, s)) !=
            CHEM_OK)
          return st;
      }
      const size_t o1 = (size_t)g * layer_elems(m->L[1]);
      if ((st = ann::tile_bf16(m->L[1].doutp, m->L[1].dinp, m->Wb[1] + o1, m->W2p + o1, s,
                               true)) != CHEM_OK)
        return st;
    }
    m->wt_stale = false;
  }
  const int uo = m->L[3].doutp;  // a member's padded output width
  for (int g = 0; g < G; ++g) {
    size_t ow[4], ob[4];
    for (int l = 0; l < 4; ++l) {
      ow[l] = (size_t)g * layer_elems(m->L[l]);
      ob[l] = (size_t)g * m->L[l].doutp;
    }
    const u16 *in = w.X;
    bool in_tiled = false;
    int l0 = 0;
    {
      const ann::Layer &L0 = m->L[0], &L1 = m->L[1];
      ann::Mlp12Args f{};
      f.M = (int)n;
      f.N = L1.doutp;
      f.K = L1.dinp;
      f.X = w.X;
      f.W1 = m->Wb[0] + ow[0];
      f.b1 = m->bm[0] + ob[0];
      f.W2p = m->W2p + ow[1];
      f.ldw2 = (long)L1.doutp * 32;
      f.b2 = m->bm[1] + ob[1];
      f.H = w.H[1];
      f.ldh = tl ? cap * 32 : L1.doutp;
      f.tiled = tl;
      if (L0.dinp == 32 && L0.doutp == L1.dinp && ann::mlp12_ok(f)) {
        if ((st = ann::mlp12(f, s, "mlp_l12")) != CHEM_OK) return st;
        in = w.H[1];
        in_tiled = tl;
        l0 = 2;
      }
    }
    bool done = false;
    for (int l = l0; l < 4 && !done; ++l) {
      const ann::Layer &L = m->L[l];
      ann::GemmArgs a{};
      a.M = (int)n;
      a.K = L.dinp;
      a.A = in;
      a.lda = in_tiled ? cap * 32 : L.dinp;
      const bool wt = tl && (l == 1 || l == 2);
      a.B = (wt ? m->Wt[l] : m->Wb[l]) + ow[l];
      a.ldb = wt ? (long)L.doutp * 32 : L.dinp;
      a.bias = m->bm[l] + ob[l];
      a.tiled = (in_tiled ? ann::TILED_A : 0) | (wt ? ann::TILED_B : 0);
      if (l == 2) {
        a.N = L.doutp;
        a.B2 = m->Wb[3] + ow[3];
        a.bias2 = m->bm[3] + ob[3];
        a.N2 = uo;
        a.Cf = w.Um;
        a.ldcf = uo;
        if (ann::gemm_fuses_next(a)) {
          if ((st = ann::gemm(a, true, true, ann::EPI_GELU_NEXT, s, "mlp_l3_l4")) != CHEM_OK)
            return st;
          done = true;
          break;
        }
        a.B2 = nullptr;
        a.bias2 = nullptr;
        a.N2 = 0;
        a.Cf = nullptr;
        a.ldcf = 0;
      }
      if (l < 3) {
        const bool ct = tl && l < 2;
        a.N = L.doutp;
        a.Cb = w.H[l];
        a.ldcb = ct ? cap * 32 : L.doutp;
        a.tiled |= ct ? ann::TILED_C : 0;
        static const char *lab[3] = {"mlp_l1", "mlp_l2", "mlp_l3"};
        st = ann::gemm(a, true, true, ann::EPI_GELU, s, lab[l]);
        in = w.H[l];
        in_tiled = ct;
      } else {
        a.N = uo;
        a.Cf = w.Um;
        a.ldcf = uo;
        st = ann::gemm(a, true, true, ann::EPI_F32, s, "mlp_l4");
      }
      if (st != CHEM_OK) return st;
    }
    if ((st = ann::take_col(n, w.Um, uo, U + g, ldu, s)) != CHEM_OK) return st;
  }
  return CHEM_OK;
}

// keep_h1: write the first two layers' activations row-major to H[0], H[1]
// (no fused first two layers, no K-blocked layouts), for the FP8 calibration
// that reads their first n rows
chem_status forward_chunk(ann_model *m, const InferWs &w, int64_t n, int64_t ld, const double *T,
                          const double *p, const double *Y, float *U, int ldu, uint8_t *ood,
                          float ood_margin, hipStream_t s, bool keep_h1 = false) {
  ann::FeatArgs fa{n, ld, T, p, Y, nullptr, m->n_out, m->L[0].dinp, m->nm.mu_in, m->nm.sd_in,
                   m->nm.lambda, w.X, ood, m->nm.lo, m->nm.hi, ood_margin};
  chem_status st = ann::features(fa, s);
  if (st != CHEM_OK) return st;
  if (m->G > 1) return forward_members(m, w, n, U, ldu, s);
  const bool tl = !keep_h1 && tiled_path(m, n);
  const long cap = (long)w.cap;  // rows between K-blocks of the activations
  if (!m->use_fp8 && m->wt_stale) {
    for (int l = 1; l <= 2; ++l)
      if ((st = ann::tile_bf16(m->L[l].doutp, m->L[l].dinp, m->Wb[l], m->Wt[l], s)) != CHEM_OK)
        return st;
    if ((st = ann::tile_bf16(m->L[1].doutp, m->L[1].dinp, m->Wb[1], m->W2p, s, true)) !=
        CHEM_OK)
      return st;
    m->wt_stale = false;
  }
  if (m->use_fp8) {
    // L1 (BF16) -> E4M3 activations; L2, L3 on FP8 MFMA; L4 (BF16)
    const ann::Layer &L0 = m->L[0], &L2 = m->L[2], &L3 = m->L[3];
    ann::GemmArgs g{};
    g.M = (int)n;
    g.N = L0.doutp;
    g.K = L0.dinp;
    g.A = w.X;
    g.lda = L0.dinp;
    g.B = m->Wb[0];
    g.ldb = L0.dinp;
    g.bias = m->bm[0];
    g.Cq = w.H1q;
    g.ldcq = tl ? cap * 128 : m->kq1;
    g.tiled = tl ? ann::TILED_C : 0;
    g.qinv = 1.0f / m->sa[1];
    if ((st = ann::gemm(g, true, true, ann::EPI_GELU_Q8, s, "mlp_l1")) != CHEM_OK) return st;
    ann::GemmArgs h{};
    h.M = (int)n;
    h.N = m->n2p;
    h.K = m->kq1;
    h.A8 = w.H1q;
    h.lda = tl ? cap * 128 : m->kq1;
    h.B8 = tl ? m->Wq1t : m->Wq1;
    h.ldb = tl ? (long)m->n2p * 128 : m->kq1;
    h.bias = m->bq1;
    h.scale = m->sa[1] * m->sw[1];
    h.Cq = w.H2q;
    h.ldcq = tl ? cap * 128 : m->k3p;
    h.qinv = 1.0f / m->sa[2];
    h.tiled = tl ? (ann::TILED_A | ann::TILED_B | ann::TILED_C) : 0;
    if ((st = ann::gemm8(h, ann::EPI_GELU_Q8, s, "mlp_l2_fp8")) != CHEM_OK) return st;
    ann::GemmArgs q{};
    q.M = (int)n;
    q.N = L2.doutp;
    q.K = m->k3p;
    q.A8 = w.H2q;
    q.lda = tl ? cap * 128 : m->k3p;
    q.B8 = tl ? m->Wq2t : m->Wq2;
    q.ldb = tl ? (long)L2.doutp * 128 : m->k3p;
    q.bias = m->bm[2];
    q.scale = m->sa[2] * m->sw[2];
    q.Cb = w.H[2];
    q.ldcb = L2.doutp;
    q.tiled = tl ? (ann::TILED_A | ann::TILED_B) : 0;
    // the output layer rides in the epilogue of the last hidden layer when
    // the tiling allows it (its activations then never reach HBM)
    q.B2 = m->Wb[3];
    q.bias2 = m->bm[3];
    q.N2 = m->L[3].doutp;
    q.Cf = U;
    q.ldcf = ldu;
    if (ann::gemm8_fuses_next(q)) return ann::gemm8(q, ann::EPI_GELU_NEXT, s, "mlp_l3_l4_fp8");
    q.B2 = nullptr;
    q.bias2 = nullptr;
    q.N2 = 0;
    q.Cf = nullptr;
    q.ldcf = 0;
    if ((st = ann::gemm8(q, ann::EPI_GELU, s, "mlp_l3_fp8")) != CHEM_OK) return st;
    ann::GemmArgs o{};
    o.M = (int)n;
    o.N = ldu;
    o.K = L3.dinp;
    o.A = w.H[2];
    o.lda = L3.dinp;
    o.B = m->Wb[3];
    o.ldb = L3.dinp;
    o.bias = m->bm[3];
    o.Cf = U;
    o.ldcf = ldu;
    return ann::gemm(o, true, true, ann::EPI_F32, s, "mlp_l4");
  }
  const u16 *in = w.X;
  bool in_tiled = false;  // X (K = 32) is one K-block either way
  int l0 = 0;
  {
    // the first two layers in one kernel (the 1600-wide activations stay on
    // chip) when their shapes allow it
    const ann::Layer &L0 = m->L[0], &L1 = m->L[1];
    ann::Mlp12Args f{};
    f.M = (int)n;
    f.N = L1.doutp;
    f.K = L1.dinp;
    f.X = w.X;
    f.W1 = m->Wb[0];
    f.b1 = m->bm[0];
    f.W2p = m->W2p;
    f.ldw2 = (long)L1.doutp * 32;
    f.b2 = m->bm[1];
    f.H = w.H[1];
    f.ldh = tl ? cap * 32 : L1.doutp;
    f.tiled = tl;
    if (!keep_h1 && L0.dinp == 32 && L0.doutp == L1.dinp && ann::mlp12_ok(f)) {
      if ((st = ann::mlp12(f, s, "mlp_l12")) != CHEM_OK) return st;
      in = w.H[1];
      in_tiled = tl;
      l0 = 2;
    }
  }
  for (int l = l0; l < 4; ++l) {
    const ann::Layer &L = m->L[l];
    ann::GemmArgs g{};
    g.M = (int)n;
    g.K = L.dinp;
    g.A = in;
    g.lda = in_tiled ? cap * 32 : L.dinp;
    const bool wt = tl && (l == 1 || l == 2);
    g.B = wt ? m->Wt[l] : m->Wb[l];
    g.ldb = wt ? (long)L.doutp * 32 : L.dinp;
    g.bias = m->bm[l];
    g.tiled = (in_tiled ? ann::TILED_A : 0) | (wt ? ann::TILED_B : 0);
    if (l == 2) {
      // the output layer rides in the epilogue of the last hidden layer when
      // the tiling allows it (its activations then never reach HBM)
      g.N = L.doutp;
      g.B2 = m->Wb[3];
      g.bias2 = m->bm[3];
      g.N2 = m->L[3].doutp;
      g.Cf = U;
      g.ldcf = ldu;
      if (ann::gemm_fuses_next(g)) return ann::gemm(g, true, true, ann::EPI_GELU_NEXT, s,
                                                    "mlp_l3_l4");
      g.B2 = nullptr;
      g.bias2 = nullptr;
      g.N2 = 0;
      g.Cf = nullptr;
      g.ldcf = 0;
    }
    if (l < 3) {
      // hidden activations K-blocked when the next layer reads them on the
      // tiled path (L3's output feeds the 32-wide output layer row-major)
      const bool ct = tl && l < 2;
      g.N = L.doutp;
      g.Cb = w.H[l];
      g.ldcb = ct ? cap * 32 : L.doutp;
      g.tiled |= ct ? ann::TILED_C : 0;
      static const char *lab[3] = {"mlp_l1", "mlp_l2", "mlp_l3"};
      st = ann::gemm(g, true, true, ann::EPI_GELU, s, lab[l]);
      in = w.H[l];
      in_tiled = ct;
    } else {
      g.N = ldu;
      g.Cf = U;
      g.ldcf = ldu;
      st = ann::gemm(g, true, true, ann::EPI_F32, s, "mlp_l4");
    }
    if (st != CHEM_OK) return st;
  }
  return CHEM_OK;
}

}  // namespace

extern "C" chem_status ann_forward(ann_model *m, chem_batch batch, const double *T,
                                   const double *p, const double *Y, float *U, void *stream) {
  chem_status st = check_model("ann_forward", m);
  if (st != CHEM_OK) return st;
  if (!m->has_norm) {
    set_error("ann_forward: normalisation statistics are not set");
    return CHEM_EMODEL;
  }
  if (batch.n < 0 || batch.ld < batch.n || (batch.n > 0 && (!T || !p || !Y || !U))) {
    set_error("ann_forward: bad batch or null array");
    return CHEM_EINVAL;
  }
  if (m->n_in != m->n_out + 2) {
    set_error("ann_forward: the network must have n_in = n_out + 2");
    return CHEM_EMODEL;
  }
  if (batch.n == 0) return CHEM_OK;
  st = grow_infer(m, batch.n);
  if (st != CHEM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  for (int64_t c0 = 0; c0 < batch.n; c0 += m->wi.cap) {
    const int64_t nc = (batch.n - c0 < m->wi.cap) ? batch.n - c0 : m->wi.cap;
    st = forward_chunk(m, model_ws(m), nc, batch.ld, T + c0, p + c0, Y + c0, U + c0 * m->n_out,
                       m->n_out, nullptr, 0.0f, s);
    if (st != CHEM_OK) return st;
  }
  return CHEM_OK;
}

namespace {
// Workspace and fallback list for an ann_step over n cells (the only
// allocations of the step).
chem_status step_prepare(ann_model *m, int64_t n, bool fallback) {
  chem_status st = grow_infer(m, n);
  if (st != CHEM_OK) return st;
  if (fallback && m->fb_cap < n) {
    if (m->graph_refs > 0) {
      set_error("ann_step: the fallback list is held by a captured step (destroy its graphs "
                "before a call with more cells)");
      return CHEM_EINVAL;
    }
    if (m->fb_index) (void)hipFree(m->fb_index);
    m->fb_index = nullptr;
    m->fb_cap = 0;
    if (hipMalloc((void **)&m->fb_index, (size_t)n * 4) != hipSuccess) {
      set_error("ann_step: cannot allocate the fallback list");
      return CHEM_ENOMEM;
    }
    m->fb_cap = n;
  }
  return CHEM_OK;
}

void release_graph(void *owner) { ((ann_model *)owner)->graph_refs--; }

__global__ void k_zero_counter(unsigned long long *c) {
  if (threadIdx.x == 0) *c = 0ull;
}
__global__ void k_add_counter(const unsigned long long *c, int64_t *total, int first) {
  if (threadIdx.x == 0) *total = (first ? 0 : *total) + (int64_t)*c;
}
}  // namespace

namespace {

// Argument checks shared by the step entry points.
chem_status step_check(const char *fn, ann_model *m, const chem_mech *mech, chem_batch batch,
                       double dt, const double *T, const double *p, const double *Y,
                       const ann_step_opts *opts, ann_step_opts *o) {
  if (opts && (!(opts->audit_fraction >= 0.0f && opts->audit_fraction <= 1.0f) ||
               (opts->audit_fraction > 0.0f && !opts->audit))) {
    set_error("%s: audit_fraction must be in [0, 1], with an audit array when above 0", fn);
    return CHEM_EINVAL;
  }
  chem_status st = check_model(fn, m);
  if (st != CHEM_OK) return st;
  if (!mech) {
    set_error("%s: null mechanism", fn);
    return CHEM_EINVAL;
  }
  if (!m->has_norm) {
    set_error("%s: normalisation statistics are not set", fn);
    return CHEM_EMODEL;
  }
  if (m->n_out != mech->K || m->n_in != mech->K + 2) {
    set_error("%s: network has %d inputs / %d outputs, mechanism has K=%d", fn, m->n_in,
              m->n_out, mech->K);
    return CHEM_EMODEL;
  }
  if (batch.n < 0 || batch.ld < batch.n || batch.n > INT32_MAX || !(dt > 0.0) || !isfinite(dt)) {
    set_error("%s: bad batch or dt", fn);
    return CHEM_EINVAL;
  }
  if (batch.n > 0 && (!T || !p || !Y)) {
    set_error("%s: T, p and Y must be non-null", fn);
    return CHEM_EINVAL;
  }
  *o = ann_step_opts{1e-6f, 0.05f, 1, 0.0f, nullptr};
  if (opts) *o = *opts;
  if (!(o->residual_tol >= 0.0f) || !(o->ood_margin >= 0.0f)) {
    set_error("%s: residual_tol and ood_margin must be >= 0", fn);
    return CHEM_EINVAL;
  }
  return CHEM_OK;
}

// Stride of the audited cells: every s-th cell, s the integer nearest 1 / f.
int64_t audit_stride(float f) {
  const double s = floor(1.0 / (double)f + 0.5);
  return s < 1.0 ? 1 : (s > 1e15 ? (int64_t)1e15 : (int64_t)s);
}

// The audit workspace for chunks of up to cap cells (allocates when it grows).
chem_status audit_prepare(ann_model *m, int64_t cap, float f) {
  const int64_t na = (cap + audit_stride(f) - 1) / audit_stride(f);
  if (m->aud_cells >= na && m->aud_flag_cap >= cap) return CHEM_OK;
  if (m->graph_refs > 0) {
    set_error("ann_step: the audit workspace is held by a captured step");
    return CHEM_EINVAL;
  }
  const int K = m->n_out;
  size_t off = 0;
  auto sect = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t oT = sect((size_t)na * 8), oP = sect((size_t)na * 8);
  const size_t oY = sect((size_t)na * K * 8), oY0 = sect((size_t)na * K * 8);
  const size_t oS = sect((size_t)na * 3 * 4), oF = sect((size_t)cap);
  if (m->aud_buf) (void)hipFree(m->aud_buf);
  m->aud_buf = nullptr;
  m->aud_cells = m->aud_flag_cap = 0;
  if (hipMalloc(&m->aud_buf, off) != hipSuccess) {
    m->aud_buf = nullptr;
    set_error("ann_step: cannot allocate the audit workspace");
    return CHEM_ENOMEM;
  }
  unsigned char *b = (unsigned char *)m->aud_buf;
  m->aud_T = (double *)(b + oT);
  m->aud_p = (double *)(b + oP);
  m->aud_Y = (double *)(b + oY);
  m->aud_Y0 = (double *)(b + oY0);
  m->aud_stats = (int32_t *)(b + oS);
  m->aud_flags = b + oF;
  m->aud_cells = na;
  m->aud_flag_cap = cap;
  return CHEM_OK;
}

// The step over batch.n cells in chunks of w.cap, with the fallback list
// fb_index (n entries, or null without fallback) and count w.fb_count.
chem_status step_impl(ann_model *m, const chem_mech *mech, chem_batch batch, double dt, double *T,
                      const double *p, double *Y, double *RR, uint8_t *flags,
                      int64_t *n_fallback, const ann_step_opts &o, const StepOpts &fo,
                      const InferWs &w, int32_t *fb_index, hipStream_t s) {
  chem_status st;
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, w.fb_count);
  // a step other than the one the network was trained for: every cell falls back
  const bool dt_mismatch = fabs(dt - m->nm.dt_model) > 1e-6 * m->nm.dt_model;
  const bool audit = o.audit_fraction > 0.0f;
  const int64_t astride = audit ? audit_stride(o.audit_fraction) : 1;
  if (audit && (st = ann::audit_init(o.audit, m->n_out, s)) != CHEM_OK) return st;
  for (int64_t c0 = 0; c0 < batch.n; c0 += w.cap) {
    const int64_t nc = (batch.n - c0 < w.cap) ? batch.n - c0 : w.cap;
    ann::AuditArgs aa{};
    if (audit) {
      // the audited cells (global indices 0, s, 2s, ...) of this chunk: their
      // inputs, before the network overwrites them
      const int64_t first = (astride - c0 % astride) % astride;
      const int64_t na = first < nc ? (nc - first + astride - 1) / astride : 0;
      uint8_t *fl = (flags ? flags + c0 : m->aud_flags) + first;
      aa = ann::AuditArgs{na, astride, batch.ld, m->n_out, T + c0 + first, p + c0 + first,
                          Y + c0 + first, fl, m->aud_T, m->aud_p, m->aud_Y, m->aud_Y0,
                          m->aud_stats, o.audit};
      if ((st = ann::audit_gather(aa, s)) != CHEM_OK) return st;
    }
    st = forward_chunk(m, w, nc, batch.ld, T + c0, p + c0, Y + c0, w.U, uw(m), w.ood,
                       o.ood_margin, s);
    if (st != CHEM_OK) return st;
    ann::PostArgs pa{};
    pa.n = nc;
    pa.ld = batch.ld;
    pa.dt = dt;
    pa.T = T + c0;
    pa.p = p + c0;
    pa.Y = Y + c0;
    pa.RR = RR ? RR + c0 : nullptr;
    pa.flags = flags ? flags + c0 : (audit ? m->aud_flags : nullptr);
    pa.U = w.U;
    pa.doutp = uw(m);
    pa.nm = m->nm;
    pa.n_in = m->n_in;
    pa.residual_tol = o.residual_tol;
    pa.ood_margin = o.ood_margin;
    pa.ood = w.ood;
    pa.force_flag = dt_mismatch ? 1 : 0;
    pa.fb_index = o.fallback ? fb_index : nullptr;
    pa.fb_count = w.fb_count;
    pa.index_base = c0;
    st = ann::post(mech->d, pa, s);
    if (st != CHEM_OK) return st;
    if (audit) {
      // the reference: the plain step on the copies, then the comparison
      if (aa.na > 0) {
        st = launch_step(mech, aa.na, aa.na, dt, nullptr, m->aud_T, m->aud_p, m->aud_Y, nullptr,
                         nullptr, m->aud_stats, fo, nullptr, s);
        if (st != CHEM_OK) return st;
      }
      if ((st = ann::audit_compare(aa, s)) != CHEM_OK) return st;
    }
  }
  if (o.fallback) {
    st = launch_step(mech, batch.n, batch.ld, dt, nullptr, T, p, Y, RR, nullptr, nullptr, fo,
                     fb_index, s, w.fb_count, flags);
    if (st != CHEM_OK) return st;
  }
  if (n_fallback) hipLaunchKernelGGL(k_add_counter, dim3(1), dim3(64), 0, s, w.fb_count,
                                     n_fallback, 1);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

// Workspace of the no-allocation step: one array per GPU, resident for the
// life of the process.  Host code reaches it only through the address that
// hipGetSymbolAddress returns on each device (the symbol's name is a host
// stand-in there, not a device address).
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
constexpr int SCRATCH_MAXDEV = 64;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
void *g_scratch[SCRATCH_MAXDEV] = {};
std::mutex g_scratch_mu;

chem_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= SCRATCH_MAXDEV) {
    set_error("ann_step_noalloc: device %d beyond the %d supported", dev, SCRATCH_MAXDEV);
    return CHEM_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "ann_step_noalloc: hipGetSymbolAddress");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return CHEM_OK;
}

__global__ void k_fill_zero(unsigned char *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace

extern "C" chem_status ann_step(ann_model *m, const chem_mech *mech, chem_batch batch, double dt,
                                double *T, const double *p, double *Y, double *RR,
                                uint8_t *flags, int64_t *n_fallback, const ann_step_opts *opts,
                                const chem_step_opts *fb_opts, void *stream) {
  ann_step_opts o;
  chem_status st = step_check("ann_step", m, mech, batch, dt, T, p, Y, opts, &o);
  if (st != CHEM_OK || batch.n == 0) return st;
  const StepOpts fo = resolve_opts(fb_opts);
  st = step_prepare(m, batch.n, o.fallback != 0);
  if (st != CHEM_OK) return st;
  if (o.audit_fraction > 0.0f && (st = audit_prepare(m, m->wi.cap, o.audit_fraction)) != CHEM_OK)
    return st;
  return step_impl(m, mech, batch, dt, T, p, Y, RR, flags, n_fallback, o, fo, model_ws(m),
                   m->fb_index, (hipStream_t)stream);
}

extern "C" chem_status ann_step_noalloc(ann_model *m, const chem_mech *mech, chem_batch batch,
                                        double dt, double *T, const double *p, double *Y,
                                        double *RR, uint8_t *flags, int64_t *n_fallback,
                                        const ann_step_opts *opts,
                                        const chem_step_opts *fb_opts, void *stream) {
  ann_step_opts o;
  chem_status st = step_check("ann_step_noalloc", m, mech, batch, dt, T, p, Y, opts, &o);
  if (st != CHEM_OK || batch.n == 0) return st;
  if (o.audit_fraction > 0.0f) {
    set_error("ann_step_noalloc: the audit needs its own workspace (audit_fraction must be 0)");
    return CHEM_EINVAL;
  }
  int dev = -1;
  CHEM_HIP(hipGetDevice(&dev));
  if (dev != m->device || dev != mech->device) {
    set_error("ann_step_noalloc: the model (device %d) and mechanism (device %d) must be on "
              "the current device (%d)", m->device, mech->device, dev);
    return CHEM_EINVAL;
  }
  // the largest chunk whose workspace and fallback list fit in the scratch
  // array: one chunk, so every cell of the call must fit
  int64_t cap = 0, hi = (int64_t)(SCRATCH_BYTES / 8);  // layout grows with cap
  while (hi - cap > 1) {
    const int64_t mid = cap + (hi - cap) / 2;
    if (infer_layout(m, mid, true, nullptr, nullptr) <= SCRATCH_BYTES) cap = mid;
    else hi = mid;
  }
  if (batch.n > cap) {
    set_error("ann_step_noalloc: %lld cells exceed the %lld this network fits in the %zu-byte "
              "scratch array", (long long)batch.n, (long long)cap, SCRATCH_BYTES);
    return CHEM_EINVAL;
  }
  void *base = nullptr;
  if ((st = scratch_address(dev, &base)) != CHEM_OK) return st;
  InferWs w;
  infer_layout(m, batch.n, true, (unsigned char *)base, &w);
  hipStream_t s = (hipStream_t)stream;
  if (m->use_fp8) {
    // the E4M3 rows' padding must read as zero; earlier calls may have left
    // other data there
    hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(256), 0, s, w.H1q, w.q_bytes);
    CHEM_HIP(hipGetLastError());
  }
  const StepOpts fo = resolve_opts(fb_opts);
  return step_impl(m, mech, batch, dt, T, p, Y, RR, flags, n_fallback, o, fo, w, w.fb_index, s);
}

namespace {

// The eleven GEMMs of a training step at batch B: p = 0..3 the forward of
// layer p, 4..7 the weight gradient of layer p - 4 (split S ways along the
// batch, partials [S][members][weights]), 8..10 the data gradient into layer
// p - 8 (through GELU').  An ensemble's members are the groups of each product.
struct TrainProduct {
  ann::GemmArgs g;
  bool AK, BK;
  int epi;
  const char *label;
};

TrainProduct train_product(const ann_model *m, int64_t B, int p, int S) {
  TrainProduct t{};
  ann::GemmArgs &g = t.g;
  const int G = m->G;
  g.groups = G;
  if (p < 4) {
    const int l = p;
    const ann::Layer &L = m->L[l];
    g.M = (int)B;
    g.N = L.doutp;
    g.K = L.dinp;
    g.A = l == 0 ? m->tX : m->tH[l - 1];
    g.lda = L.dinp;
    g.B = m->Wb[l];
    g.ldb = L.dinp;
    g.bias = m->bm[l];
    g.gA = l == 0 ? 0 : (long)B * L.dinp;
    g.gB = (long)layer_elems(L);
    g.gbias = L.doutp;
    g.gcb = g.gcf = g.gz = (long)B * L.doutp;
    if (l < 3) {
      g.Cb = m->tH[l];
      g.ldcb = L.doutp;
      g.Z = m->tZ[l];
      g.ldz = L.doutp;
      t.epi = ann::EPI_GELU;
    } else {
      g.Cf = m->tU;
      g.ldcf = L.doutp;
      t.epi = ann::EPI_F32;
    }
    t.AK = t.BK = true;
    t.label = "train_fwd";
  } else if (p < 8) {
    const int l = p - 4;
    const ann::Layer &L = m->L[l];
    const long wn = (long)L.doutp * L.dinp;
    g.M = L.doutp;
    g.N = L.dinp;
    g.K = (int)B;
    g.A = m->tGb[l];
    g.lda = L.doutp;
    g.B = l > 0 ? m->tH[l - 1] : m->tX;
    g.ldb = L.dinp;
    g.ldcf = L.dinp;
    g.Cf = S > 1 ? m->wg_part : m->gW[l];
    g.ksplit = S;
    g.split_stride = (long)G * wn;
    g.gA = (long)B * L.doutp;
    g.gB = l > 0 ? (long)B * L.dinp : 0;
    g.gcf = wn;
    t.AK = t.BK = false;
    t.epi = ann::EPI_F32;
    t.label = "train_wgrad";
  } else {
    const int l = p - 7;  // the layer whose input gradient this is
    const ann::Layer &L = m->L[l], &P = m->L[l - 1];
    g.M = (int)B;
    g.N = L.dinp;
    g.K = L.doutp;
    g.A = m->tGb[l];
    g.lda = L.doutp;
    g.B = m->Wb[l];
    g.ldb = L.dinp;
    g.Z = m->tZ[l - 1];
    g.ldz = P.doutp;
    g.Cb = m->tGb[l - 1];
    g.ldcb = P.doutp;
    g.Cf = m->tGf[l - 1];
    g.ldcf = P.doutp;
    g.gA = (long)B * L.doutp;
    g.gB = (long)layer_elems(L);
    g.gz = g.gcb = g.gcf = (long)B * P.doutp;
    t.AK = true;
    t.BK = false;
    t.epi = ann::EPI_GELUGRAD;
    t.label = "train_dgrad";
  }
  return t;
}

// Split factor of layer l's weight gradient: the tuned one at the tuned
// batch, else the built-in rule.
int train_split(const ann_model *m, int64_t B, int l) {
  if (m->tt_B == B && m->tt_split[l] > 0) return m->tt_split[l];
  return wgrad_splits(m->L[l].doutp, m->L[l].dinp, B, m->G);
}

chem_status run_product(const ann_model *m, int64_t B, int p, int S, hipStream_t s) {
  TrainProduct t = train_product(m, B, p, S);
  if (m->tt_B == B) {
    t.g.tile = m->tt_tile[p];
    t.g.bk = m->tt_bk[p];
  }
  return ann::gemm(t.g, t.AK, t.BK, t.epi, s, t.label);
}

}  // namespace

extern "C" chem_status ann_train_step(ann_model *m, const chem_mech *mech, chem_batch batch,
                                      const double *T, const double *p, const double *Y0,
                                      const double *Y1, const double *T1, const int64_t *index,
                                      const ann_train_opts *opts, float *loss, float *terms,
                                      void *stream) {
  chem_status st = check_model("ann_train_step", m);
  if (st != CHEM_OK) return st;
  if (!m->has_norm) {
    set_error("ann_train_step: normalisation statistics are not set");
    return CHEM_EMODEL;
  }
  const bool phys = opts && (opts->w_mass != 0.0f || opts->w_energy != 0.0f ||
                             opts->w_hrr != 0.0f || terms);
  if (opts && (!(opts->w_mass >= 0.0f) || !(opts->w_energy >= 0.0f) || !(opts->w_hrr >= 0.0f))) {
    set_error("ann_train_step: physics weights must be >= 0");
    return CHEM_EINVAL;
  }
  if (phys && m->G > 1) {
    set_error("ann_train_step: the physics terms act on the whole predicted change; the members "
              "of a per-species ensemble each see one species");
    return CHEM_EINVAL;
  }
  if (phys && (!mech || mech->K != m->n_out || !T1)) {
    set_error("ann_train_step: the physics terms need the mechanism of the network's %d species "
              "and the reference final temperatures T1", m->n_out);
    return CHEM_EINVAL;
  }
  const int64_t B = batch.n;
  if (B < 32 || B % 32 != 0 || B > (1 << 24) || (!index && batch.ld < B) || !T || !p || !Y0 ||
      !Y1 || !loss || !opts) {
    set_error("ann_train_step: batch must be a positive multiple of 32 (<= 2^24), arrays, "
              "options and loss non-null");
    return CHEM_EINVAL;
  }
  if (m->n_in != m->n_out + 2) {
    set_error("ann_train_step: the network must have n_in = n_out + 2");
    return CHEM_EMODEL;
  }
  st = grow_train(m, B);
  if (st != CHEM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int K = m->n_out;
  if (opts->lr > 0.0f) {  // the E4M3 weights no longer match: back to BF16 inference
    m->fp8_ready = false;
    m->use_fp8 = false;
  }
  ann::FeatArgs fa{B, batch.ld, T, p, Y0, index, K, m->L[0].dinp, m->nm.mu_in, m->nm.sd_in,
                   m->nm.lambda, m->tX, nullptr, nullptr, nullptr, 0.0f};
  if ((st = ann::features(fa, s)) != CHEM_OK) return st;
  ann::TargetArgs ta{B, batch.ld, Y0, Y1, index, K, uw(m), m->nm.mu_out, m->nm.sd_out,
                     m->nm.lambda, m->tUt};
  if ((st = ann::targets(ta, s)) != CHEM_OK) return st;
  // forward, keeping pre-activations (FP32) and activations (BF16); an
  // ensemble's members are the groups of each product (the first layer reads
  // the shared input rows)
  const int G = m->G;
  for (int l = 0; l < 4; ++l)
    if ((st = run_product(m, B, l, 1, s)) != CHEM_OK) return st;
  if (G > 1)
    st = ann::l1_grad_members(B, G, m->L[3].doutp, (long)B * m->L[3].doutp, m->tU, m->tUt, uw(m),
                              m->tGb[3], m->tGf[3], m->loss_part, LOSS_PARTS, loss, s);
  else
    st = ann::l1_grad(B, K, m->L[3].doutp, m->tU, m->tUt, m->tGb[3], m->tGf[3], m->loss_part,
                      LOSS_PARTS, loss, s);
  if (st != CHEM_OK) return st;
  if (phys) {
    ann::PhysArgs pa{};
    pa.n = B;
    pa.ld = batch.ld;
    pa.K = K;
    pa.doutp = m->L[3].doutp;
    pa.U = m->tU;
    pa.Ut = m->tUt;
    pa.Gf = m->tGf[3];
    pa.Gb = m->tGb[3];
    pa.mu = m->nm.mu_out;
    pa.sd = m->nm.sd_out;
    pa.T1 = T1;
    pa.index = index;
    pa.w[0] = opts->w_mass;
    pa.w[1] = opts->w_energy;
    pa.w[2] = opts->w_hrr;
    if ((st = ann::phys_grad(pa, mech->d, m->phys_part, loss, terms, s)) != CHEM_OK) return st;
  }
  // backward: wgrad, bias grad, dgrad (through GELU') per layer
  for (int l = 3; l >= 0; --l) {
    const ann::Layer &L = m->L[l];
    const int S = train_split(m, B, l);
    const long wn = (long)L.doutp * L.dinp;
    if ((st = run_product(m, B, 4 + l, S, s)) != CHEM_OK) return st;
    if (S > 1 && (st = ann::sum_splits((long)G * wn, S, m->wg_part, (long)G * wn, m->gW[l], s)) !=
                     CHEM_OK)
      return st;
    if ((st = ann::colsum(B, L.doutp, m->tGf[l], L.doutp, m->gb[l], m->col_part, s, G,
                          (long)B * L.doutp, L.doutp)) != CHEM_OK)
      return st;
    if (l > 0 && (st = run_product(m, B, 7 + l, 1, s)) != CHEM_OK) return st;
  }
  if (opts->lr > 0.0f) {
    m->step += 1;
    m->wt_stale = true;
    const double bc1 = 1.0 - pow((double)opts->beta1, (double)m->step);
    const double bc2 = 1.0 - pow((double)opts->beta2, (double)m->step);
    // the four weight tensors and the four biases in one launch
    ann::AdamTable at{};
    at.count = 8;
    int64_t o = 0;
    for (int l = 0; l < 4; ++l) {
      const ann::Layer &L = m->L[l];
      at.start[2 * l] = o;
      at.W[2 * l] = m->Wm[l];
      at.g[2 * l] = m->gW[l];
      at.m[2 * l] = m->mW[l];
      at.v[2 * l] = m->vW[l];
      at.Wb[2 * l] = m->Wb[l];
      o += (int64_t)G * layer_elems(L);
      at.start[2 * l + 1] = o;
      at.W[2 * l + 1] = m->bm[l];
      at.g[2 * l + 1] = m->gb[l];
      at.m[2 * l + 1] = m->mb[l];
      at.v[2 * l + 1] = m->vb[l];
      at.Wb[2 * l + 1] = nullptr;
      o += (int64_t)G * L.doutp;
    }
    at.start[8] = o;
    st = ann::adam_multi(at, opts->lr, opts->beta1, opts->beta2, opts->eps, (float)bc1,
                         (float)bc2, s);
    if (st != CHEM_OK) return st;
  }
  return CHEM_OK;
}

extern "C" int64_t ann_num_steps(const ann_model *m) { return m ? m->step : -1; }

extern "C" chem_status ann_autotune_train(ann_model *m, int64_t B, double *ms_default,
                                          double *ms_tuned, void *stream) {
  chem_status st = check_model("ann_autotune_train", m);
  if (st != CHEM_OK) return st;
  if (B < 32 || B % 32 != 0 || B > (1 << 24)) {
    set_error("ann_autotune_train: the batch must be a positive multiple of 32 (<= 2^24)");
    return CHEM_EINVAL;
  }
  if ((st = grow_train(m, B)) != CHEM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  char kb[256];
  snprintf(kb, sizeof(kb), "ann_train %s in=%d hidden=%d,%d,%d out=%d members=%d B=%lld",
           tune_device_key().c_str(), m->n_in, m->L[0].dout, m->L[1].dout, m->L[2].dout,
           m->n_out, m->G, (long long)B);
  std::string cached;
  if (tune_cache_get(kb, &cached)) {
    int tl[11], bk[11], sp[4];
    double d0 = 0, d1 = 0;
    std::istringstream in(cached);
    bool ok = true;
    for (int p = 0; p < 11 && ok; ++p) ok = (bool)(in >> tl[p] >> bk[p]);
    for (int l = 0; l < 4 && ok; ++l) ok = (bool)(in >> sp[l]);
    ok = ok && (bool)(in >> d0 >> d1);
    for (int p = 0; p < 11 && ok; ++p)
      ok = tl[p] >= 0 && tl[p] <= ann::GEMM_TILES && (bk[p] == 0 || bk[p] == 32 || bk[p] == 64);
    for (int l = 0; l < 4 && ok; ++l) {
      const long wn = (long)m->L[l].doutp * m->L[l].dinp;
      ok = sp[l] >= 1 && sp[l] <= 16 && B % (32L * sp[l]) == 0 &&
           (sp[l] == 1 || (size_t)sp[l] * m->G * wn <= m->wg_cap);
    }
    if (ok) {
      std::copy(tl, tl + 11, m->tt_tile);
      std::copy(bk, bk + 11, m->tt_bk);
      std::copy(sp, sp + 4, m->tt_split);
      m->tt_B = B;
      if (ms_default) *ms_default = d0;
      if (ms_tuned) *ms_tuned = d1;
      return CHEM_OK;
    }
  }
  // the products' times do not depend on the values: run them on a cleared
  // workspace (the last step's gradients are overwritten)
  CHEM_HIP(hipMemsetAsync(m->wt.base, 0, m->wt.bytes, s));
  hipEvent_t ea = nullptr, eb = nullptr;
  if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
    if (ea) (void)hipEventDestroy(ea);
    set_error("ann_autotune_train: hipEventCreate failed");
    return CHEM_EHIP;
  }
  const int G = m->G;
  constexpr int REPS = 4;
  // one product (and its split-K reduction) with the given tiling: its
  // average over REPS launches after a warm-up, or infinity if it cannot run
  auto timed = [&](int p, int tile, int bkv, int S) -> float {
    TrainProduct t = train_product(m, B, p, S);
    t.g.tile = tile;
    t.g.bk = bkv;
    const int l = p - 4;
    const long wn = p >= 4 && p < 8 ? (long)m->L[l].doutp * m->L[l].dinp : 0;
    auto once = [&]() -> chem_status {
      chem_status r = ann::gemm(t.g, t.AK, t.BK, t.epi, s, "autotune");
      if (r == CHEM_OK && S > 1)
        r = ann::sum_splits((long)G * wn, S, m->wg_part, (long)G * wn, m->gW[l], s);
      return r;
    };
    if (once() != CHEM_OK) return INFINITY;
    if (hipEventRecord(ea, s) != hipSuccess) return INFINITY;
    for (int r = 0; r < REPS; ++r)
      if (once() != CHEM_OK) return INFINITY;
    float ms = 0.0f;
    if (hipEventRecord(eb, s) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
        hipEventElapsedTime(&ms, ea, eb) != hipSuccess)
      return INFINITY;
    return ms / REPS;
  };
  double tot0 = 0.0, tot1 = 0.0;
  int tl[11], bk[11], sp[4];
  for (int p = 0; p < 11; ++p) {
    const bool wg = p >= 4 && p < 8;
    const int l = wg ? p - 4 : 0;
    const int S0 = wg ? wgrad_splits(m->L[l].doutp, m->L[l].dinp, B, G) : 1;
    const float t0 = timed(p, 0, 0, S0);
    if (!(t0 < INFINITY)) {
      (void)hipEventDestroy(ea);
      (void)hipEventDestroy(eb);
      set_error("ann_autotune_train: the built-in tiling of product %d failed to run", p);
      return CHEM_EHIP;
    }
    float best = t0;
    int bt = 0, bb = 0, bs = S0;
    for (int S = 1; S <= (wg ? 16 : 1); S *= 2) {
      if (wg) {
        const long wn = (long)m->L[l].doutp * m->L[l].dinp;
        if (B % (32L * S) != 0 || (S > 1 && (size_t)S * G * wn > m->wg_cap)) continue;
      }
      for (int tile = 1; tile <= ann::GEMM_TILES; ++tile)
        for (int bkv : {32, 64}) {
          const float t = timed(p, tile, bkv, S);
          if (t < best) {
            best = t;
            bt = tile;
            bb = bkv;
            bs = S;
          }
        }
    }
    tl[p] = bt;
    bk[p] = bb;
    if (wg) sp[l] = bs;
    tot0 += t0;
    tot1 += best;
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  std::copy(tl, tl + 11, m->tt_tile);
  std::copy(bk, bk + 11, m->tt_bk);
  std::copy(sp, sp + 4, m->tt_split);
  m->tt_B = B;
  if (ms_default) *ms_default = tot0;
  if (ms_tuned) *ms_tuned = tot1;
  std::ostringstream v;
  for (int p = 0; p < 11; ++p) v << tl[p] << " " << bk[p] << " ";
  for (int l = 0; l < 4; ++l) v << sp[l] << " ";
  v << std::setprecision(17) << tot0 << " " << tot1;
  tune_cache_put(kb, v.str());
  return CHEM_OK;
}

namespace {
// file versions: 1 = one network; 2 adds the member count after the header
const char MAGIC[8] = {'C', 'H', 'E', 'M', 'A', 'N', 'N', '1'};
const char MAGIC2[8] = {'C', 'H', 'E', 'M', 'A', 'N', 'N', '2'};

bool wr(FILE *f, const void *p, size_t n) { return fwrite(p, 1, n, f) == n; }
bool rd(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }
}  // namespace

extern "C" chem_status ann_save(const ann_model *m, const char *path) {
  chem_status st = check_model("ann_save", m);
  if (st != CHEM_OK) return st;
  if (!path) {
    set_error("ann_save: null path");
    return CHEM_EINVAL;
  }
  FILE *f = fopen(path, "wb");
  if (!f) {
    set_error("ann_save: cannot open %s", path);
    return CHEM_EINVAL;
  }
  bool ok = wr(f, m->G > 1 ? MAGIC2 : MAGIC, 8);
  int32_t hdr[7] = {m->n_in, m->n_out, m->L[0].dout, m->L[1].dout, m->L[2].dout, m->prec,
                    m->has_norm ? 1 : 0};
  const int32_t members = m->G;
  ok = ok && wr(f, hdr, sizeof(hdr)) && (m->G == 1 || wr(f, &members, 4)) &&
       wr(f, &m->step, 8) && wr(f, &m->nm.lambda, 4) && wr(f, &m->nm.dt_model, 8);
  if (m->has_norm)
    for (auto *v : {&m->h_mu_in, &m->h_sd_in, &m->h_lo, &m->h_hi, &m->h_mu_out, &m->h_sd_out})
      ok = ok && wr(f, v->data(), v->size() * 4);
  for (int idx = 0; idx < 4 * m->G && ok; ++idx) {
    const int l = idx & 3;
    const ann::Layer &L = m->L[l];
    std::vector<float> W((size_t)L.dout * L.din), b(L.dout);
    const float *srcW[3] = {m->Wm[l], m->mW[l], m->vW[l]};
    const float *srcb[3] = {m->bm[l], m->mb[l], m->vb[l]};
    for (int q = 0; q < 3 && ok; ++q) {
      st = download_pair(m, idx, srcW[q], srcb[q], W.data(), b.data());
      if (st != CHEM_OK) {
        fclose(f);
        return st;
      }
      ok = wr(f, W.data(), W.size() * 4) && wr(f, b.data(), b.size() * 4);
    }
  }
  ok = (fclose(f) == 0) && ok;
  if (!ok) {
    set_error("ann_save: write to %s failed", path);
    return CHEM_EINVAL;
  }
  return CHEM_OK;
}

extern "C" chem_status ann_load(const char *path, ann_model **out) {
  if (!path || !out) {
    set_error("ann_load: null argument");
    return CHEM_EINVAL;
  }
  *out = nullptr;
  FILE *f = fopen(path, "rb");
  if (!f) {
    set_error("ann_load: cannot open %s", path);
    return CHEM_EINVAL;
  }
  char mg[8];
  int32_t hdr[7];
  int32_t members = 1;
  int64_t step = 0;
  float lambda = 0;
  double dtm = 0;
  bool ok = rd(f, mg, 8);
  const bool v2 = ok && memcmp(mg, MAGIC2, 8) == 0;
  ok = ok && (v2 || memcmp(mg, MAGIC, 8) == 0) && rd(f, hdr, sizeof(hdr)) &&
       (!v2 || rd(f, &members, 4)) && rd(f, &step, 8) && rd(f, &lambda, 4) && rd(f, &dtm, 8);
  if (!ok) {
    fclose(f);
    set_error("ann_load: %s is not a model file", path);
    return CHEM_EMODEL;
  }
  ann_arch arch{hdr[0], hdr[1], {hdr[2], hdr[3], hdr[4]}, hdr[5], members};
  ann_model *m = nullptr;
  chem_status st = ann_create(&arch, 0, &m);
  if (st != CHEM_OK) {
    fclose(f);
    return st;
  }
  if (hdr[6]) {
    std::vector<float> v[6];
    const int sz[6] = {m->n_in, m->n_in, m->n_in, m->n_in, m->n_out, m->n_out};
    for (int q = 0; q < 6 && ok; ++q) {
      v[q].resize(sz[q]);
      ok = rd(f, v[q].data(), sz[q] * 4);
    }
    if (ok) {
      ann_norm nn{lambda, dtm, v[0].data(), v[1].data(), v[2].data(), v[3].data(), v[4].data(),
                  v[5].data()};
      st = ann_set_norm(m, &nn);
      ok = st == CHEM_OK;
    }
  }
  for (int idx = 0; idx < 4 * m->G && ok; ++idx) {
    const int l = idx & 3;
    const ann::Layer &L = m->L[l];
    const size_t ow = (size_t)(idx >> 2) * layer_elems(L), ob = (size_t)(idx >> 2) * L.doutp;
    std::vector<float> W((size_t)L.dout * L.din), b(L.dout);
    float *dstW[3] = {m->Wm[l] + ow, m->mW[l] + ow, m->vW[l] + ow};
    float *dstb[3] = {m->bm[l] + ob, m->mb[l] + ob, m->vb[l] + ob};
    for (int q = 0; q < 3 && ok; ++q) {
      ok = rd(f, W.data(), W.size() * 4) && rd(f, b.data(), b.size() * 4);
      if (!ok) break;
      std::vector<float> Wp((size_t)L.doutp * L.dinp, 0.0f), bp(L.doutp, 0.0f);
      for (int o = 0; o < L.dout; ++o) {
        for (int i = 0; i < L.din; ++i) Wp[(size_t)o * L.dinp + i] = W[(size_t)o * L.din + i];
        bp[o] = b[o];
      }
      ok = hipMemcpy(dstW[q], Wp.data(), Wp.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(dstb[q], bp.data(), bp.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (ok)
      ok = ann::to_bf16((int64_t)layer_elems(L), m->Wm[l] + ow, m->Wb[l] + ow, nullptr) ==
           CHEM_OK;
    m->wt_stale = true;
  }
  fclose(f);
  if (!ok || hipDeviceSynchronize() != hipSuccess) {
    ann_destroy(m);
    set_error("ann_load: %s is truncated or inconsistent", path);
    return CHEM_EMODEL;
  }
  m->step = step;
  *out = m;
  return CHEM_OK;
}

namespace {
float reduce_amax(const std::vector<float> &p) {
  float a = 0.0f;
  for (float v : p) a = fmaxf(a, v);
  return a;
}
}  // namespace

extern "C" chem_status ann_quantize_fp8(ann_model *m, chem_batch calib, const double *T,
                                        const double *p, const double *Y, void *stream) {
  chem_status st = check_model("ann_quantize_fp8", m);
  if (st != CHEM_OK) return st;
  if (m->G > 1) {
    set_error("ann_quantize_fp8: the FP8 variant is built for the single network only");
    return CHEM_EUNSUPPORTED;
  }
  if (!m->has_norm || m->n_in != m->n_out + 2) {
    set_error("ann_quantize_fp8: statistics not set or n_in != n_out + 2");
    return CHEM_EMODEL;
  }
  if (calib.n < 1 || calib.ld < calib.n || !T || !p || !Y) {
    set_error("ann_quantize_fp8: needs a non-empty calibration batch");
    return CHEM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = calib.n < CHUNK ? calib.n : CHUNK;
  if ((st = grow_infer(m, n)) != CHEM_OK) return st;
  const bool prev = m->use_fp8;
  m->use_fp8 = false;  // calibrate on the BF16 activations
  st = forward_chunk(m, model_ws(m), n, calib.ld, T, p, Y, m->U, m->L[3].doutp, nullptr, 0.0f, s,
                     true);
  m->use_fp8 = prev;
  if (st != CHEM_OK) return st;
  m->n2p = fp8_n2p(m);
  m->k3p = fp8_k3p(m);
  m->kq1 = fp8_kq1(m);
  if (!m->fp8_buf) {
    const size_t b1 = (size_t)m->n2p * m->kq1, b2 = (size_t)m->L[2].doutp * m->k3p;
    const size_t off1 = align256(b1), off2 = off1 + align256(b2);
    const size_t off3 = off2 + align256(b1), off4 = off3 + align256(b2);
    CHEM_HIP(hipMalloc(&m->fp8_buf, off4 + (size_t)m->n2p * 4 + 1024 * 4));
    unsigned char *b = (unsigned char *)m->fp8_buf;
    m->Wq1 = b;
    m->Wq2 = b + off1;
    m->Wq1t = b + off2;
    m->Wq2t = b + off3;
    m->bq1 = (float *)(b + off4);
  }
  float *part = m->bq1 + m->n2p;  // 1024 floats of scratch for the amax partials
  const int NP = 256;
  std::vector<float> h(NP);
  float amax_v[4];
  const void *srcs[4] = {m->H[0], m->H[1], m->Wm[1], m->Wm[2]};
  const int64_t cnt[4] = {n * m->L[0].doutp, n * m->L[1].doutp,
                          (int64_t)layer_elems(m->L[1]), (int64_t)layer_elems(m->L[2])};
  for (int q = 0; q < 4; ++q) {
    if ((st = ann::amax(cnt[q], srcs[q], q < 2, part, NP, s)) != CHEM_OK) return st;
    hipError_t e = hipMemcpyAsync(h.data(), part, NP * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "ann_quantize_fp8: amax read back");
    amax_v[q] = reduce_amax(h);
  }
  auto sc = [](float a) { return a > 0.0f && isfinite(a) ? a / 448.0f : 1.0f; };
  m->sa[1] = sc(amax_v[0]);
  m->sa[2] = sc(amax_v[1]);
  m->sw[1] = sc(amax_v[2]);
  m->sw[2] = sc(amax_v[3]);
  st = ann::quant_e4m3(m->Wm[1], m->L[1].dinp, m->L[1].dout, m->L[1].din, m->Wq1, m->n2p,
                       m->kq1, 1.0f / m->sw[1], s);
  if (st != CHEM_OK) return st;
  st = ann::quant_e4m3(m->Wm[2], m->L[2].dinp, m->L[2].doutp, m->L[2].din, m->Wq2,
                       m->L[2].doutp, m->k3p, 1.0f / m->sw[2], s);
  if (st != CHEM_OK) return st;
  if ((st = ann::tile_e4m3(m->n2p, m->kq1, m->Wq1, m->Wq1t, s)) != CHEM_OK) return st;
  if ((st = ann::tile_e4m3(m->L[2].doutp, m->k3p, m->Wq2, m->Wq2t, s)) != CHEM_OK) return st;
  CHEM_HIP(hipStreamSynchronize(s));
  std::vector<float> hb(m->n2p, 0.0f);  // layer-1 bias, zero-padded to the FP8 width
  CHEM_HIP(hipMemcpy(hb.data(), m->bm[1], (size_t)m->L[1].dout * 4, hipMemcpyDeviceToHost));
  CHEM_HIP(hipMemcpy(m->bq1, hb.data(), hb.size() * 4, hipMemcpyHostToDevice));
  m->fp8_ready = true;
  m->use_fp8 = true;
  return CHEM_OK;
}

extern "C" chem_status ann_set_precision(ann_model *m, int32_t prec) {
  chem_status st = check_model("ann_set_precision", m);
  if (st != CHEM_OK) return st;
  if (prec == 0) {
    m->use_fp8 = false;
    return CHEM_OK;
  }
  if (prec == 1) {
    if (!m->fp8_ready) {
      set_error("ann_set_precision: call ann_quantize_fp8 first");
      return CHEM_EMODEL;
    }
    m->use_fp8 = true;
    return CHEM_OK;
  }
  set_error("ann_set_precision: prec must be 0 (BF16) or 1 (FP8 hidden layers)");
  return CHEM_EINVAL;
}

extern "C" chem_status ann_get_fp8_scales(const ann_model *m, float *act, float *wgt) {
  chem_status st = check_model("ann_get_fp8_scales", m);
  if (st != CHEM_OK) return st;
  if (!m->fp8_ready) {
    set_error("ann_get_fp8_scales: not quantised");
    return CHEM_EMODEL;
  }
  if (act) {
    act[0] = m->sa[1];
    act[1] = m->sa[2];
  }
  if (wgt) {
    wgt[0] = m->sw[1];
    wgt[1] = m->sw[2];
  }
  return CHEM_OK;
}

extern "C" chem_status ann_step_graph_create(ann_model *m, const chem_mech *mech, chem_batch batch,
                                             double dt, double *T, const double *p, double *Y,
                                             double *RR, uint8_t *flags, int64_t *n_fallback,
                                             const ann_step_opts *opts,
                                             const chem_step_opts *fb_opts, void *stream,
                                             chem_graph **out) {
  (void)stream;  // the preparation allocates synchronously; nothing is enqueued
  chem_status st = check_model("ann_step_graph_create", m);
  if (st != CHEM_OK) return st;
  if (batch.n < 1) {
    set_error("ann_step_graph_create: empty batch");
    return CHEM_EINVAL;
  }
  // allocations before the capture; inside it, the BF16 weight layouts are
  // rebuilt from the BF16 copies (so replays follow weight updates)
  st = step_prepare(m, batch.n, !opts || opts->fallback != 0);
  if (st != CHEM_OK) return st;
  if (opts && opts->audit_fraction > 0.0f &&
      (st = audit_prepare(m, m->wi.cap, opts->audit_fraction)) != CHEM_OK)
    return st;
  m->wt_stale = true;
  st = capture_graph(
      [&](hipStream_t cs) {
        return ann_step(m, mech, batch, dt, T, p, Y, RR, flags, n_fallback, opts, fb_opts, cs);
      },
      out);
  m->wt_stale = true;  // nothing ran during the capture
  if (st != CHEM_OK) return st;
  m->graph_refs++;
  (*out)->release = release_graph;
  (*out)->owner = m;
  return CHEM_OK;
}
