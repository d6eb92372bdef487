// Internal declarations of the surrogate (ANN) path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chem_internal.h"

namespace ann {

typedef unsigned short u16;  // bfloat16 storage

constexpr int NLAYER = 4;

// Dense layer l maps din[l] -> dout[l]; stored dims are padded to a multiple
// of 32 with zero weights and biases (padded units are exactly zero).
struct Layer {
  int din, dout;    // logical
  int dinp, doutp;  // padded
};

struct Norm {
  float lambda;
  double dt_model;
  float *mu_in, *sd_in, *lo, *hi;  // device [n_in]
  float *mu_out, *sd_out;          // device [n_out]
};

enum { EPI_F32 = 0, EPI_GELU = 1, EPI_GELUGRAD = 2, EPI_GELU_Q8 = 3, EPI_GELU_NEXT = 4 };

struct GemmArgs {
  int M, N, K;
  const u16 *A;
  long lda;
  const u16 *B;
  long ldb;
  const float *bias;
  u16 *Cb;
  long ldcb;
  float *Cf;
  long ldcf;
  float *Z;
  long ldz;
  // FP8 variants: operands A8 [M][K], B8 [N][K] (E4M3), output Cq (E4M3)
  const uint8_t *A8;
  const uint8_t *B8;
  uint8_t *Cq;
  long ldcq;
  float scale;  // multiplies the accumulator before the bias (FP8 operands)
  float qinv;   // 1/scale of the E4M3 output (EPI_GELU_Q8)
  // split-K (EPI_F32 without bias only): K is cut into ksplit equal ranges,
  // range s writes its partial product to Cf + s * split_stride
  int ksplit;
  long split_stride;
  // EPI_GELU_NEXT: the activations never leave the chip; the next (output)
  // layer Cf[m][0..N2) = B2 [N2][N] * GELU(...)[m][:] + bias2 follows in the
  // same kernel (N2 a multiple of 16, Cf row stride ldcf)
  const u16 *B2;
  const float *bias2;
  int N2;
  // K-blocked operand layouts of the inference path (bits: 1 = A, 2 = B,
  // 4 = the BF16 / E4M3 output): element (r, k) of a K-blocked matrix sits at
  // (k / KB) ld + r KB + k % KB with KB = 32 elements (BF16) or 128 bytes
  // (E4M3), so the rows of one K-step are contiguous; ld is then the stride
  // between K-blocks.  Only the direct-to-LDS kernels accept it.
  int tiled;
  // grouped product (the networks of a per-species ensemble, one per
  // blockIdx.z): group z reads A + z gA, B + z gB, bias + z gbias and writes
  // Cb + z gcb, Cf + z gcf, Z + z gz (element strides; 0 = shared operand).
  // Only the generic tiling (training products) accepts groups > 1.
  int groups;
  long gA, gB, gbias, gcb, gcf, gz;
  // tiling of the generic kernel chosen by the autotuner: tile 0 = the
  // built-in rule, 1..GEMM_TILES = gemm_tile_shape(tile); bk 0 = the built-in
  // rule, else the K-step (32 or 64).  The direct-to-LDS paths ignore them.
  int tile, bk;
};
constexpr int GEMM_TILES = 4;
// Block shape (rows x columns of C) of generic tiling t in 1..GEMM_TILES.
void gemm_tile_shape(int t, int *bm, int *bn);
enum { TILED_A = 1, TILED_B = 2, TILED_C = 4 };

// C = epi(A * op(B)); AK: A is [M][K] row-major (else [K][M]); BK: B is [N][K]
// row-major (else [K][N]).
chem_status gemm(const GemmArgs &g, bool AK, bool BK, int epi, hipStream_t s,
                 const char *label);
// Whether gemm() can run this forward layer with EPI_GELU_NEXT (the output
// layer fused into its epilogue).
bool gemm_fuses_next(const GemmArgs &g);
// The first two hidden layers in one kernel: H = GELU(W2 GELU(W1 x + b1) + b2)
// for every cell, the first layer recomputed per K-step of the second from the
// cell's 32 inputs, so its activations never reach HBM.
struct Mlp12Args {
  int M, N, K;      // cells, second-layer outputs, first-layer outputs
  const u16 *X;     // [M][32] BF16 network inputs
  const u16 *W1;    // [K][32] BF16 first-layer weights
  const float *b1;  // [K]
  const u16 *W2p;   // second-layer weights [N][K] K-blocked by 32, each block
                    // permuted by mlp12_slot (tile_bf16 with permute = true)
  long ldw2;        // elements between K-blocks of W2p (>= 32 N)
  const float *b2;  // [N]
  u16 *H;           // BF16 output: [M][ldh] row-major, or K-blocked by 32
  long ldh;         // (tiled: elements between K-blocks) when tiled is set
  bool tiled;
};
// Position of first-layer feature f (0..31 within one K-step) in mlp12's
// second-layer K-step: the MFMA leaves features 4g..4g+3 and 16+4g..16+4g+3
// with the lanes of 16-lane group g, which supply K positions 8g..8g+7.
__host__ __device__ inline int mlp12_slot(int f) {
  return 8 * ((f & 15) >> 2) + 4 * (f >> 4) + (f & 3);
}
// Whether mlp12() takes this shape (32 inputs, K a multiple of 32 up to
// 2048, N a multiple of 400, aligned operands).
bool mlp12_ok(const Mlp12Args &g);
chem_status mlp12(const Mlp12Args &g, hipStream_t s, const char *label);
// Whether gemm8() can run this layer with EPI_GELU_NEXT (the BF16 output
// layer fused into its epilogue).
bool gemm8_fuses_next(const GemmArgs &g);
// E4M3 x E4M3 GEMM (both K-contiguous, K a multiple of 64), epi GELU, GELU_Q8
// or GELU_NEXT.
chem_status gemm8(const GemmArgs &g, int epi, hipStream_t s, const char *label);
// max |x| over n BF16 (bf16 = true) or FP32 values, into part[0..nparts)
chem_status amax(int64_t n, const void *x, bool bf16, float *part, int nparts, hipStream_t s);
// dst [rows_p][cols_p] E4M3 = e4m3(src[r][c] * qinv) for r < rows, c < cols, else 0
chem_status quant_e4m3(const float *src, long ld_src, int rows, int cols, uint8_t *dst,
                       int rows_p, int cols_p, float qinv, hipStream_t s);
// dst [cols_p/128][rows_p][128] (E4M3) from the row-major E4M3 src [rows_p][cols_p]
chem_status tile_e4m3(int rows_p, int cols_p, const uint8_t *src, uint8_t *dst, hipStream_t s);

struct FeatArgs {
  int64_t n, ld;
  const double *T, *p, *Y;
  const int64_t *index;  // optional gather list
  int K, dinp;
  const float *mu, *sd;
  float lambda;
  u16 *X;  // [n][dinp] bf16
  // optional out-of-distribution test of the raw features against the
  // training range widened by ood_margin of its span: ood[i] = 1 if outside
  uint8_t *ood;
  const float *lo, *hi;
  float ood_margin;
};
chem_status features(const FeatArgs &a, hipStream_t s);

struct TargetArgs {
  int64_t n, ld;
  const double *Y0, *Y1;
  const int64_t *index;
  int K, doutp;
  const float *mu, *sd;
  float lambda;
  float *U;  // [n][doutp] fp32
};
chem_status targets(const TargetArgs &a, hipStream_t s);

chem_status l1_grad(int64_t n, int K, int doutp, const float *U, const float *Ut, u16 *Gb,
                    float *Gf, double *loss_part, int nparts, float *loss, hipStream_t s);

// Physics terms of the training loss (mass-fraction sum, energy at the
// reference final temperature T1, heat release at 298.15 K): their gradient
// is added to Gf (and Gb refreshed from it), w-weighted batch means are
// added to *loss, the unweighted means written to terms[3] (nullable).
struct PhysArgs {
  int64_t n, ld;
  int K, doutp;
  const float *U, *Ut;  // network output and targets, z-space [n][doutp]
  float *Gf;
  u16 *Gb;
  const float *mu, *sd;  // output statistics
  const double *T1;      // [ld] reference final temperature, gathered through index
  const int64_t *index;
  float w[3];
};
constexpr int PHYS_PARTS = 64;
chem_status phys_grad(const PhysArgs &a, const chem::DevMech &M, double *part, float *loss,
                      float *terms, hipStream_t s);
// out[j] = sum over the M rows of X[:, j]; part: COLSUM_PARTS * N doubles.
// With groups > 1, group z sums X + z gx into out + z gout (part: groups
// times as many doubles).
constexpr int COLSUM_PARTS = 64;
chem_status colsum(int64_t M, int N, const float *X, long ldx, float *out, double *part,
                   hipStream_t s, int groups = 1, long gx = 0, long gout = 0);
// Per-species ensemble: member g's output is column 0 of U + g gu (row
// stride ldu) and its target column g of Ut (row stride ldt); the gradient
// sign(u - u*) / (n G) goes to column 0 of Gb/Gf + g gu (every other column
// 0), and *loss is the mean of |u - u*| over samples and members.
chem_status l1_grad_members(int64_t n, int G, int ldu, long gu, const float *U, const float *Ut,
                            int ldt, u16 *Gb, float *Gf, double *loss_part, int nparts,
                            float *loss, hipStream_t s);
// dst[i * ldd] = src[i * lds] for i < n (one output column of an ensemble
// member into the ensemble's output)
chem_status take_col(int64_t n, const float *src, int lds, float *dst, int ldd, hipStream_t s);
// out[i] = sum_{s < S} part[s * stride + i], in order of s
chem_status sum_splits(int64_t n, int S, const float *part, long stride, float *out,
                       hipStream_t s);
// Adam over several tensors in one launch: tensor k holds elements
// start[k] .. start[k + 1] - 1 of the concatenation (start[0] = 0).
constexpr int ADAM_MAX = 8;
struct AdamTable {
  int count;
  int64_t start[ADAM_MAX + 1];
  float *W[ADAM_MAX];
  const float *g[ADAM_MAX];
  float *m[ADAM_MAX];
  float *v[ADAM_MAX];
  u16 *Wb[ADAM_MAX];  // BF16 copy of W, or null
};
chem_status adam_multi(const AdamTable &t, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, hipStream_t s);
chem_status to_bf16(int64_t n, const float *src, u16 *dst, hipStream_t s);
// dst [K/32][N][32] from src [N][K] (BF16, K a multiple of 32); with permute,
// element k % 32 of each block goes to position mlp12_slot(k % 32) (the K
// order in which mlp12 produces the first layer's features)
chem_status tile_bf16(int N, int K, const u16 *src, u16 *dst, hipStream_t s,
                      bool permute = false);

struct PostArgs {
  int64_t n, ld;
  double dt;
  double *T;
  const double *p;
  double *Y;
  double *RR;
  uint8_t *flags;
  const float *U;  // [n][doutp] z-space outputs
  int doutp;
  Norm nm;
  int n_in;
  float residual_tol, ood_margin;
  const uint8_t *ood;             // per-cell out-of-distribution bits (k_features), nullable
  int force_flag;                 // flag bits set on every cell
  int32_t *fb_index;              // fallback list (cell indices index_base + i)
  unsigned long long *fb_count;   // device counter
  int64_t index_base;
};
chem_status post(const chem::DevMech &M, const PostArgs &a, hipStream_t s);

// The audit of a chunk: cells 0, stride, 2 stride, ... of the chunk's arrays
// (T, p, Y with leading dimension ld; flags as post wrote them) against their
// copies Ta, pa, Ya (integrated by the plain step; Y0a keeps the inputs),
// na cells, stats_a [3][na] the reference integration's rows.
struct AuditArgs {
  int64_t na, stride, ld;
  int K;
  const double *T, *p, *Y;
  const uint8_t *flags;
  double *Ta, *pa, *Ya, *Y0a;
  const int32_t *stats_a;
  double *audit;
};
chem_status audit_init(double *audit, int K, hipStream_t s);
chem_status audit_gather(const AuditArgs &a, hipStream_t s);
chem_status audit_compare(const AuditArgs &a, hipStream_t s);

struct StatArgs {
  int64_t n, ld;
  const double *T, *p, *Y0, *Y1;
  int K;
  float lambda;
  double *part;  // [nblocks][F][4] sums and sums of squares of x - shift_f, min, max; then shift[F]
  int nblocks;
};
chem_status stats_partial(const StatArgs &a, hipStream_t s);

}  // namespace ann
