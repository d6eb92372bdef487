// Surrogate-form kernels for gfx950: BF16 MFMA GEMM with fused epilogues
// (bias + GELU, GELU-derivative, FP32 out), the Box-Cox/z-score prologue, the
// L1-loss gradient, deterministic column sums, Adam, and the per-cell
// post-processing of the network output (de-normalisation, element-conserving
// projection, clipping, residual and out-of-distribution flags, enthalpy
// Newton for T, reaction rates).
#include <math.h>

#include "ann_internal.h"

namespace ann {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr double RG = 8.314462618;

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ u16 f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}

// erf(x) by the approximation of Abramowitz & Stegun 7.1.28,
// erf(x) = 1 - (1 + a1 x + ... + a6 x^6)^-16 (|error| <= 3e-7 exactly, about
// 2e-6 in FP32): six FMAs, four squarings and one hardware reciprocal -- a
// single transcendental, well inside the BF16 rounding of the activations it
// feeds.  Large |x| overflows the power to +inf and gives exactly +-1.
__device__ __forceinline__ float erf_as(float x) {
  const float a = fabsf(x);
  float q = fmaf(a, fmaf(a, fmaf(a, fmaf(a, fmaf(a, fmaf(a, 0.0000430638f, 0.0002765672f),
                                                   0.0001520143f),
                                          0.0092705272f),
                                 0.0422820123f),
                        0.0705230784f),
               1.0f);
  q *= q;
  q *= q;
  q *= q;
  q *= q;
  return copysignf(1.0f - __builtin_amdgcn_rcpf(q), x);
}

// GELU(x) = x Phi(x) = max(x, 0) - (|x| / 2) erfc(|x| / sqrt 2) (both signs),
// with erfc(z) = (1 + a1 z + ... + a6 z^6)^-16 of 7.1.28.  The coefficients
// carry the powers of 1/sqrt 2, and all of them (the leading 1 included) a
// factor 2^(1/16), so that the 16th power is twice the original and its
// reciprocal already holds the 1/2: six FMAs, four squarings, one
// reciprocal, a max and a final FMA.  No cancellation for negative x; over
// [-12, 12] the FP32 result is within 7e-7 of the exact GELU.
__device__ __forceinline__ float gelu(float x) {
  const float a = fabsf(x);
  float q = fmaf(a, fmaf(a, fmaf(a, fmaf(a, fmaf(a, fmaf(a, 5.6213e-06f, 5.105521e-05f),
                                                   3.9686136e-05f),
                                          0.0034227392f),
                                 0.022076998f),
                        0.052075163f),
               1.0442737f);
  q *= q;
  q *= q;
  q *= q;
  q *= q;
  return fmaf(-a, __builtin_amdgcn_rcpf(q), fmaxf(x, 0.0f));
}

__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) +
         x * __builtin_amdgcn_exp2f(-0.5f * x * x * 1.4426950408889634f) * 0.39894228040143268f;
}

// FP32 -> OCP FP8 E4M3 (e4m3fn: no infinities, max 448), saturating, round to
// nearest even.
__device__ __forceinline__ uint8_t f2e4m3(float x) {
  if (x != x) return 0x7f;
  const unsigned sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fminf(fabsf(x), 448.0f);
  unsigned code;
  if (a < 0.015625f) {  // below 2^-6: subnormals, spacing 2^-9 (8 -> smallest normal)
    code = (unsigned)rintf(a * 512.0f);
  } else {
    unsigned u = __float_as_uint(a);
    u += 0x7ffffu + ((u >> 20) & 1u);  // keep 3 mantissa bits, ties to even
    code = ((((u >> 23) & 0xffu) - 120u) << 3) | ((u >> 20) & 7u);
  }
  return (uint8_t)(sign | code);
}

// Four values to packed E4M3 with the hardware conversion (round to nearest
// even) after clamping to +-448: bit-identical to f2e4m3 for every finite
// float (checked exhaustively on gfx950); a NaN input becomes -448.
__device__ __forceinline__ unsigned e4m3x4(float a, float b, float c, float d) {
  auto cl = [](float x) { return fminf(fmaxf(x, -448.0f), 448.0f); };
  int r = __builtin_amdgcn_cvt_pk_fp8_f32(cl(a), cl(b), 0, false);
  r = __builtin_amdgcn_cvt_pk_fp8_f32(cl(c), cl(d), r, true);
  return (unsigned)r;
}


// ------------------------------------------------------------------ GEMM
// Block = WM x WN waves; each wave owns TM x TN tiles of 32x32 computed with
// v_mfma_f32_32x32x16_bf16.  Operand tiles are staged through LDS in a
// K-contiguous layout (double buffered); operands stored MN-contiguous in
// global memory are transposed while being written to LDS.
//
// BK (32 or 64) is the K-step: with one step prefetched into registers while
// the current one is multiplied, each step waits for one round trip of its
// loads, so the training-size products (few blocks per CU) take 64-wide steps
// when the K range of a block allows it.
template <int WM, int WN, int TM, int TN, bool AK, bool BKC, int EPI, int BK = 32>
__global__ __launch_bounds__(WM *WN * 64) void k_gemm(GemmArgs g) {
  if (g.groups > 1) {
    // this block's member of a grouped product
    const long z = blockIdx.z;
    g.A += z * g.gA;
    g.B += z * g.gB;
    if (g.bias) g.bias += z * g.gbias;
    if (g.Cb) g.Cb += z * g.gcb;
    if (g.Cf) g.Cf += z * g.gcf;
    if (g.Z) g.Z += z * g.gz;
  }
  constexpr int BM = WM * TM * 32, BN = WN * TN * 32, LK = BK + 8;
  constexpr int NT = WM * WN * 64;
  __shared__ __attribute__((aligned(16))) u16 As[2][BM * LK];
  __shared__ __attribute__((aligned(16))) u16 Bs[2][BN * LK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  // Block order: the N-tiles of one M-tile are consecutive logical blocks on
  // the same XCD (blocks are dealt round-robin over the 8 XCDs), so an
  // activation tile is fetched from HBM once and reused from that XCD's L2.
  const int ntn = (g.N + BN - 1) / BN;
  const int ntm = (g.M + BM - 1) / BM;
  const int total = ntn * ntm;
  const int per_xcd = (total + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (logical >= total) return;
  const long m0 = (long)(logical / ntn) * BM, n0 = (long)(logical % ntn) * BN;
  // split-K range of this block (blockIdx.y); the whole K when not split
  const int kper = g.ksplit > 1 ? g.K / g.ksplit : g.K;
  const int kbase = (int)blockIdx.y * kper, kend = kbase + kper;
  // K-contiguous operands move as 16-byte chunks (8 K values of one row).  An
  // MN-contiguous operand moves as blocks of 4 K rows x 8 columns: four
  // coalesced 16-byte loads, a transpose in registers, and eight 8-byte LDS
  // stores (4 K values of one column each), in place of 2-byte stores that
  // fell on four LDS banks.
  constexpr int ACH = BM * BK / 8, BCH = BN * BK / 8;
  constexpr int ATB = BM * BK / 32, BTB = BN * BK / 32;
  constexpr int APT = AK ? (ACH + NT - 1) / NT : 4 * ((ATB + NT - 1) / NT);
  constexpr int BPT = BKC ? (BCH + NT - 1) / NT : 4 * ((BTB + NT - 1) / NT);
  uint4 ra[APT], rb[BPT];
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  // chunk c of a K-contiguous tile: row c / (BK / 8), K offset 8 (c % (BK / 8));
  // block c of an MN-contiguous tile: K rows 4 (c % (BK / 4)) + 0..3, columns
  // 8 (c / (BK / 4)) + 0..7
  auto load_kc = [&](const u16 *src, long ld, long r0, long rows, int k0, int nch, uint4 *v,
                     int cnt) {
#pragma unroll
    for (int i = 0; i < cnt; ++i) {
      const int c = tid + i * NT;
      uint4 x = make_uint4(0, 0, 0, 0);
      if (c < nch) {
        const int r = c / (BK / 8), kc = (c % (BK / 8)) * 8;
        if (r0 + r < rows && k0 + kc < kend) x = *(const uint4 *)(src + (r0 + r) * ld + k0 + kc);
      }
      v[i] = x;
    }
  };
  auto load_mn = [&](const u16 *src, long ld, long c0, long cols, int k0, int nblk_, uint4 *v,
                     int cnt) {
#pragma unroll
    for (int i = 0; i < cnt / 4; ++i) {
      const int c = tid + i * NT;
      const int kq = (c % (BK / 4)) * 4, mc = (c / (BK / 4)) * 8;
      const bool in = c < nblk_ && c0 + mc < cols;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        v[4 * i + q] = in && k0 + kq + q < kend
                           ? *(const uint4 *)(src + (long)(k0 + kq + q) * ld + c0 + mc)
                           : make_uint4(0, 0, 0, 0);
    }
  };
  auto store_kc = [&](u16 *dst, int nch, const uint4 *v, int cnt) {
#pragma unroll
    for (int i = 0; i < cnt; ++i) {
      const int c = tid + i * NT;
      if (c < nch) {
        const int r = c / (BK / 8), kc = (c % (BK / 8)) * 8;
        *(uint4 *)&dst[r * LK + kc] = v[i];
      }
    }
  };
  auto store_mn = [&](u16 *dst, int nblk_, const uint4 *v, int cnt) {
    auto dw = [](const uint4 &x, int d) { return d == 0 ? x.x : (d == 1 ? x.y : (d == 2 ? x.z : x.w)); };
    // the two BF16 of column j in K rows (a, b), row a in the low half
    auto pair = [](unsigned a, unsigned b, int h) {
      return h == 0 ? (a & 0xffffu) | (b << 16) : (a >> 16) | (b & 0xffff0000u);
    };
#pragma unroll
    for (int i = 0; i < cnt / 4; ++i) {
      const int c = tid + i * NT;
      if (c < nblk_) {
        const int kq = (c % (BK / 4)) * 4, mc = (c / (BK / 4)) * 8;
        const uint4 *x = v + 4 * i;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int d = j >> 1, h = j & 1;
          *(uint2 *)&dst[(mc + j) * LK + kq] = make_uint2(pair(dw(x[0], d), dw(x[1], d), h),
                                                          pair(dw(x[2], d), dw(x[3], d), h));
        }
      }
    }
  };
  auto load = [&](int k0) {
    if constexpr (AK) load_kc(g.A, g.lda, m0, g.M, k0, ACH, ra, APT);
    else load_mn(g.A, g.lda, m0, g.M, k0, ATB, ra, APT);
    if constexpr (BKC) load_kc(g.B, g.ldb, n0, g.N, k0, BCH, rb, BPT);
    else load_mn(g.B, g.ldb, n0, g.N, k0, BTB, rb, BPT);
  };
  auto store = [&](int buf) {
    if constexpr (AK) store_kc(As[buf], ACH, ra, APT);
    else store_mn(As[buf], ATB, ra, APT);
    if constexpr (BKC) store_kc(Bs[buf], BCH, rb, BPT);
    else store_mn(Bs[buf], BTB, rb, BPT);
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = *(const bf16x8 *)&As[buf][(wm * TM * 32 + i * 32 + (lane & 31)) * LK + kk +
                                         8 * (lane >> 5)];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = *(const bf16x8 *)&Bs[buf][(wn * TN * 32 + j * 32 + (lane & 31)) * LK + kk +
                                         8 * (lane >> 5)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  // a K range that is not a multiple of BK ends with a zero-filled step (K is
  // a multiple of 32, so 8-wide chunks and 4-row blocks are wholly in or out)
  const int nk = (kper + BK - 1) / BK;
  load(kbase);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load(kbase + (kt + 1) * BK);
    compute(cur);
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  float *const Cf = (EPI == EPI_F32 && g.ksplit > 1) ? g.Cf + blockIdx.y * g.split_stride : g.Cf;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const long col = n0 + wn * TN * 32 + j * 32 + (lane & 31);
      if (col >= g.N) continue;
      const float bias = g.bias ? g.bias[col] : 0.0f;
      // the tile's 16 pre-activations are loaded before its first store (the
      // stores may alias them as far as the compiler knows, which would make
      // every load wait for the store before it)
      float zt[16];
      if constexpr (EPI == EPI_GELUGRAD) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const long row = m0 + wm * TM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          zt[r] = row < g.M ? g.Z[row * g.ldz + col] : 0.0f;
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long row = m0 + wm * TM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row >= g.M) continue;
        const float v = acc[i][j][r];
        if (EPI == EPI_F32) {
          Cf[row * g.ldcf + col] = v + bias;
        } else if (EPI == EPI_GELU) {
          const float z = v + bias;
          if (g.Z) g.Z[row * g.ldz + col] = z;
          if (g.Cb) g.Cb[row * g.ldcb + col] = f2bf(gelu(z));
          if (g.Cf) g.Cf[row * g.ldcf + col] = gelu(z);
        } else if (EPI == EPI_GELU_Q8) {
          g.Cq[row * g.ldcq + col] = f2e4m3(gelu(v + bias) * g.qinv);
        } else {
          const float d = v * gelu_grad(zt[r]);
          if (g.Cb) g.Cb[row * g.ldcb + col] = f2bf(d);
          if (g.Cf) g.Cf[row * g.ldcf + col] = d;
        }
      }
    }
}

// ------------------------------------------------- forward-layer GEMM
// Operand tiles are streamed into LDS by direct global->LDS loads
// (global_load_lds_dwordx4: lane i's 16 bytes land at M0 + 16 i), so no
// registers stage them.  A tile row holds 32 K values (64 bytes, four 16-byte
// chunks); chunk c of row r is stored at position c ^ swz(r).  A fragment
// read has rows r..r+15 (r a multiple of 16) read one chunk each; the
// swizzle puts any 8 consecutive of those lanes on distinct 4-byte banks of
// a 32-bank window, and all 16 on distinct banks of a 64-bank one (row r
// starts at bank 16 r: rows of equal parity within an octet, and rows equal
// mod 4 within the 16, get distinct positions), whichever way the LDS splits
// a 16-byte read into phases.  It depends on r mod 16 only.
__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ ((r >> 3) & 1)) & 3; }

// One direct load of 16 bytes per lane: wave-uniform 64-bit base in SGPRs, a
// 32-bit per-lane byte offset, destination M0 = lds_addr (wave-uniform).
// (M0 is listed as clobbered; the compiler sets it before each of its own uses.)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void lds_dma16s(const void *sbase, unsigned voff, unsigned lds_addr) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
               :
               : "v"(voff), "s"(sbase), "s"(lds_addr)
               : "memory", "m0");
}
#pragma clang diagnostic pop

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

// Forward-layer GEMM with 16x16 output tiles (v_mfma_f32_16x16x32_bf16, one
// MFMA K-step per 32-wide stage), so the feature tile can be any multiple of
// 16: BN = TN16 16 (e.g. 400 = 800 / 2), BM = WM TM16 16 cells, waves split
// the cells.  Large tiles cut the bytes each block streams from L2 per flop
// (BM BN / (BM + BN) flops per byte).  The K-steps stream through a ring of
// STAGES LDS buffers: two are in flight while the waves multiply the third.
// Each wave waits for its own loads of a stage (vmcnt) and a workgroup
// barrier publishes all of them; rows past M or N are clamped to the last
// valid row (their results are never stored).  K must be a multiple of 32.
// Fragment: lane l holds row l % 16 and the 8 K values 8 (l / 16) ..; result:
// lane l holds cell l % 16 and features 4 (l / 16) .. + 3 of its tile.
template <int WM, int TM16, int TN16, int EPI, int STAGES>
__global__ __launch_bounds__(WM * 64) void k_gemm_dma16(GemmArgs g) {
  constexpr int BK = 32;
  constexpr int BM = WM * TM16 * 16, BN = TN16 * 16, ROWS = BM + BN;
  constexpr int NI = ROWS / 16;
  constexpr int NPW = (NI + WM - 1) / WM;
  constexpr int NMIN = NI / WM;
  static_assert(BM % 16 == 0 && BN % 16 == 0, "tile rows must be multiples of 16");
  static_assert(STAGES == 1 || STAGES == 2 || STAGES == 3,
                "ring of 2 or 3 stages, or 1 for a single K-step");
  __shared__ __attribute__((aligned(1024))) u16 S[STAGES * ROWS * BK];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ntn = (g.N + BN - 1) / BN;
  const int ntm = (g.M + BM - 1) / BM;
  const int total = ntn * ntm;
  const int per_xcd = (total + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (logical >= total) return;
  const long m0 = (long)(logical / ntn) * BM, n0 = (long)(logical % ntn) * BN;
  // the tile's bias in LDS (published by the barrier below) so that the
  // epilogue does not wait on global loads per feature tile
  __shared__ __attribute__((aligned(16))) float bias_s[BN];
  for (int c = tid; c < BN / 4; c += WM * 64) {
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (g.bias && n0 + 4 * c < g.N) v = *(const float4 *)(g.bias + n0 + 4 * c);
    *(float4 *)&bias_s[4 * c] = v;
  }
  __syncthreads();

  // per-lane byte offsets of this wave's DMA rows within the tile (rows past
  // M or N clamped to the last valid one) and the wave-uniform tile bases;
  // a K-blocked operand keeps the tile's rows of one K-step contiguous
  const bool ta = g.tiled & TILED_A, tb = g.tiled & TILED_B;
  const u16 *const sA = g.A + m0 * (ta ? BK : g.lda);
  const u16 *const sB = g.B + n0 * (tb ? BK : g.ldb);
  const long kA = ta ? g.lda : BK, kB = tb ? g.ldb : BK;  // step between K-blocks
  unsigned voff[NPW];
#pragma unroll
  for (int i = 0; i < NPW; ++i) {
    const int gi = i * WM + wave;
    const int row = gi * 16 + (lane >> 2);
    const int chunk = (lane & 3) ^ swz(row);
    unsigned o = 0;
    if (gi < NI) {
      if (row < BM) {
        const long m = m0 + row < g.M ? m0 + row : g.M - 1;
        o = (unsigned)(((m - m0) * (ta ? BK : g.lda) + chunk * 8) * 2);
      } else {
        const long n = n0 + (row - BM) < g.N ? n0 + (row - BM) : g.N - 1;
        o = (unsigned)(((n - n0) * (tb ? BK : g.ldb) + chunk * 8) * 2);
      }
    }
    voff[i] = o;
  }
  const unsigned lds0 =
      (unsigned)(uintptr_t)(__attribute__((address_space(3))) u16 *)(S);
  auto issue = [&](int stage, int kt) {
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int gi = i * WM + wave;
      if (gi < NI)
        lds_dma16s(gi * 16 < BM ? sA + kt * kA : sB + kt * kB, voff[i],
                   lds0 + (unsigned)((stage * ROWS + gi * 16) * BK * 2));
    }
  };

  f32x4 acc[TM16][TN16];
#pragma unroll
  for (int i = 0; i < TM16; ++i)
#pragma unroll
    for (int j = 0; j < TN16; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};

  const int nk = g.K / BK;
  const int cc = lane >> 4;
  // STAGES - 1 K-steps in flight ahead of the one being multiplied (a single
  // stage serves layers with one K-step only; two stages leave the CU room
  // for a second block, whose work covers this one's waits)
  issue(0, 0);
  if (STAGES == 3 && nk > 1) issue(1, 1);
  for (int kt = 0; kt < nk; ++kt) {
    // this wave's loads of stage kt are done once at most the next stage's
    // (NMIN or more instructions) remain; the barrier publishes every wave's
    if (STAGES == 3 && kt + 1 < nk)
      asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" : : "n"(NMIN) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" : : : "memory");
    // STAGES = 3: the ring slot of stage kt + 2 was last read in iteration
    // kt - 1, which every wave finished before the barrier above
    if (STAGES == 3 && kt + 2 < nk) issue((kt + 2) % STAGES, kt + 2);
    // STAGES = 2: the slot of stage kt + 1 was last read in iteration kt - 1
    if (STAGES == 2 && kt + 1 < nk) issue((kt + 1) % STAGES, kt + 1);
    const u16 *T = S + (kt % STAGES) * ROWS * BK;
    bf16x8 x[TM16];
#pragma unroll
    for (int i = 0; i < TM16; ++i) {
      const int row = wave * TM16 * 16 + i * 16 + (lane & 15);
      x[i] = *(const bf16x8 *)&T[row * BK + ((cc ^ swz(row)) * 8)];
    }
#pragma unroll
    for (int j = 0; j < TN16; ++j) {
      const int row = BM + j * 16 + (lane & 15);
      const bf16x8 w = *(const bf16x8 *)&T[row * BK + ((cc ^ swz(row)) * 8)];
#pragma unroll
      for (int i = 0; i < TM16; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x[i], acc[i][j], 0, 0, 0);
    }
  }

  const int hf = 4 * (lane >> 4);
  if constexpr (EPI == EPI_GELU_NEXT) {
    // The block holds every feature of its cells (one N-tile, BN >= N): the
    // GELU activations, rounded to BF16, are in the 16x16 C layout (lane l:
    // cell l % 16, features 4 (l / 16) .. + 3 of tile j), which is exactly the
    // B operand of v_mfma_f32_16x16x16_bf16 over the K-slice of tile j.  The
    // output layer's weights [N2 = 32][BN] are staged in the (now idle) ring
    // with rows padded by 4 elements (conflict-free 8-byte fragment reads).
    constexpr int LW = BN + 4;
    static_assert(BN % 16 == 0, "");
    asm volatile("s_barrier" : : : "memory");  // every wave is done with the ring
    u16 *Wl = S;
    for (int c = tid; c < g.N2 * (BN / 4); c += WM * 64) {
      const int r = c / (BN / 4), q = (c % (BN / 4)) * 4;
      uint2 v = make_uint2(0, 0);
      if (q < g.N) v = *(const uint2 *)(g.B2 + (long)r * g.N + q);
      *(uint2 *)&Wl[r * LW + q] = v;
    }
    __syncthreads();
    // one feature tile at a time: its activations feed both 16-wide output
    // tiles and its accumulators die (keeps the register peak at the main
    // loop's)
    constexpr int TO = 2;  // output tiles (N2 = 32)
    f32x4 u[TO][TM16];
#pragma unroll
    for (int o = 0; o < TO; ++o)
#pragma unroll
      for (int i = 0; i < TM16; ++i) u[o][i] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < TN16; ++j) {
      const float4 b = *(const float4 *)&bias_s[j * 16 + hf];
      s16x4 w[TO];
#pragma unroll
      for (int o = 0; o < TO; ++o)
        w[o] = *(const s16x4 *)&Wl[(o * 16 + (lane & 15)) * LW + j * 16 + hf];
#pragma unroll
      for (int i = 0; i < TM16; ++i) {
        const bf16x2 lo = __builtin_convertvector(
            (f32x2){gelu(acc[i][j][0] + b.x), gelu(acc[i][j][1] + b.y)}, bf16x2);
        const bf16x2 hi = __builtin_convertvector(
            (f32x2){gelu(acc[i][j][2] + b.z), gelu(acc[i][j][3] + b.w)}, bf16x2);
        const unsigned ul = __builtin_bit_cast(unsigned, lo), uh = __builtin_bit_cast(unsigned, hi);
        const s16x4 h = (s16x4){(short)(ul & 0xffff), (short)(ul >> 16), (short)(uh & 0xffff),
                                (short)(uh >> 16)};
#pragma unroll
        for (int o = 0; o < TO; ++o)
          u[o][i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[o], h, u[o][i], 0, 0, 0);
      }
    }
#pragma unroll
    for (int o = 0; o < TO; ++o) {
      const float4 b2 = *(const float4 *)(g.bias2 + o * 16 + hf);
#pragma unroll
      for (int i = 0; i < TM16; ++i) {
        const long row = m0 + wave * TM16 * 16 + i * 16 + (lane & 15);
        if (row < g.M)
          *(float4 *)(g.Cf + row * g.ldcf + o * 16 + hf) =
              make_float4(u[o][i][0] + b2.x, u[o][i][1] + b2.y, u[o][i][2] + b2.z,
                          u[o][i][3] + b2.w);
      }
    }
    return;
  }
  // per-lane row bases (the lane's cell and first feature) and wave-uniform
  // offsets of each 16-feature tile
  const bool tc = g.tiled & TILED_C;
  long rb[TM16];
  bool live[TM16];
#pragma unroll
  for (int i = 0; i < TM16; ++i) {
    const long row = m0 + wave * TM16 * 16 + i * 16 + (lane & 15);
    live[i] = row < g.M;
    rb[i] = row;
  }
#pragma unroll
  for (int j = 0; j < TN16; ++j) {
    const long cj = n0 + j * 16;  // uniform
    if (cj >= g.N) break;
    const float4 b = *(const float4 *)&bias_s[j * 16 + hf];
#pragma unroll
    for (int i = 0; i < TM16; ++i) {
      if (!live[i]) continue;
      const long row = rb[i];
      const float4 v = make_float4(acc[i][j][0] + b.x, acc[i][j][1] + b.y, acc[i][j][2] + b.z,
                                   acc[i][j][3] + b.w);
      if (EPI == EPI_F32) {
        *(float4 *)(g.Cf + row * g.ldcf + hf + cj) = v;
      } else if (EPI == EPI_GELU) {
        if (g.Z) *(float4 *)(g.Z + row * g.ldz + hf + cj) = v;
        const float4 h = make_float4(gelu(v.x), gelu(v.y), gelu(v.z), gelu(v.w));
        if (g.Cb) {
          const bf16x2 lo = __builtin_convertvector((f32x2){h.x, h.y}, bf16x2);
          const bf16x2 hi = __builtin_convertvector((f32x2){h.z, h.w}, bf16x2);
          uint2 o;
          o.x = __builtin_bit_cast(unsigned, lo);
          o.y = __builtin_bit_cast(unsigned, hi);
          u16 *const at = tc ? g.Cb + (row * 32 + hf) + ((cj / 32) * g.ldcb + cj % 32)
                             : g.Cb + (row * g.ldcb + hf) + cj;
          *(uint2 *)at = o;
        }
        if (g.Cf) *(float4 *)(g.Cf + row * g.ldcf + hf + cj) = h;
      } else if (EPI == EPI_GELU_Q8) {
        uint8_t *const at = tc ? g.Cq + (row * 128 + hf) + ((cj / 128) * g.ldcq + cj % 128)
                               : g.Cq + (row * g.ldcq + hf) + cj;
        *(unsigned *)at = e4m3x4(gelu(v.x) * g.qinv, gelu(v.y) * g.qinv, gelu(v.z) * g.qinv,
                                 gelu(v.w) * g.qinv);
      }
    }
  }
}

template <int WM, int TM16, int TN16, int STAGES = 3>
chem_status gemm_dma16_cfg(const GemmArgs &g, int epi, hipStream_t s) {
  constexpr int BM = WM * TM16 * 16, BN = TN16 * 16;
  if (STAGES == 1 && g.K != 32) {
    chem::set_error("gemm: the single-stage tiling needs K = 32");
    return CHEM_EUNSUPPORTED;
  }
  const long total = (long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid((unsigned)(((total + 7) / 8) * 8));
  dim3 block(WM * 64);
  if (epi == EPI_GELU)
    hipLaunchKernelGGL((k_gemm_dma16<WM, TM16, TN16, EPI_GELU, STAGES>), grid, block, 0, s, g);
  else if (epi == EPI_F32)
    hipLaunchKernelGGL((k_gemm_dma16<WM, TM16, TN16, EPI_F32, STAGES>), grid, block, 0, s, g);
  else if (epi == EPI_GELU_Q8)
    hipLaunchKernelGGL((k_gemm_dma16<WM, TM16, TN16, EPI_GELU_Q8, STAGES>), grid, block, 0, s,
                       g);
  else if (epi == EPI_GELU_NEXT && g.N <= BN && g.N2 == 32 &&
           g.N2 * (BN + 4) <= STAGES * (BM + BN) * 32 && g.ldcf % 4 == 0)
    hipLaunchKernelGGL((k_gemm_dma16<WM, TM16, TN16, EPI_GELU_NEXT, STAGES>), grid, block, 0, s,
                       g);
  else {
    chem::set_error("gemm: unsupported epilogue for K-contiguous operands");
    return CHEM_EUNSUPPORTED;
  }
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

// ------------------------------------------- fused first two layers
// H[cell][n] = GELU(b2 + sum_k W2[n][k] GELU(b1[k] + W1[k] . x[cell])) in one
// kernel: each 32-feature K-step of the second layer is produced in
// registers by the first layer (K = 32: one v_mfma_f32_16x16x32_bf16 per
// 16 features x 16 cells, the bias as its C input) from the block's inputs,
// so the 1600-wide first activation is neither written nor read back.  The
// first layer's result leaves lane l with cell l % 16 and features 4g..4g+3
// and 16+4g..16+4g+3 (g = l / 16) of the K-step; the second layer's MFMA
// takes K positions 8g..8g+7 from lane group g, so the step's features enter
// in that permuted order and the second layer's weights are stored with the
// same permutation within each 32-wide K-block (mlp12_slot).  The tile is
// the second layer's 256 cells x 400 features: the block's two feature
// tiles each recompute the first layer for their cells (8 % more MFMA work,
// twice the GELUs of the first layer).  The ring stage of K-step kt carries
// the second layer's weights of step kt and the first layer's of step kt + 1,
// whose GELUs then overlap the multiplications of step kt.
constexpr int MLP12_KMAX = 2048;
// waves per block and 16-cell tiles per wave (block: MLP12_WM MLP12_TM16 16
// cells x 400 features)
constexpr int MLP12_WM = 8, MLP12_TM16 = 2;
// second-layer weight fragments in flight ahead of their MFMAs
constexpr int MLP12_PF = 2;
// k_mlp12p: the first tile, and the spacing in tiles, of the first layer's
// GELUs among the second layer's MFMAs (8 GELUs over 25 tiles)
constexpr int MLP12P_GSTART = 2, MLP12P_GSTEP = 3;
constexpr int PHASE = 4;

template <int TN16>
struct Mlp12Tile {
  static constexpr int WM = MLP12_WM, TM16 = MLP12_TM16, BK = 32, STAGES = 3;
  static constexpr int BM = WM * TM16 * 16, BN = TN16 * 16;
  static constexpr int R1 = 32;  // first-layer weight rows of one K-step
  static constexpr int ROWS = R1 + BN;
};

// One block's tile; MULFIRST: this wave multiplies before it produces (the
// whole body is instantiated per order, so that no accumulator crosses a
// branch).
template <int TN16, bool MULFIRST>
__device__ __forceinline__ void mlp12_tile(const Mlp12Args &g, u16 *S, float *b1_s,
                                           float *bias_s, int wave) {
  using TL = Mlp12Tile<TN16>;
  constexpr int WM = TL::WM, TM16 = TL::TM16, BK = TL::BK, STAGES = TL::STAGES;
  constexpr int BM = TL::BM, BN = TL::BN, R1 = TL::R1, ROWS = TL::ROWS;
  constexpr int NI = ROWS / 16;
  constexpr int NPW = (NI + WM - 1) / WM;
  constexpr int NMIN = NI / WM;
  const int tid = threadIdx.x, lane = tid & 63;
  const int ntn = (g.N + BN - 1) / BN;
  const int ntm = (g.M + BM - 1) / BM;
  const int total = ntn * ntm;
  const int per_xcd = (total + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (logical >= total) return;
  const long m0 = (long)(logical / ntn) * BM, n0 = (long)(logical % ntn) * BN;
  for (int c = tid; c < BN / 4; c += WM * 64) {
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (n0 + 4 * c < g.N) v = *(const float4 *)(g.b2 + n0 + 4 * c);
    *(float4 *)&bias_s[4 * c] = v;
  }
  for (int c = tid; c < g.K / 4; c += WM * 64) *(float4 *)&b1_s[4 * c] = *(const float4 *)(g.b1 + 4 * c);

  // the wave's 32 cells as the first layer's B operand (lane: cell l % 16 of
  // tile i, inputs 8g..8g+7); rows past M clamped (never stored)
  const int cc = lane >> 4, hf = 4 * cc;
  bf16x8 xin[TM16];
#pragma unroll
  for (int i = 0; i < TM16; ++i) {
    long row = m0 + wave * TM16 * 16 + i * 16 + (lane & 15);
    if (row >= g.M) row = g.M - 1;
    xin[i] = *(const bf16x8 *)(g.X + row * 32 + cc * 8);
  }
  __syncthreads();  // b1_s, bias_s

  // first layer for the 32 features of K-step kt: w1[t] = weight rows
  // 16t + l % 16 of the step (the MFMA's A operand)
  auto layer1 = [&](const bf16x8(&w1)[2], int kt, bf16x8(&h)[TM16]) __attribute__((always_inline)) {
    const float4 c0 = *(const float4 *)&b1_s[kt * 32 + hf];
    const float4 c1 = *(const float4 *)&b1_s[kt * 32 + 16 + hf];
#pragma unroll
    for (int i = 0; i < TM16; ++i) {
      f32x4 z0 = (f32x4){c0.x, c0.y, c0.z, c0.w}, z1 = (f32x4){c1.x, c1.y, c1.z, c1.w};
      z0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[0], xin[i], z0, 0, 0, 0);
      z1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[1], xin[i], z1, 0, 0, 0);
      const bf16x2 a = __builtin_convertvector((f32x2){gelu(z0[0]), gelu(z0[1])}, bf16x2);
      const bf16x2 b = __builtin_convertvector((f32x2){gelu(z0[2]), gelu(z0[3])}, bf16x2);
      const bf16x2 c = __builtin_convertvector((f32x2){gelu(z1[0]), gelu(z1[1])}, bf16x2);
      const bf16x2 d = __builtin_convertvector((f32x2){gelu(z1[2]), gelu(z1[3])}, bf16x2);
      h[i] = (bf16x8){a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]};
    }
  };

  // K-step 0 of the first layer straight from global memory
  const int nk = g.K / BK;
  bf16x8 h[TM16];
  {
    bf16x8 w1[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
      w1[t] = *(const bf16x8 *)(g.W1 + (t * 16 + (lane & 15)) * 32 + cc * 8);
    layer1(w1, 0, h);
  }

  // DMA rows: the first R1 rows of a stage are the first layer's weights of
  // the next K-step, then BN rows of the second layer's (all valid: N is a
  // multiple of BN).  A 16-row group starts at a multiple of 16, so the
  // swizzle of row 16 gi + l / 4 is swz(l / 4) for every group: one
  // per-lane byte offset serves all of them, the rest is wave-uniform.
  const u16 *const sB = g.W2p + n0 * BK;
  const unsigned loff =
      (unsigned)((lane >> 2) * BK * 2 + (((lane & 3) ^ swz(lane >> 2)) * 16));
  const unsigned lds0 =
      (unsigned)(uintptr_t)(__attribute__((address_space(3))) u16 *)(S);
  auto issue = [&](int stage, int kt) __attribute__((always_inline)) {
    const int k1 = kt + 1 < nk ? kt + 1 : nk - 1;
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int gi = i * WM + wave;
      if (gi < NI)
        lds_dma16s(gi * 16 < R1 ? g.W1 + ((long)k1 * R1 + gi * 16) * BK
                                : sB + kt * g.ldw2 + (long)(gi * 16 - R1) * BK,
                   loff, lds0 + (unsigned)((stage * ROWS + gi * 16) * BK * 2));
    }
  };

  f32x4 acc[TM16][TN16];
#pragma unroll
  for (int i = 0; i < TM16; ++i)
#pragma unroll
    for (int j = 0; j < TN16; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};

  issue(0, 0);
  if (nk > 1) issue(1, 1);
  for (int kt = 0; kt < nk; ++kt) {
    // as in k_gemm_dma16: own loads of stage kt done, barrier publishes all
    if (kt + 1 < nk)
      asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" : : "n"(NMIN) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" : : : "memory");
    if (kt + 2 < nk) issue((kt + 2) % STAGES, kt + 2);
    const u16 *T = S + (kt % STAGES) * ROWS * BK;
    // the next K-step's first-layer features (the last step recomputes its
    // own, unused): VALU-heavy
    bf16x8 hn[TM16];
    auto produce = [&]() __attribute__((always_inline)) {
      bf16x8 w1[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int row = t * 16 + (lane & 15);
        w1[t] = *(const bf16x8 *)&T[row * BK + ((cc ^ swz(row)) * 8)];
      }
      layer1(w1, kt + 1 < nk ? kt + 1 : kt, hn);
    };
    // this K-step of the second layer: MFMA-heavy; the weight fragments are
    // read MLP12_PF feature tiles ahead of their MFMAs
    auto bfrag = [&](int j) __attribute__((always_inline)) {
      const int row = R1 + j * 16 + (lane & 15);
      return *(const bf16x8 *)&T[row * BK + ((cc ^ swz(row)) * 8)];
    };
    auto multiply = [&]() __attribute__((always_inline)) {
      bf16x8 wq[MLP12_PF];
#pragma unroll
      for (int q = 0; q < MLP12_PF; ++q) wq[q] = bfrag(q);
#pragma unroll
      for (int j = 0; j < TN16; ++j) {
        const bf16x8 w = wq[j % MLP12_PF];
        if (j + MLP12_PF < TN16) wq[j % MLP12_PF] = bfrag(j + MLP12_PF);
#pragma unroll
        for (int i = 0; i < TM16; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, h[i], acc[i][j], 0, 0, 0);
      }
    };
    if (MULFIRST) {
      multiply();
      produce();
    } else {
      produce();
      multiply();
    }
#pragma unroll
    for (int i = 0; i < TM16; ++i) h[i] = hn[i];
  }

  // epilogue: bias + GELU, BF16 (lane: 4 consecutive features of one cell)
  long rb[TM16];
  bool live[TM16];
#pragma unroll
  for (int i = 0; i < TM16; ++i) {
    rb[i] = m0 + wave * TM16 * 16 + i * 16 + (lane & 15);
    live[i] = rb[i] < g.M;
  }
#pragma unroll
  for (int j = 0; j < TN16; ++j) {
    const long cj = n0 + j * 16;  // uniform
    if (cj >= g.N) break;
    const float4 b = *(const float4 *)&bias_s[j * 16 + hf];
#pragma unroll
    for (int i = 0; i < TM16; ++i) {
      if (!live[i]) continue;
      const long row = rb[i];
      const bf16x2 lo = __builtin_convertvector(
          (f32x2){gelu(acc[i][j][0] + b.x), gelu(acc[i][j][1] + b.y)}, bf16x2);
      const bf16x2 hi = __builtin_convertvector(
          (f32x2){gelu(acc[i][j][2] + b.z), gelu(acc[i][j][3] + b.w)}, bf16x2);
      uint2 o;
      o.x = __builtin_bit_cast(unsigned, lo);
      o.y = __builtin_bit_cast(unsigned, hi);
      u16 *const at = g.tiled ? g.H + (row * 32 + hf) + ((cj / 32) * g.ldh + cj % 32)
                              : g.H + (row * g.ldh + hf) + cj;
      *(uint2 *)at = o;
    }
  }
}

// waves (wave & PHASE) != 0 multiply before they produce: one wave's GELUs
// can then overlap the other's MFMAs on the same SIMD
template <int TN16>
__global__ __launch_bounds__(MLP12_WM * 64) void k_mlp12(Mlp12Args g) {
  using TL = Mlp12Tile<TN16>;
  __shared__ __attribute__((aligned(1024))) u16 S[TL::STAGES * TL::ROWS * TL::BK];
  __shared__ __attribute__((aligned(16))) float b1_s[MLP12_KMAX];
  __shared__ __attribute__((aligned(16))) float bias_s[TL::BN];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wave & PHASE)
    mlp12_tile<TN16, true>(g, S, b1_s, bias_s, wave);
  else
    mlp12_tile<TN16, false>(g, S, b1_s, bias_s, wave);
}

// ------------------------------------ fused first two layers, paired halves
// The same computation as k_mlp12 on a 128-cell x 800-feature tile: wave w
// takes cells 32 (w & 3) .. + 31 and second-layer features 400 (w >> 2) ..
// + 399, so the two waves of a SIMD (w and w + 4) share their cells.  Each
// produces one of the two 16-feature halves of the next K-step's first layer
// (one MFMA and eight GELUs per cell tile instead of two and sixteen: the
// first layer is computed once per cell, not once per 400 features) and
// leaves it in LDS (8 bytes per lane and tile); after the step's barrier the
// partner's half completes the MFMA operand, in the order k_mlp12 builds it.
// Within a K-step the first layer's GELUs sit between the second layer's
// MFMAs of the same wave.  The 832-row stage (the first layer's 32 rows, the second's 800) allows a
// ring of two, so each K-step prefetches only the next one.
template <int TN16>
struct Mlp12PTile {
  static constexpr int WM = 8, TM16 = 2, BK = 32, STAGES = 2, RW = 4;
  static constexpr int BM = RW * TM16 * 16, BNH = TN16 * 16, BN = 2 * BNH;
  static constexpr int R1 = 32;
  static constexpr int ROWS = R1 + BN;
  // exchange buffer: [2 steps][RW][TM16][2 halves][64 lanes] of 8 bytes
  static constexpr int XB = 2 * RW * TM16 * 2 * 64;
};

// CW: the wave's feature half (waves 4..7: 1)
template <int TN16, int CW>
__device__ __forceinline__ void mlp12p_tile(const Mlp12Args &g, u16 *S, float *b1_s,
                                            float *bias_s, uint2 *xb, int wave) {
  constexpr int cw = CW;
  using TL = Mlp12PTile<TN16>;
  constexpr int WM = TL::WM, TM16 = TL::TM16, BK = TL::BK, STAGES = TL::STAGES;
  constexpr int BM = TL::BM, BNH = TL::BNH, BN = TL::BN, R1 = TL::R1, ROWS = TL::ROWS;
  constexpr int NI = ROWS / 16;
  constexpr int NPW = (NI + WM - 1) / WM;
  const int tid = threadIdx.x, lane = tid & 63;
  const int rw = wave & 3;
  const int ntn = g.N / BN;
  const int ntm = (g.M + BM - 1) / BM;
  const int total = ntn * ntm;
  const int per_xcd = (total + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (logical >= total) return;  // uniform over the block: no barrier is skipped by part of it
  const long m0 = (long)(logical / ntn) * BM, n0 = (long)(logical % ntn) * BN;
  for (int c = tid; c < BN / 4; c += WM * 64)
    *(float4 *)&bias_s[4 * c] = *(const float4 *)(g.b2 + n0 + 4 * c);
  for (int c = tid; c < g.K / 4; c += WM * 64) *(float4 *)&b1_s[4 * c] = *(const float4 *)(g.b1 + 4 * c);

  // the wave's 32 cells as the first layer's B operand (rows past M clamped)
  const int cc = lane >> 4, hf = 4 * cc;
  bf16x8 xin[TM16];
#pragma unroll
  for (int i = 0; i < TM16; ++i) {
    long row = m0 + rw * TM16 * 16 + i * 16 + (lane & 15);
    if (row >= g.M) row = g.M - 1;
    xin[i] = *(const bf16x8 *)(g.X + row * 32 + cc * 8);
  }
  __syncthreads();  // b1_s, bias_s

  // this wave's half (features 16 cw .. 16 cw + 15) of K-step kt's first
  // layer: lane l gets features 16 cw + 4 (l / 16) .. + 3 of cell l % 16
  auto layer1h = [&](const bf16x8 &w1, int kt, uint2(&hh)[TM16]) __attribute__((always_inline)) {
    const float4 c = *(const float4 *)&b1_s[kt * 32 + 16 * cw + hf];
#pragma unroll
    for (int i = 0; i < TM16; ++i) {
      f32x4 z = (f32x4){c.x, c.y, c.z, c.w};
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, xin[i], z, 0, 0, 0);
      const bf16x2 a = __builtin_convertvector((f32x2){gelu(z[0]), gelu(z[1])}, bf16x2);
      const bf16x2 b = __builtin_convertvector((f32x2){gelu(z[2]), gelu(z[3])}, bf16x2);
      hh[i] = make_uint2(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b));
    }
  };
  // slot of (step parity, tile i, half) for this wave's cells
  auto xslot = [&](int par, int i, int half) __attribute__((always_inline)) {
    return xb + (((par * TL::RW + rw) * TM16 + i) * 2 + half) * 64 + lane;
  };

  // K-step 0 of the first layer straight from global memory
  const int nk = g.K / BK;
  uint2 hh[TM16];
  {
    const bf16x8 w1 = *(const bf16x8 *)(g.W1 + (16 * cw + (lane & 15)) * 32 + cc * 8);
    layer1h(w1, 0, hh);
#pragma unroll
    for (int i = 0; i < TM16; ++i) *xslot(0, i, cw) = hh[i];
  }

  // DMA rows as in k_mlp12: the first R1 rows of a stage are the first
  // layer's weights of the next K-step, then the BN rows of the second's
  const u16 *const sB = g.W2p + n0 * BK;
  const unsigned loff =
      (unsigned)((lane >> 2) * BK * 2 + (((lane & 3) ^ swz(lane >> 2)) * 16));
  const unsigned lds0 =
      (unsigned)(uintptr_t)(__attribute__((address_space(3))) u16 *)(S);
  auto issue = [&](int stage, int kt) __attribute__((always_inline)) {
    const int k1 = kt + 1 < nk ? kt + 1 : nk - 1;
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int gi = i * WM + wave;
      if (gi < NI)
        lds_dma16s(gi * 16 < R1 ? g.W1 + ((long)k1 * R1 + gi * 16) * BK
                                : sB + kt * g.ldw2 + (long)(gi * 16 - R1) * BK,
                   loff, lds0 + (unsigned)((stage * ROWS + gi * 16) * BK * 2));
    }
  };

  f32x4 acc[TM16][TN16];
#pragma unroll
  for (int i = 0; i < TM16; ++i)
#pragma unroll
    for (int j = 0; j < TN16; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};

  issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    // this wave's loads of stage kt and its half of step kt's first layer
    // done; the barrier publishes every wave's
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" : : : "memory");
    if (kt + 1 < nk) issue((kt + 1) % STAGES, kt + 1);
    const u16 *T = S + (kt % STAGES) * ROWS * BK;
    // step kt's operand: the z0 half (features 4g..) then the z1 half (16 + 4g..)
    bf16x8 h[TM16];
#pragma unroll
    for (int i = 0; i < TM16; ++i) {
      const uint2 o = *xslot(kt & 1, i, cw ^ 1);
      const uint2 lo = CW == 0 ? hh[i] : o, hi = CW == 0 ? o : hh[i];
      const unsigned v[4] = {lo.x, lo.y, hi.x, hi.y};
      h[i] = __builtin_bit_cast(bf16x8, v);
    }
    uint2 hn[TM16];
    // step kt + 1's first-layer products go first; their eight GELUs are
    // then spread between the second layer's MFMAs of step kt, one every
    // MLP12P_GSTEP feature tiles from tile MLP12P_GSTART, each tile fenced
    // off from the scheduler so that the VALU work stays between the MFMAs
    f32x4 z[TM16];
    {
      const int row = 16 * cw + (lane & 15);
      const bf16x8 w1 = *(const bf16x8 *)&T[row * BK + ((cc ^ swz(row)) * 8)];
      const int k1 = kt + 1 < nk ? kt + 1 : kt;
      const float4 c = *(const float4 *)&b1_s[k1 * 32 + 16 * cw + hf];
#pragma unroll
      for (int i = 0; i < TM16; ++i) {
        z[i] = (f32x4){c.x, c.y, c.z, c.w};
        z[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, xin[i], z[i], 0, 0, 0);
      }
    }
    auto bfrag = [&](int j) __attribute__((always_inline)) {
      const int row = R1 + cw * BNH + j * 16 + (lane & 15);
      return *(const bf16x8 *)&T[row * BK + ((cc ^ swz(row)) * 8)];
    };
    {
      static_assert(MLP12P_GSTART + (TM16 * 4 - 1) * MLP12P_GSTEP < TN16,
                    "each first-layer GELU needs a feature tile of its own");
      float gz[TM16 * 4];
      bf16x8 wq[MLP12_PF];
#pragma unroll
      for (int q = 0; q < MLP12_PF; ++q) wq[q] = bfrag(q);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < TN16; ++j) {
        const bf16x8 w = wq[j % MLP12_PF];
        if (j + MLP12_PF < TN16) wq[j % MLP12_PF] = bfrag(j + MLP12_PF);
#pragma unroll
        for (int i = 0; i < TM16; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, h[i], acc[i][j], 0, 0, 0);
        if (j >= MLP12P_GSTART && (j - MLP12P_GSTART) % MLP12P_GSTEP == 0 &&
            (j - MLP12P_GSTART) / MLP12P_GSTEP < TM16 * 4) {
          const int q = (j - MLP12P_GSTART) / MLP12P_GSTEP;
          gz[q] = gelu(z[q / 4][q % 4]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int i = 0; i < TM16; ++i) {
        const bf16x2 lo = __builtin_convertvector((f32x2){gz[4 * i], gz[4 * i + 1]}, bf16x2);
        const bf16x2 hi = __builtin_convertvector((f32x2){gz[4 * i + 2], gz[4 * i + 3]}, bf16x2);
        hn[i] = make_uint2(__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi));
      }
    }
#pragma unroll
    for (int i = 0; i < TM16; ++i) *xslot((kt + 1) & 1, i, cw) = hn[i];
#pragma unroll
    for (int i = 0; i < TM16; ++i) hh[i] = hn[i];
  }

  // epilogue: bias + GELU, BF16 (lane: 4 consecutive features of one cell)
  long rb[TM16];
  bool live[TM16];
#pragma unroll
  for (int i = 0; i < TM16; ++i) {
    rb[i] = m0 + rw * TM16 * 16 + i * 16 + (lane & 15);
    live[i] = rb[i] < g.M;
  }
#pragma unroll
  for (int j = 0; j < TN16; ++j) {
    const long cj = n0 + cw * BNH + j * 16;  // uniform
    const float4 b = *(const float4 *)&bias_s[cw * BNH + j * 16 + hf];
#pragma unroll
    for (int i = 0; i < TM16; ++i) {
      if (!live[i]) continue;
      const long row = rb[i];
      const bf16x2 lo = __builtin_convertvector(
          (f32x2){gelu(acc[i][j][0] + b.x), gelu(acc[i][j][1] + b.y)}, bf16x2);
      const bf16x2 hi = __builtin_convertvector(
          (f32x2){gelu(acc[i][j][2] + b.z), gelu(acc[i][j][3] + b.w)}, bf16x2);
      uint2 o;
      o.x = __builtin_bit_cast(unsigned, lo);
      o.y = __builtin_bit_cast(unsigned, hi);
      u16 *const at = g.tiled ? g.H + (row * 32 + hf) + ((cj / 32) * g.ldh + cj % 32)
                              : g.H + (row * g.ldh + hf) + cj;
      *(uint2 *)at = o;
    }
  }
}

template <int TN16>
__global__ __launch_bounds__(8 * 64) void k_mlp12p(Mlp12Args g) {
  using TL = Mlp12PTile<TN16>;
  __shared__ __attribute__((aligned(1024))) u16 S[TL::STAGES * TL::ROWS * TL::BK];
  __shared__ __attribute__((aligned(16))) float b1_s[MLP12_KMAX];
  __shared__ __attribute__((aligned(16))) float bias_s[TL::BN];
  __shared__ __attribute__((aligned(16))) uint2 xb[TL::XB];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wave & PHASE)
    mlp12p_tile<TN16, 1>(g, S, b1_s, bias_s, xb, wave);
  else
    mlp12p_tile<TN16, 0>(g, S, b1_s, bias_s, xb, wave);
}

template <int WM, int WN, int TM, int TN, int BK>
chem_status gemm_launch(const GemmArgs &g, bool AK, bool BKC, int epi, dim3 grid, dim3 block,
                        hipStream_t s) {
  if (AK && BKC && epi == EPI_GELU)
    hipLaunchKernelGGL((k_gemm<WM, WN, TM, TN, true, true, EPI_GELU, BK>), grid, block, 0, s, g);
  else if (AK && BKC && epi == EPI_F32)
    hipLaunchKernelGGL((k_gemm<WM, WN, TM, TN, true, true, EPI_F32, BK>), grid, block, 0, s, g);
  else if (AK && BKC && epi == EPI_GELU_Q8)
    hipLaunchKernelGGL((k_gemm<WM, WN, TM, TN, true, true, EPI_GELU_Q8, BK>), grid, block, 0, s,
                       g);
  else if (AK && !BKC && epi == EPI_GELUGRAD)
    hipLaunchKernelGGL((k_gemm<WM, WN, TM, TN, true, false, EPI_GELUGRAD, BK>), grid, block, 0,
                       s, g);
  else if (!AK && !BKC && epi == EPI_F32)
    hipLaunchKernelGGL((k_gemm<WM, WN, TM, TN, false, false, EPI_F32, BK>), grid, block, 0, s,
                       g);
  else {
    chem::set_error("gemm: unsupported layout/epilogue combination");
    return CHEM_EUNSUPPORTED;
  }
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

template <int WM, int WN, int TM, int TN>
chem_status gemm_cfg(const GemmArgs &g, bool AK, bool BKC, int epi, hipStream_t s) {
  constexpr int BM = WM * TM * 32, BN = WN * TN * 32;
  const long total = (long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid((unsigned)(((total + 7) / 8) * 8), g.ksplit > 1 ? g.ksplit : 1,
            g.groups > 1 ? g.groups : 1);
  dim3 block(WM * WN * 64);
  // 64-wide K-steps for launches of up to 1024 blocks (the training batch);
  // larger grids keep the smaller LDS footprint and more blocks per CU
  // (unless the autotuner chose)
  const int kper = g.ksplit > 1 ? g.K / g.ksplit : g.K;
  const bool bk64 = g.bk ? (g.bk == 64 && kper >= 64)
                         : (kper >= 64 && (long)grid.x * grid.y * grid.z <= 1024);
  if (bk64) return gemm_launch<WM, WN, TM, TN, 64>(g, AK, BKC, epi, grid, block, s);
  return gemm_launch<WM, WN, TM, TN, 32>(g, AK, BKC, epi, grid, block, s);
}

// The generic tilings the autotuner chooses from: 128 x 128, 128 x 32,
// 64 x 64 and 128 x 64 blocks of C (waves x 32 x 32 MFMA tiles per wave).
chem_status gemm_tiled(const GemmArgs &g, bool AK, bool BKC, int epi, hipStream_t s) {
  switch (g.tile) {
    case 1: return gemm_cfg<2, 2, 2, 2>(g, AK, BKC, epi, s);
    case 2: return gemm_cfg<4, 1, 1, 1>(g, AK, BKC, epi, s);
    case 3: return gemm_cfg<2, 2, 1, 1>(g, AK, BKC, epi, s);
    case 4: return gemm_cfg<4, 2, 1, 1>(g, AK, BKC, epi, s);
    default: break;
  }
  if (g.N <= 32) return gemm_cfg<4, 1, 1, 1>(g, AK, BKC, epi, s);
  return gemm_cfg<2, 2, 2, 2>(g, AK, BKC, epi, s);
}

// ------------------------------------------------------------ FP8 GEMM
// E4M3 operands with v_mfma_scale_f32_32x32x64_f8f6f4 (block scales fixed at
// 2^0), FP32 accumulation; the per-tensor scales multiply the accumulator in
// the epilogue.  K-step 64; same tiling, staging and XCD-aware block order as
// the BF16 kernel.  Fragment layout: lane l holds row l % 32 and the 32
// consecutive k values 32 (l / 32) .. 32 (l / 32) + 31.
typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int WM, int WN, int TM, int TN, int EPI>
__global__ __launch_bounds__(WM *WN * 64) void k_gemm8(GemmArgs g) {
  constexpr int BM = WM * TM * 32, BN = WN * TN * 32, BK = 64, LK = BK + 16;
  constexpr int NT = WM * WN * 64;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][BM * LK];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][BN * LK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int ntn = (g.N + BN - 1) / BN;
  const int ntm = (g.M + BM - 1) / BM;
  const int total = ntn * ntm;
  const int per_xcd = (total + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (logical >= total) return;
  const long m0 = (long)(logical / ntn) * BM, n0 = (long)(logical % ntn) * BN;
  constexpr int ACH = BM * BK / 16, BCH = BN * BK / 16;
  constexpr int APT = (ACH + NT - 1) / NT, BPT = (BCH + NT - 1) / NT;
  uint4 ra[APT], rb[BPT];
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      const int c = tid + i * NT;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (c < ACH) {
        const int r = c / (BK / 16), kc = (c % (BK / 16)) * 16;
        if (m0 + r < g.M) v = *(const uint4 *)(g.A8 + (m0 + r) * g.lda + k0 + kc);
      }
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int c = tid + i * NT;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (c < BCH) {
        const int r = c / (BK / 16), kc = (c % (BK / 16)) * 16;
        if (n0 + r < g.N) v = *(const uint4 *)(g.B8 + (n0 + r) * g.ldb + k0 + kc);
      }
      rb[i] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      const int c = tid + i * NT;
      if (c < ACH) {
        const int r = c / (BK / 16), kc = (c % (BK / 16)) * 16;
        *(uint4 *)&As[buf][r * LK + kc] = ra[i];
      }
    }
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int c = tid + i * NT;
      if (c < BCH) {
        const int r = c / (BK / 16), kc = (c % (BK / 16)) * 16;
        *(uint4 *)&Bs[buf][r * LK + kc] = rb[i];
      }
    }
  };
  auto compute = [&](int buf) {
    i32x8 a[TM], b[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
      a[i] = *(const i32x8 *)&As[buf][(wm * TM * 32 + i * 32 + (lane & 31)) * LK +
                                      32 * (lane >> 5)];
#pragma unroll
    for (int j = 0; j < TN; ++j)
      b[j] = *(const i32x8 *)&Bs[buf][(wn * TN * 32 + j * 32 + (lane & 31)) * LK +
                                      32 * (lane >> 5)];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i], b[j], acc[i][j], 0, 0,
                                                                     0, 127, 0, 127);
  };
  const int nk = g.K / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
    compute(cur);
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const long col = n0 + wn * TN * 32 + j * 32 + (lane & 31);
      if (col >= g.N) continue;
      const float bias = g.bias ? g.bias[col] : 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long row = m0 + wm * TM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row >= g.M) continue;
        const float h = gelu(acc[i][j][r] * g.scale + bias);
        if (EPI == EPI_GELU_Q8) g.Cq[row * g.ldcq + col] = f2e4m3(h * g.qinv);
        else g.Cb[row * g.ldcb + col] = f2bf(h);
      }
    }
}

// E4M3 x E4M3 forward GEMM on the direct-to-LDS ring: 16x16 output tiles with
// v_mfma_scale_f32_16x16x128_f8f6f4 (block scales 2^0), one MFMA K-step per
// 128-byte stage row.  A DMA instruction covers 8 rows of 128 bytes; chunk c
// of row r sits at c ^ swz8(r), which keeps the 16-lane phases of the
// fragment reads (rows r..r+15, one chunk each) on distinct banks.  K must be
// a multiple of 128 (operands zero-padded by the caller).  Fragment: lane l
// holds row l % 16 and the 32 K bytes 32 (l / 16) ..; the per-tensor scales
// multiply the accumulator in the epilogue.
__device__ __forceinline__ int swz8(int r) { return (r >> 1) & 7; }

template <int WM, int TM16, int TN16, int EPI, int STAGES = 3>
__global__ __launch_bounds__(WM * 64) void k_gemm8_dma16(GemmArgs g) {
  constexpr int BK = 128;
  static_assert(STAGES == 2 || STAGES == 3, "ring of 3 stages, or 2 for the widest tiles");
  constexpr int BM = WM * TM16 * 16, BN = TN16 * 16, ROWS = BM + BN;
  constexpr int NI = ROWS / 8;
  constexpr int NPW = (NI + WM - 1) / WM;
  constexpr int NMIN = NI / WM;
  static_assert(BM % 16 == 0 && BN % 16 == 0, "tile rows must be multiples of 16");
  __shared__ __attribute__((aligned(1024))) uint8_t S[STAGES * ROWS * BK];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ntn = (g.N + BN - 1) / BN;
  const int ntm = (g.M + BM - 1) / BM;
  const int total = ntn * ntm;
  const int per_xcd = (total + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (logical >= total) return;
  const long m0 = (long)(logical / ntn) * BM, n0 = (long)(logical % ntn) * BN;
  __shared__ __attribute__((aligned(16))) float bias_s[BN];  // as in k_gemm_dma16
  for (int c = tid; c < BN / 4; c += WM * 64) {
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (g.bias && n0 + 4 * c < g.N) v = *(const float4 *)(g.bias + n0 + 4 * c);
    *(float4 *)&bias_s[4 * c] = v;
  }
  __syncthreads();

  const bool ta = g.tiled & TILED_A, tb = g.tiled & TILED_B;
  const uint8_t *const sA = g.A8 + m0 * (ta ? BK : g.lda);
  const uint8_t *const sB = g.B8 + n0 * (tb ? BK : g.ldb);
  const long kA = ta ? g.lda : BK, kB = tb ? g.ldb : BK;  // step between K-blocks
  unsigned voff[NPW];
#pragma unroll
  for (int i = 0; i < NPW; ++i) {
    const int gi = i * WM + wave;
    const int row = gi * 8 + (lane >> 3);
    const int chunk = (lane & 7) ^ swz8(row);
    unsigned o = 0;
    if (gi < NI) {
      if (row < BM) {
        const long m = m0 + row < g.M ? m0 + row : g.M - 1;
        o = (unsigned)((m - m0) * (ta ? BK : g.lda) + chunk * 16);
      } else {
        const long n = n0 + (row - BM) < g.N ? n0 + (row - BM) : g.N - 1;
        o = (unsigned)((n - n0) * (tb ? BK : g.ldb) + chunk * 16);
      }
    }
    voff[i] = o;
  }
  const unsigned lds0 =
      (unsigned)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)(S);
  auto issue = [&](int stage, int kt) {
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int gi = i * WM + wave;
      if (gi < NI)
        lds_dma16s(gi * 8 < BM ? sA + kt * kA : sB + kt * kB, voff[i],
                   lds0 + (unsigned)((stage * ROWS + gi * 8) * BK));
    }
  };

  f32x4 acc[TM16][TN16];
#pragma unroll
  for (int i = 0; i < TM16; ++i)
#pragma unroll
    for (int j = 0; j < TN16; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};

  const int nk = g.K / BK;
  const int c0 = 2 * (lane >> 4);
  auto frag = [&](const uint8_t *T, int row) {
    const uint4 lo = *(const uint4 *)&T[row * BK + ((c0 ^ swz8(row)) * 16)];
    const uint4 hi = *(const uint4 *)&T[row * BK + (((c0 + 1) ^ swz8(row)) * 16)];
    return (i32x8){(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                   (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
  };
  issue(0, 0);
  if (STAGES == 3 && nk > 1) issue(1, 1);
  for (int kt = 0; kt < nk; ++kt) {
    // 3 stages: as in k_gemm_dma16.  2 stages: the only loads in flight are
    // stage kt's; after the barrier the other stage (read in step kt - 1)
    // takes step kt + 1.
    if (STAGES == 3 && kt + 1 < nk)
      asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" : : "n"(NMIN) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" : : : "memory");
    if (STAGES == 3 && kt + 2 < nk) issue((kt + 2) % STAGES, kt + 2);
    if (STAGES == 2 && kt + 1 < nk) issue((kt + 1) % STAGES, kt + 1);
    const uint8_t *T = S + (kt % STAGES) * ROWS * BK;
    i32x8 x[TM16];
#pragma unroll
    for (int i = 0; i < TM16; ++i) x[i] = frag(T, wave * TM16 * 16 + i * 16 + (lane & 15));
#pragma unroll
    for (int j = 0; j < TN16; ++j) {
      const i32x8 w = frag(T, BM + j * 16 + (lane & 15));
#pragma unroll
      for (int i = 0; i < TM16; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(w, x[i], acc[i][j], 0, 0,
                                                                      0, 127, 0, 127);
    }
  }

  const int hf = 4 * (lane >> 4);
  if constexpr (EPI == EPI_GELU_NEXT) {
    // the output layer in the epilogue, as in k_gemm_dma16: the block holds
    // all BN >= N features of its cells; W2 [N2 = 32][N] BF16 staged in the
    // idle ring (rows padded by 4 elements)
    constexpr int LW = BN + 4;
    asm volatile("s_barrier" : : : "memory");  // every wave is done with the ring
    u16 *const Wl = (u16 *)S;
    for (int c = tid; c < g.N2 * (BN / 4); c += WM * 64) {
      const int r = c / (BN / 4), q = (c % (BN / 4)) * 4;
      uint2 v = make_uint2(0, 0);
      if (q < g.N) v = *(const uint2 *)(g.B2 + (long)r * g.N + q);
      *(uint2 *)&Wl[r * LW + q] = v;
    }
    __syncthreads();
    constexpr int TO = 2;  // output tiles (N2 = 32)
    f32x4 u[TO][TM16];
#pragma unroll
    for (int o = 0; o < TO; ++o)
#pragma unroll
      for (int i = 0; i < TM16; ++i) u[o][i] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < TN16; ++j) {
      const float4 b = *(const float4 *)&bias_s[j * 16 + hf];
      s16x4 w[TO];
#pragma unroll
      for (int o = 0; o < TO; ++o)
        w[o] = *(const s16x4 *)&Wl[(o * 16 + (lane & 15)) * LW + j * 16 + hf];
#pragma unroll
      for (int i = 0; i < TM16; ++i) {
        const bf16x2 lo = __builtin_convertvector(
            (f32x2){gelu(acc[i][j][0] * g.scale + b.x), gelu(acc[i][j][1] * g.scale + b.y)},
            bf16x2);
        const bf16x2 hi = __builtin_convertvector(
            (f32x2){gelu(acc[i][j][2] * g.scale + b.z), gelu(acc[i][j][3] * g.scale + b.w)},
            bf16x2);
        const unsigned ul = __builtin_bit_cast(unsigned, lo), uh = __builtin_bit_cast(unsigned, hi);
        const s16x4 h = (s16x4){(short)(ul & 0xffff), (short)(ul >> 16), (short)(uh & 0xffff),
                                (short)(uh >> 16)};
#pragma unroll
        for (int o = 0; o < TO; ++o)
          u[o][i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[o], h, u[o][i], 0, 0, 0);
      }
    }
#pragma unroll
    for (int o = 0; o < TO; ++o) {
      const float4 b2 = *(const float4 *)(g.bias2 + o * 16 + hf);
#pragma unroll
      for (int i = 0; i < TM16; ++i) {
        const long row = m0 + wave * TM16 * 16 + i * 16 + (lane & 15);
        if (row < g.M)
          *(float4 *)(g.Cf + row * g.ldcf + o * 16 + hf) =
              make_float4(u[o][i][0] + b2.x, u[o][i][1] + b2.y, u[o][i][2] + b2.z,
                          u[o][i][3] + b2.w);
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < TN16; ++j) {
    if (n0 + j * 16 >= g.N) break;
    const long col = n0 + j * 16 + hf;
    const float4 b = *(const float4 *)&bias_s[j * 16 + hf];
#pragma unroll
    for (int i = 0; i < TM16; ++i) {
      const long row = m0 + wave * TM16 * 16 + i * 16 + (lane & 15);
      if (row >= g.M) continue;
      const float4 h = make_float4(gelu(acc[i][j][0] * g.scale + b.x),
                                   gelu(acc[i][j][1] * g.scale + b.y),
                                   gelu(acc[i][j][2] * g.scale + b.z),
                                   gelu(acc[i][j][3] * g.scale + b.w));
      if (EPI == EPI_GELU_Q8) {
        const long at = (g.tiled & TILED_C) ? (col / 128) * g.ldcq + row * 128 + col % 128
                                            : row * g.ldcq + col;
        *(unsigned *)(g.Cq + at) = e4m3x4(h.x * g.qinv, h.y * g.qinv, h.z * g.qinv, h.w * g.qinv);
      } else {
        const bf16x2 lo = __builtin_convertvector((f32x2){h.x, h.y}, bf16x2);
        const bf16x2 hi = __builtin_convertvector((f32x2){h.z, h.w}, bf16x2);
        uint2 o;
        o.x = __builtin_bit_cast(unsigned, lo);
        o.y = __builtin_bit_cast(unsigned, hi);
        *(uint2 *)(g.Cb + row * g.ldcb + col) = o;
      }
    }
  }
}

template <int WM, int TM16, int TN16, int STAGES = 3>
chem_status gemm8_dma16_cfg(const GemmArgs &g, int epi, hipStream_t s) {
  constexpr int BM = WM * TM16 * 16, BN = TN16 * 16;
  const long total = (long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid((unsigned)(((total + 7) / 8) * 8)), block(WM * 64);
  if (epi == EPI_GELU_Q8)
    hipLaunchKernelGGL((k_gemm8_dma16<WM, TM16, TN16, EPI_GELU_Q8, STAGES>), grid, block, 0, s,
                       g);
  else if (epi == EPI_GELU)
    hipLaunchKernelGGL((k_gemm8_dma16<WM, TM16, TN16, EPI_GELU, STAGES>), grid, block, 0, s, g);
  else if (epi == EPI_GELU_NEXT && g.N <= BN && g.N2 == 32 &&
           g.N2 * (BN + 4) * 2 <= STAGES * (BM + BN) * 128 && g.ldcf % 4 == 0)
    hipLaunchKernelGGL((k_gemm8_dma16<WM, TM16, TN16, EPI_GELU_NEXT, STAGES>), grid, block, 0, s,
                       g);
  else {
    chem::set_error("gemm8: unsupported epilogue");
    return CHEM_EUNSUPPORTED;
  }
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

__global__ void k_amax(int64_t n, const void *x, int bf16, float *part) {
  __shared__ float red[256];
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = bf16 ? __uint_as_float((unsigned)((const u16 *)x)[i] << 16)
                         : ((const float *)x)[i];
    m = fmaxf(m, fabsf(v));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_quant(const float *src, long ld_src, int rows, int cols, uint8_t *dst,
                        int rows_p, int cols_p, float qinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows_p * cols_p) return;
  const int r = (int)(i / cols_p), c = (int)(i % cols_p);
  dst[i] = (r < rows && c < cols) ? f2e4m3(src[(int64_t)r * ld_src + c] * qinv) : (uint8_t)0;
}

// ------------------------------------------------------------- prologue

// Box-Cox with the hardware base-2 logarithm and exponential (y <= 0, and
// y below the FP32 normal range, give y^lambda = 0).
__device__ __forceinline__ float boxcox_fast(float y, float lam) {
  const float yl = y > 0.0f ? __builtin_amdgcn_exp2f(lam * __builtin_amdgcn_logf(y)) : 0.0f;
  return (yl - 1.0f) / lam;
}

// One thread per cell: raw features (T, p, Box-Cox of Y), the optional
// out-of-distribution bit, z-scored BF16 row of X.  DINP > 0 fixes the padded
// width at compile time, so all of a cell's loads are issued before the first
// one is used, and the block's rows are staged in LDS (rows padded by one
// 16-byte chunk: conflict-free) and stored as consecutive 16-byte chunks per
// lane, whole 128-byte lines per store (a lane writing its own row left every
// line a quarter full per store and doubled the bytes written).
// BLK cells per block: 256 for large batches, 64 for small ones (a training
// batch of 8192 cells fills 128 blocks instead of 32).
template <int DINP, int BLK>
__global__ __launch_bounds__(BLK) void k_features(FeatArgs a) {
  constexpr int CH = DINP > 0 ? DINP / 8 : 1;  // 16-byte chunks per row
  __shared__ uint4 stage[DINP > 0 ? BLK * (CH + 1) : 1];
  const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
  const bool live = i < a.n;
  if (DINP == 0 && !live) return;
  const int dinp = DINP > 0 ? DINP : a.dinp;
  if (live) {
    const int64_t c = a.index ? a.index[i] : i;
    u16 *out = a.X + i * dinp;
    bool outside = false;
    constexpr int UNROLL = DINP > 0 ? DINP / 8 : 1;
#pragma unroll UNROLL
    for (int j0 = 0; j0 < (DINP > 0 ? DINP : 1 << 30); j0 += 8) {
      if (DINP == 0 && j0 >= dinp) break;
      float z[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int j = j0 + t;
        z[t] = 0.0f;
        if (j < a.K + 2) {
          float x;
          if (j == 0) x = (float)a.T[c];
          else if (j == 1) x = (float)a.p[c];
          else x = boxcox_fast((float)a.Y[(int64_t)(j - 2) * a.ld + c], a.lambda);
          if (a.ood) {
            const float lo = a.lo[j], hi = a.hi[j], span = hi - lo;
            const float tol =
                span > 0.0f ? a.ood_margin * span : 1e-6f * fmaxf(fabsf(hi), 1e-30f);
            if (!(x >= lo - tol && x <= hi + tol)) outside = true;
          }
          z[t] = (x - a.mu[j]) / a.sd[j];
        }
      }
      uint4 o;
      o.x = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){z[0], z[1]}, bf16x2));
      o.y = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){z[2], z[3]}, bf16x2));
      o.z = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){z[4], z[5]}, bf16x2));
      o.w = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){z[6], z[7]}, bf16x2));
      if (DINP > 0)
        stage[threadIdx.x * (CH + 1) + j0 / 8] = o;
      else
        *(uint4 *)(out + j0) = o;
    }
    if (a.ood) a.ood[i] = outside ? 1 : 0;
  }
  if (DINP > 0) {
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * BLK;
    const int rows = a.n - r0 < BLK ? (int)(a.n - r0) : BLK;
    uint4 *const dst = (uint4 *)(a.X + r0 * DINP);
    for (int f = threadIdx.x; f < rows * CH; f += BLK)
      dst[f] = stage[(f / CH) * (CH + 1) + f % CH];
  }
}

// One cell per thread.  The loads of a batch of TGT_BATCH outputs are all
// issued before the first store (the output rows may not alias the inputs, but
// the compiler cannot know that), and a padded width that is a multiple of 4
// is written with 16-byte stores.
constexpr int TGT_BATCH = 16;

__global__ void k_targets(TargetArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t c = a.index ? a.index[i] : i;
  float *out = a.U + i * a.doutp;
  const bool vec = (a.doutp & 3) == 0 && ((uintptr_t)a.U & 15) == 0;
  for (int k0 = 0; k0 < a.doutp; k0 += TGT_BATCH) {
    double y1[TGT_BATCH], y0[TGT_BATCH];
#pragma unroll
    for (int j = 0; j < TGT_BATCH; ++j) {
      const int k = k0 + j;
      y1[j] = k < a.K ? a.Y1[(int64_t)k * a.ld + c] : 0.0;
      y0[j] = k < a.K ? a.Y0[(int64_t)k * a.ld + c] : 0.0;
    }
    float v[TGT_BATCH];
#pragma unroll
    for (int j = 0; j < TGT_BATCH; ++j) {
      const int k = k0 + j;
      // the change of the mass fraction over the step (FP64 difference)
      v[j] = k < a.K ? (float)((y1[j] - y0[j] - a.mu[k]) / a.sd[k]) : 0.0f;
    }
    if (vec && k0 + TGT_BATCH <= a.doutp) {
#pragma unroll
      for (int j = 0; j < TGT_BATCH; j += 4)
        *(float4 *)(out + k0 + j) = make_float4(v[j], v[j + 1], v[j + 2], v[j + 3]);
    } else {
      for (int j = 0; j < TGT_BATCH && k0 + j < a.doutp; ++j) out[k0 + j] = v[j];
    }
  }
}

// ------------------------------------------------------------ training

// g = sign(u - u*) / (n K) (sign(0) = 0) on the K real outputs, 0 on padding;
// per-block partial sums of |u - u*| for the loss.
__global__ void k_l1(int64_t n, int K, int doutp, const float *U, const float *Ut, u16 *Gb,
                     float *Gf, double *part) {
  __shared__ double red[256];
  const double scale = 1.0 / ((double)n * K);
  double s = 0.0;
  const int64_t total = n * doutp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e % doutp);
    float gv = 0.0f;
    if (k < K) {
      const float d = U[e] - Ut[e];
      s += fabs((double)d);
      gv = (float)(((d > 0.0f) - (d < 0.0f)) * scale);
    }
    Gb[e] = f2bf(gv);
    Gf[e] = gv;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Per-species ensemble: member g's single output is column 0 of its [n][ldu]
// block; g = sign(u - u*) / (n G) there, 0 on the padding columns.
__global__ void k_l1_members(int64_t n, int G, int ldu, long gu, const float *U, const float *Ut,
                             int ldt, u16 *Gb, float *Gf, double *part) {
  __shared__ double red[256];
  const double scale = 1.0 / ((double)n * G);
  double s = 0.0;
  const int64_t per = n * ldu, total = per * G;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = e / per, r = (e % per) / ldu;
    const int c = (int)(e % ldu);
    const int64_t at = g * gu + r * ldu + c;
    float gv = 0.0f;
    if (c == 0) {
      const float d = U[at] - Ut[r * ldt + g];
      s += fabs((double)d);
      gv = (float)(((d > 0.0f) - (d < 0.0f)) * scale);
    }
    Gb[at] = f2bf(gv);
    Gf[at] = gv;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_take_col(int64_t n, const float *src, int lds, float *dst, int ldd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i * ldd] = src[i * lds];
}

// Weight of species k in the element projection: the expected variance of
// the network's error in its change, sd^2 (sd = the target's standard
// deviation), tapered to zero as the species' own mass fraction vanishes:
// sd^2 (Y+ + 1e-10) / (Y+ + sd), Y+ = max(Y', 0).
__device__ __forceinline__ double proj_weight(double y, float sdf) {
  const double yp = fmax(y, 0.0), sd = (double)sdf;
  return sd * sd * (yp + 1e-10) / (yp + sd);
}

// h_k(T) in J/kg from the folded h/RT polynomial of species k's range at T.
__device__ __forceinline__ double species_h(const chem::DevMech &M, int k, double T) {
  const double *c = (T <= M.Tmid[k] ? M.nasa_h : M.nasa_hh) + 7 * k;
  const double hRT = c[0] + T * (c[1] + T * (c[2] + T * (c[3] + T * c[4]))) + c[5] / T;
  return 8.314462618 * T * hRT * M.invW[k];
}

// One sample per thread.  With dY = sd u + mu the predicted change and
// e = (u - u*) sd its error (FP64 from the FP32 u), each term is an L1
// penalty |s_t| / D_t on a linear functional s_t: the sum of dY (weights 1),
// sum_k h_k(T1) e_k and sum_k h_k(298.15 K) e_k; D_t = sum_k |a_tk| sd_k is
// the functional's size for errors of one standard deviation.  d/du_k of
// w_t |s_t| / (D_t n) is w_t sign(s_t) a_tk sd_k / (D_t n).
__global__ void k_phys(PhysArgs a, chem::DevMech M, double *part) {
  __shared__ double red[3][256];
  constexpr double TREF = 298.15;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = a.index ? a.index[i] : i;
    const double T1 = a.T1 ? a.T1[c] : TREF;
    const float *u = a.U + i * a.doutp, *ut = a.Ut + i * a.doutp;
    double sm = 0.0, se = 0.0, sh = 0.0, dm = 0.0, de = 0.0, dh = 0.0;
    for (int k = 0; k < a.K; ++k) {
      const double sd = a.sd[k], mu = a.mu[k];
      const double dY = sd * (double)u[k] + mu;
      const double e = ((double)u[k] - (double)ut[k]) * sd;
      const double h1 = species_h(M, k, T1), h0 = species_h(M, k, TREF);
      sm += dY;
      dm += sd;
      se += h1 * e;
      de += fabs(h1) * sd;
      sh += h0 * e;
      dh += fabs(h0) * sd;
    }
    acc[0] += fabs(sm) / dm;
    acc[1] += fabs(se) / de;
    acc[2] += fabs(sh) / dh;
    const double inv_n = 1.0 / (double)a.n;
    const double gm = a.w[0] * ((sm > 0.0) - (sm < 0.0)) / dm * inv_n;
    const double ge = a.w[1] * ((se > 0.0) - (se < 0.0)) / de * inv_n;
    const double gh = a.w[2] * ((sh > 0.0) - (sh < 0.0)) / dh * inv_n;
    float *gf = a.Gf + i * a.doutp;
    u16 *gb = a.Gb + i * a.doutp;
    for (int k = 0; k < a.K; ++k) {
      const double sd = a.sd[k];
      const double g = (gm + ge * species_h(M, k, T1) + gh * species_h(M, k, TREF)) * sd;
      const float v = gf[k] + (float)g;
      gf[k] = v;
      gb[k] = f2bf(v);
    }
  }
  for (int t = 0; t < 3; ++t) red[t][threadIdx.x] = acc[t];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int t = 0; t < 3; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// Batch means of the three terms (partials added in block order); the
// weighted sum joins the L1 loss.
__global__ void k_phys_final(const double *part, int nparts, double inv_n, float w0, float w1,
                             float w2, float *loss, float *terms) {
  if (threadIdx.x != 0) return;
  double t[3] = {0.0, 0.0, 0.0};
  for (int b = 0; b < nparts; ++b)
    for (int q = 0; q < 3; ++q) t[q] += part[b * 3 + q];
  for (int q = 0; q < 3; ++q) t[q] *= inv_n;
  if (terms)
    for (int q = 0; q < 3; ++q) terms[q] = (float)t[q];
  *loss = (float)((double)*loss + w0 * t[0] + w1 * t[1] + w2 * t[2]);
}

__global__ void k_loss_final(const double *part, int nparts, double scale, float *loss) {
  if (threadIdx.x != 0) return;
  // partials added in order, loaded eight at a time
  double s = 0.0;
  int i = 0;
  for (; i + 8 <= nparts; i += 8) {
    double x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = part[i + r];
#pragma unroll
    for (int r = 0; r < 8; ++r) s += x[r];
  }
  for (; i < nparts; ++i) s += part[i];
  *loss = (float)(s * scale);
}

// Column sums in two fixed-order passes (FP64 accumulation): block row q
// sums rows [q M / P, (q + 1) M / P) of its columns into part[q][j]; the final
// pass adds the P partials in order of q.
// Both passes issue COLSUM_BATCH loads before adding them, in order, to the
// running sum (the same order as one load at a time).
constexpr int COLSUM_BATCH = 16;

__global__ void k_colsum_part(int64_t M, int N, const float *X, long ldx, double *part,
                              long gx) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  X += (long)blockIdx.z * gx;                       // member of a grouped sum
  part += (long)blockIdx.z * gridDim.y * (long)N;
  const int P = gridDim.y, q = blockIdx.y;
  const int64_t m0 = M * q / P, m1 = M * (q + 1) / P;
  double s = 0.0;
  int64_t m = m0;
  for (; m + COLSUM_BATCH <= m1; m += COLSUM_BATCH) {
    float x[COLSUM_BATCH];
#pragma unroll
    for (int r = 0; r < COLSUM_BATCH; ++r) x[r] = X[(m + r) * ldx + j];
#pragma unroll
    for (int r = 0; r < COLSUM_BATCH; ++r) s += x[r];
  }
  for (; m < m1; ++m) s += X[m * ldx + j];
  part[(int64_t)q * N + j] = s;
}

__global__ void k_colsum_fin(int N, int P, const double *part, float *out, long gout) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  part += (long)blockIdx.z * P * (long)N;
  out += (long)blockIdx.z * gout;
  double s = 0.0;
  int q = 0;
  for (; q + COLSUM_BATCH <= P; q += COLSUM_BATCH) {
    double x[COLSUM_BATCH];
#pragma unroll
    for (int r = 0; r < COLSUM_BATCH; ++r) x[r] = part[(int64_t)(q + r) * N + j];
#pragma unroll
    for (int r = 0; r < COLSUM_BATCH; ++r) s += x[r];
  }
  for (; q < P; ++q) s += part[(int64_t)q * N + j];
  out[j] = (float)s;
}

__global__ void k_sum_splits(int64_t n, int S, const float *part, long stride, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = part[i];
  for (int q = 1; q < S; ++q) s += part[(int64_t)q * stride + i];
  out[i] = s;
}

__device__ __forceinline__ void adam_elem(int64_t i, float *W, const float *g, float *m, float *v,
                                          u16 *Wb, float lr, float b1, float b2, float eps,
                                          float bc1, float bc2) {
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = W[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  W[i] = w;
  if (Wb) Wb[i] = f2bf(w);
}

// Adam over up to ADAM_MAX tensors in one launch (a training step's weights
// and biases): element i of the concatenation belongs to the last tensor
// whose start is <= i.
__global__ void k_adam_multi(AdamTable t, float lr, float b1, float b2, float eps, float bc1,
                             float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.start[t.count]) return;
  int k = 0;
#pragma unroll
  for (int q = 1; q < ADAM_MAX; ++q)
    if (q < t.count && i >= t.start[q]) k = q;
  adam_elem(i - t.start[k], t.W[k], t.g[k], t.m[k], t.v[k], t.Wb[k], lr, b1, b2, eps, bc1, bc2);
}

__global__ void k_to_bf16(int64_t n, const float *src, u16 *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = f2bf(src[i]);
}

// K-blocked copy: element (r, k) of src [R][K] (KB-element blocks) to
// dst[(k / KB) R KB + r KB + k % KB]; one thread per element.
template <typename T, int KB, bool PERM = false>
__global__ void k_tile(int R, int K, const T *src, T *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)R * K) return;
  const int r = (int)(i / K), k = (int)(i % K);
  const int kk = PERM ? mlp12_slot(k % KB) : k % KB;
  dst[(int64_t)(k / KB) * R * KB + (int64_t)r * KB + kk] = src[i];
}

// ----------------------------------------------------------------- post

// c_p/R and h/RT of species k at T (Tp = T, T^2, T^3, T^4, 1/T): both
// ranges' coefficients are wave-uniform loads, the range is chosen per lane;
// h/RT uses the coefficients with the divisors folded in.
__device__ __forceinline__ void species_h_cp(const chem::DevMech &M, int k, const double *Tp,
                                             double &hRT, double &cpR) {
  const bool low = Tp[0] <= M.Tmid[k];
  double c[5], h[6];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double a = M.nasa_lo[7 * k + q], b = M.nasa_hi[7 * k + q];
    c[q] = low ? a : b;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double a = M.nasa_h[7 * k + q], b = M.nasa_hh[7 * k + q];
    h[q] = low ? a : b;
  }
  cpR = c[0] + c[1] * Tp[0] + c[2] * Tp[1] + c[3] * Tp[2] + c[4] * Tp[3];
  hRT = h[0] + h[1] * Tp[0] + h[2] * Tp[1] + h[3] * Tp[2] + h[4] * Tp[3] + h[5] * Tp[4];
}

__device__ __forceinline__ void tpowers(double T, double *Tp) {
  Tp[0] = T;
  Tp[1] = T * T;
  Tp[2] = Tp[1] * T;
  Tp[3] = Tp[2] * T;
  Tp[4] = 1.0 / T;
}

constexpr int EMAX = 8;

// One thread per cell.  One streaming pass over the species builds Y' =
// Y0 + dY (kept in registers, KP >= K slots), the element sums of Y0 and of
// Y0 - Y', the weighted normal matrix and h(T0, Y0); Y0 itself is not kept (it
// is read again for RR).  Four waves per SIMD (a few spilled registers) beat
// two spill-free ones: the kernel is latency-bound (FP64 Cholesky and Newton
// chains per cell).
template <int KP, int EP>
__global__ __launch_bounds__(128, 4) void k_post(chem::DevMech M, PostArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int K = M.K, E = M.E;
  const double T0 = a.T[i], p = a.p[i];
  uint8_t flag = (uint8_t)a.force_flag;
  // out of distribution: any input feature outside the widened training range
  // (tested by k_features on the same cells)
  if (a.ood && a.ood[i]) flag |= 1;
  double yn[KP];
  double A[EP][EP], r[EP], z0[EP];
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    r[e] = 0.0;
    z0[e] = 0.0;
#pragma unroll
    for (int f = 0; f < EP; ++f) A[e][f] = 0.0;
  }
  double S0 = 0.0, h0 = 0.0, Tp[5];
  tpowers(T0, Tp);
  const bool vec = a.doutp % 4 == 0;
  // Species in chunks of CH: the chunk's Y0 and U loads are issued together
  // (indices past the last species are clamped into range and their values
  // unused), ahead of the per-species branches that would otherwise hold
  // each load back until the previous species is done.  All of a cell's U
  // (one row of doutp floats) is then read while its lines are in cache.
  constexpr int CH = 8;
#pragma unroll
  for (int k0 = 0; k0 < KP; k0 += CH) {
    double y0c[CH];
    float uc[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) y0c[t] = a.Y[(int64_t)min(k0 + t, K - 1) * a.ld + i];
    if (vec) {
#pragma unroll
      for (int q = 0; q < CH; q += 4) {
        const float4 v = *(const float4 *)(a.U + i * a.doutp + min(k0 + q, a.doutp - 4));
        uc[q] = v.x;
        uc[q + 1] = v.y;
        uc[q + 2] = v.z;
        uc[q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int t = 0; t < CH; ++t) uc[t] = a.U[i * a.doutp + min(k0 + t, K - 1)];
    }
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int k = k0 + t;
      yn[k] = 0.0;
      if (k < K) {
        const double y0 = y0c[t];
        const float du = uc[t] * a.nm.sd_out[k] + a.nm.mu_out[k];
        const double y = y0 + (double)du;  // Y' = Y0 + sd u + mu
        yn[k] = y;
        const double d = proj_weight(y, a.nm.sd_out[k]);
        S0 += y0 * M.invW[k];
        double hRT, cpR;
        species_h_cp(M, k, Tp, hRT, cpR);
        h0 += y0 * RG * T0 * hRT * M.invW[k];
        // weighted least-squares projection onto M Y = M Y0, D = diag(proj_weight)
#pragma unroll
        for (int e = 0; e < EP; ++e) {
          if (e < E) {
            const double me = M.Mel[e * K + k];
            r[e] += me * (y0 - y);
            z0[e] += me * y0;
#pragma unroll
            for (int f = 0; f <= e; ++f) A[e][f] += me * d * M.Mel[f * K + k];
          }
        }
      }
    }
  }
  double Lc[EP][EP], lam[EP];
  bool ok = true;
#pragma unroll
  for (int e = 0; e < EP; ++e) {
#pragma unroll
    for (int f = 0; f <= e; ++f) {
      if (e < E) {
        double v = A[e][f];
#pragma unroll
        for (int q = 0; q < f; ++q) v -= Lc[e][q] * Lc[f][q];
        if (e == f) {
          if (!(v > 0.0)) ok = false;
          Lc[e][e] = sqrt(fmax(v, 1e-300));
        } else {
          Lc[e][f] = v / Lc[f][f];
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    lam[e] = 0.0;
    if (e < E) {
      double v = r[e];
#pragma unroll
      for (int q = 0; q < e; ++q) v -= Lc[e][q] * lam[q];
      lam[e] = v / Lc[e][e];
    }
  }
#pragma unroll
  for (int e = EP - 1; e >= 0; --e) {
    if (e < E) {
      double v = lam[e];
#pragma unroll
      for (int q = e + 1; q < EP; ++q)
        if (q < E) v -= Lc[q][e] * lam[q];
      lam[e] = v / Lc[e][e];
    }
  }
  // projected and clipped state, and its element residual
  double z1[EP];
#pragma unroll
  for (int e = 0; e < EP; ++e) z1[e] = 0.0;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (k < K) {
      double corr = 0.0;
#pragma unroll
      for (int e = 0; e < EP; ++e)
        if (e < E) corr += M.Mel[e * K + k] * lam[e];
      const double y = fmax(yn[k] + proj_weight(yn[k], a.nm.sd_out[k]) * corr, 0.0);
      yn[k] = y;
#pragma unroll
      for (int e = 0; e < EP; ++e)
        if (e < E) z1[e] += M.Mel[e * K + k] * y;
    }
  }
  // residuals: of the network's own state Y' (r = M Y0 - M Y', which the
  // projection removes), and of the projected, clipped state; either above
  // the tolerance (or non-finite) flags the cell
  const double rtol_e = (double)a.residual_tol;
  bool bad = !ok;
#pragma unroll
  for (int e = 0; e < EP; ++e)
    if (e < E) bad = bad || !(fabs(z1[e] - z0[e]) <= rtol_e) || !(fabs(r[e]) <= rtol_e);
  if (bad) flag |= 2;

  if (flag == 0) {
    // temperature from h(T, Y) = h(T0, Y0) by Newton in FP64.  h and c_p of
    // the mixture are linear in Y: with every species in the NASA range it
    // takes at a reference temperature, they are polynomials in T whose
    // coefficients are the Y / W-weighted sums of the species' (hm: h/RT
    // terms with the divisors folded in, cm: c_p/R terms), exact for
    // tlo < T <= thi; a Newton step then costs O(1), and the sums are built
    // again only if an iterate leaves that interval.
    double hm[6], cm[5], tlo = 0.0, thi = -1.0;
    auto mixture = [&](double Tr) __attribute__((always_inline)) {
#pragma unroll
      for (int q = 0; q < 6; ++q) hm[q] = 0.0;
#pragma unroll
      for (int q = 0; q < 5; ++q) cm[q] = 0.0;
      tlo = -INFINITY;
      thi = INFINITY;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        if (k < K) {
          const double w = yn[k] * M.invW[k];
          const double tm = M.Tmid[k];
          const bool low = Tr <= tm;
          thi = low ? fmin(thi, tm) : thi;
          tlo = low ? tlo : fmax(tlo, tm);
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const double lo = M.nasa_h[7 * k + q], hi = M.nasa_hh[7 * k + q];
            hm[q] += w * (low ? lo : hi);
          }
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            const double lo = M.nasa_lo[7 * k + q], hi = M.nasa_hi[7 * k + q];
            cm[q] += w * (low ? lo : hi);
          }
        }
      }
    };
    double T = T0;
    for (int it = 0; it < 20; ++it) {
      if (!(T > tlo && T <= thi)) mixture(T);
      tpowers(T, Tp);
      const double hRT = hm[0] + hm[1] * Tp[0] + hm[2] * Tp[1] + hm[3] * Tp[2] +
                         hm[4] * Tp[3] + hm[5] * Tp[4];
      const double cpR = cm[0] + cm[1] * Tp[0] + cm[2] * Tp[1] + cm[3] * Tp[2] + cm[4] * Tp[3];
      const double dT = (RG * T * hRT - h0) / (RG * cpR);
      T -= dT;
      if (!isfinite(T) || fabs(dT) < 1e-9 * T) break;
    }
    if (!isfinite(T) || !(T > 0.0)) flag |= 2;
    if (flag == 0) {
      const double rho0 = p / (RG * T0 * S0);
      const double sc = rho0 / a.dt;
      // Y0 is read again for the rates, eight species at a time before their
      // stores (a load placed after a store that may alias it waits for it)
      constexpr int WB = 8;
#pragma unroll
      for (int k0 = 0; k0 < KP; k0 += WB) {
        double y0[WB];
#pragma unroll
        for (int t = 0; t < WB; ++t)
          y0[t] = (a.RR && k0 + t < K) ? a.Y[(int64_t)(k0 + t) * a.ld + i] : 0.0;
#pragma unroll
        for (int t = 0; t < WB; ++t) {
          const int k = k0 + t;
          if (k < K) {
            if (a.RR) a.RR[(int64_t)k * a.ld + i] = sc * (yn[k] - y0[t]);
            a.Y[(int64_t)k * a.ld + i] = yn[k];
          }
        }
      }
      a.T[i] = T;
    }
  }
  if (flag != 0 && a.RR) {
#pragma unroll
    for (int k = 0; k < KP; ++k)
      if (k < K) a.RR[(int64_t)k * a.ld + i] = 0.0;
  }
  if (a.flags) a.flags[i] = flag;
  if (flag != 0) {
    const unsigned long long slot = atomicAdd(a.fb_count, 1ull);
    if (a.fb_index) a.fb_index[slot] = (int32_t)(a.index_base + i);
  }
}


// ------------------------------------------------------------- audit
// The integrator judging the network: the audited cells (every s-th of a
// chunk) are copied before the network runs, integrated by the plain step
// afterwards, and compared with what the network left in the caller's arrays.

__global__ void k_audit_init(double *audit, int K) {
  for (int q = threadIdx.x; q < 3 + 3 * K; q += blockDim.x) {
    const int r = q < 3 ? 0 : (q - 3) % 3;
    audit[q] = q < 3 ? 0.0 : (r == 0 ? 0.0 : (r == 1 ? INFINITY : -INFINITY));
  }
}

__global__ void k_audit_gather(AuditArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.na) return;
  const int64_t i = j * a.stride;
  a.Ta[j] = a.T[i];
  a.pa[j] = a.p[i];
  for (int k = 0; k < a.K; ++k) {
    const double y = a.Y[(int64_t)k * a.ld + i];
    a.Ya[(int64_t)k * a.na + j] = y;
    a.Y0a[(int64_t)k * a.na + j] = y;
  }
}

__device__ __forceinline__ void atomic_min_f64(double *p, double v) {
  unsigned long long *u = (unsigned long long *)p;
  unsigned long long old = *u;
  while (v < __longlong_as_double(old)) {
    const unsigned long long seen = atomicCAS(u, old, __double_as_longlong(v));
    if (seen == old) break;
    old = seen;
  }
}
__device__ __forceinline__ void atomic_max_f64(double *p, double v) {
  unsigned long long *u = (unsigned long long *)p;
  unsigned long long old = *u;
  while (v > __longlong_as_double(old)) {
    const unsigned long long seen = atomicCAS(u, old, __double_as_longlong(v));
    if (seen == old) break;
    old = seen;
  }
}

// The block's cells are reduced first (wave shuffles, then the four waves'
// partials in LDS), so each of the audit's sums, minima and maxima takes one
// atomic per block instead of one per cell.
constexpr int AUDIT_THREADS = 256;
__global__ __launch_bounds__(AUDIT_THREADS) void k_audit_compare(AuditArgs a) {
  __shared__ double part[AUDIT_THREADS / 64][3];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool in = j < a.na;
  const int64_t i = in ? j * a.stride : 0;
  bool cmp = false;
  if (in) cmp = a.flags[i] == 0 && a.stats_a[2 * a.na + j] == 0;
  const int n_cmp = __syncthreads_count(cmp);
  const int n_in = __syncthreads_count(in);
  if (threadIdx.x == 0) {
    if (n_cmp) atomicAdd(&a.audit[0], (double)n_cmp);
    if (n_in > n_cmp) atomicAdd(&a.audit[1], (double)(n_in - n_cmp));
  }
  if (n_cmp == 0) return;  // uniform over the block
  // sum, min and max of three values over the block, then one atomic each
  auto reduce3 = [&](double s0, double lo, double hi, double *ps, double *pl, double *ph) {
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o);
      lo = fmin(lo, __shfl_xor(lo, o));
      hi = fmax(hi, __shfl_xor(hi, o));
    }
    if (lane == 0) {
      part[w][0] = s0;
      part[w][1] = lo;
      part[w][2] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0, l = INFINITY, h = -INFINITY;
      for (int v = 0; v < AUDIT_THREADS / 64; ++v) {
        t += part[v][0];
        l = fmin(l, part[v][1]);
        h = fmax(h, part[v][2]);
      }
      if (ps) atomicAdd(ps, t);
      if (pl) atomic_min_f64(pl, l);
      if (ph) atomic_max_f64(ph, h);
    }
    __syncthreads();
  };
  reduce3(0.0, INFINITY, cmp ? fabs(a.T[i] - a.Ta[j]) : -INFINITY, nullptr, nullptr,
          &a.audit[2]);
  for (int k = 0; k < a.K; ++k) {
    double d2 = 0.0, dl = INFINITY, dh = -INFINITY;
    if (cmp) {
      const double yr = a.Ya[(int64_t)k * a.na + j];
      const double d = a.Y[(int64_t)k * a.ld + i] - yr;
      const double dref = yr - a.Y0a[(int64_t)k * a.na + j];
      d2 = d * d;
      dl = dh = dref;
    }
    reduce3(d2, dl, dh, &a.audit[3 + 3 * k], &a.audit[4 + 3 * k], &a.audit[5 + 3 * k]);
  }
}

// ---------------------------------------------------------- statistics

// Partial statistics of the training features: block (b, f) covers feature f
// over cells b, b + nblocks, ...  Features 0..K+1 are the network inputs
// (T, p, F(Y0)), features K+2..2K+1 the targets Y1 - Y0.  FP64.  The sums are
// of x - x(cell 0) (the host adds the shift back), so the variance
// E[d^2] - E[d]^2 does not cancel for a feature whose mean is large against
// its spread; block 0 stores the shifts after the [nblocks][F][4] partials.
__device__ __forceinline__ double stat_feature(const StatArgs &a, int f, int64_t i) {
  const int K = a.K;
  if (f == 0) return a.T[i];
  if (f == 1) return a.p[i];
  if (f < K + 2) return (double)boxcox_fast((float)a.Y0[(int64_t)(f - 2) * a.ld + i], a.lambda);
  const int k = f - K - 2;
  return a.Y1[(int64_t)k * a.ld + i] - a.Y0[(int64_t)k * a.ld + i];
}

__global__ void k_stats(StatArgs a) {
  __shared__ double s1[256], s2[256], mn[256], mx[256];
  const int f = blockIdx.y;
  const double shift = stat_feature(a, f, 0);
  double x1 = 0.0, x2 = 0.0, lo = INFINITY, hi = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)a.nblocks * blockDim.x) {
    const double x = stat_feature(a, f, i);
    const double d = x - shift;
    x1 += d;
    x2 += d * d;
    lo = fmin(lo, x);
    hi = fmax(hi, x);
  }
  const int t = threadIdx.x;
  s1[t] = x1;
  s2[t] = x2;
  mn[t] = lo;
  mx[t] = hi;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      s1[t] += s1[t + off];
      s2[t] += s2[t + off];
      mn[t] = fmin(mn[t], mn[t + off]);
      mx[t] = fmax(mx[t], mx[t + off]);
    }
    __syncthreads();
  }
  if (t == 0) {
    double *o = a.part + ((int64_t)blockIdx.x * gridDim.y + f) * 4;
    o[0] = s1[0];
    o[1] = s2[0];
    o[2] = mn[0];
    o[3] = mx[0];
    if (blockIdx.x == 0) a.part[(int64_t)a.nblocks * gridDim.y * 4 + f] = shift;
  }
}

unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

namespace {
bool dma16_ok(const GemmArgs &g) {
  return g.ksplit <= 1 && g.N % 16 == 0 && g.lda % 8 == 0 && g.ldb % 8 == 0 &&
         g.ldcb % 4 == 0 && g.ldcf % 4 == 0 && g.ldz % 4 == 0 && g.ldcq % 4 == 0 &&
         g.K % 32 == 0 && ((uintptr_t)g.A & 15) == 0 && ((uintptr_t)g.B & 15) == 0;
}
}  // namespace

bool gemm_fuses_next(const GemmArgs &g) {
  return dma16_ok(g) && g.N == 416 && (long)((g.M + 255) / 256) >= 512 && g.N2 == 32 &&
         g.N2 <= g.ldcf && g.N2 * (416 + 4) <= 2 * (128 + 416) * 32 && g.B2 &&
         g.bias && g.bias2 && ((uintptr_t)g.B2 & 7) == 0;
}

chem_status gemm(const GemmArgs &g, bool AK, bool BK, int epi, hipStream_t s,
                 const char *label) {
  if (g.M <= 0 || g.N <= 0) return CHEM_OK;
  chem::ProfScope prof(label, s);
  if (g.K % 32 != 0 || (!AK && g.M % 8 != 0) || (!BK && g.N % 8 != 0)) {
    chem::set_error("gemm: K must be a multiple of 32 and transposed dims multiples of 8");
    return CHEM_EINVAL;
  }
  if (g.ksplit > 1 && (g.K % (32 * g.ksplit) != 0 || epi != EPI_F32 || g.bias)) {
    chem::set_error("gemm: split-K needs K a multiple of 32 ksplit, FP32 output, no bias");
    return CHEM_EINVAL;
  }
  if (g.groups > 1) {
    if (g.tiled || epi == EPI_GELU_NEXT || epi == EPI_GELU_Q8 || g.groups > 65535) {
      chem::set_error("gemm: grouped products take the generic tiling only");
      return CHEM_EUNSUPPORTED;
    }
    return gemm_tiled(g, AK, BK, epi, s);
  }
  if (epi == EPI_GELU_NEXT) {
    if (!AK || !BK || !gemm_fuses_next(g)) {
      chem::set_error("gemm: the fused output layer needs the 128 x 416 tiling");
      return CHEM_EUNSUPPORTED;
    }
    // 128 x 416 tiles on a two-stage ring (71 KB of LDS): two blocks per CU,
    // so one block's epilogue (GELU, output layer) runs beside the other's
    // main loop
    return gemm_dma16_cfg<4, 2, 26, 2>(g, epi, s);
  }
  if (g.tiled) {
    // K-blocked operands exist only on the direct-to-LDS path, whose launch
    // thresholds the caller has checked (ann_api: at least 2^17 cells)
    const long mt = (g.M + 255) / 256;
    if (!AK || !BK || epi == EPI_GELUGRAD || !dma16_ok(g) || (g.tiled & ~7)) {
      chem::set_error("gemm: K-blocked operands need the direct-to-LDS tiling");
      return CHEM_EUNSUPPORTED;
    }
    if (g.K == 32 && g.N % 320 == 0) return gemm_dma16_cfg<4, 1, 20, 1>(g, epi, s);
    if (g.N % 400 == 0 && mt * (g.N / 400) >= 512) return gemm_dma16_cfg<8, 2, 25>(g, epi, s);
    if (g.N % 416 == 0 && mt * (g.N / 416) >= 512) return gemm_dma16_cfg<8, 2, 26>(g, epi, s);
    if (g.N <= 32 && mt >= 512) return gemm_dma16_cfg<4, 4, 2>(g, epi, s);
    chem::set_error("gemm: no direct-to-LDS tiling for this K-blocked shape");
    return CHEM_EUNSUPPORTED;
  }
  if (AK && BK && epi != EPI_GELUGRAD && !g.tile && dma16_ok(g)) {
    // forward layers through the direct-to-LDS ring when the launch has at
    // least two blocks per CU of work: K = 32 (first layer) in 64 x 320
    // single-stage tiles; 256 x 400 (or x 416) tiles; 256 x 32 for the
    // 32-wide output layer
    const long mt = (g.M + 255) / 256;
    if (g.K == 32 && g.N % 320 == 0 && 4 * mt * (g.N / 320) >= 512)
      return gemm_dma16_cfg<4, 1, 20, 1>(g, epi, s);
    if (g.N % 400 == 0 && mt * (g.N / 400) >= 512) return gemm_dma16_cfg<8, 2, 25>(g, epi, s);
    if (g.N % 416 == 0 && mt * (g.N / 416) >= 512) return gemm_dma16_cfg<8, 2, 26>(g, epi, s);
    if (g.N <= 32 && mt >= 512) return gemm_dma16_cfg<4, 4, 2>(g, epi, s);
  }
  return gemm_tiled(g, AK, BK, epi, s);
}

void gemm_tile_shape(int t, int *bm, int *bn) {
  static const int shape[GEMM_TILES + 1][2] = {{0, 0}, {128, 128}, {128, 32}, {64, 64},
                                               {128, 64}};
  const int i = t >= 1 && t <= GEMM_TILES ? t : 0;
  *bm = shape[i][0];
  *bn = shape[i][1];
}

bool mlp12_ok(const Mlp12Args &g) {
  auto al = [](const void *p, uintptr_t a) { return p && ((uintptr_t)p & (a - 1)) == 0; };
  return g.K > 0 && g.K % 32 == 0 && g.K <= MLP12_KMAX && g.N > 0 && g.N % 400 == 0 &&
         g.ldw2 >= 32L * g.N && g.ldw2 % 8 == 0 &&
         (g.tiled ? g.ldh % 8 == 0 : (g.ldh >= g.N && g.ldh % 4 == 0)) && al(g.X, 16) &&
         al(g.W1, 16) && al(g.W2p, 16) && al(g.b1, 16) && al(g.b2, 16) && al(g.H, 8);
}

chem_status mlp12(const Mlp12Args &g, hipStream_t s, const char *label) {
  if (g.M <= 0) return CHEM_OK;
  chem::ProfScope prof(label, s);
  if (!mlp12_ok(g)) {
    chem::set_error("mlp12: unsupported shape or misaligned operand");
    return CHEM_EUNSUPPORTED;
  }
  if (g.N % 800 == 0) {
    // paired halves: the first layer once per cell
    constexpr int BM = Mlp12PTile<25>::BM;
    const long total = (long)((g.M + BM - 1) / BM) * (g.N / 800);
    hipLaunchKernelGGL((k_mlp12p<25>), dim3((unsigned)(((total + 7) / 8) * 8)), dim3(8 * 64), 0,
                       s, g);
  } else {
    constexpr int BM = Mlp12Tile<25>::BM;
    const long total = (long)((g.M + BM - 1) / BM) * (g.N / 400);
    hipLaunchKernelGGL((k_mlp12<25>), dim3((unsigned)(((total + 7) / 8) * 8)),
                       dim3(MLP12_WM * 64), 0, s, g);
  }
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

bool gemm8_fuses_next(const GemmArgs &g) {
  return g.K % 128 == 0 && g.lda % 16 == 0 && g.ldb % 16 == 0 && g.N == 416 &&
         (long)((g.M + 127) / 128) >= 512 && g.N2 == 32 && g.N2 <= g.ldcf && g.ldcf % 4 == 0 &&
         g.B2 && g.bias && g.bias2 && ((uintptr_t)g.B2 & 7) == 0 &&
         ((uintptr_t)g.A8 & 15) == 0 && ((uintptr_t)g.B8 & 15) == 0;
}

chem_status gemm8(const GemmArgs &g, int epi, hipStream_t s, const char *label) {
  if (g.M <= 0 || g.N <= 0) return CHEM_OK;
  if (g.K % 64 != 0 || g.lda % 16 != 0 || g.ldb % 16 != 0) {
    chem::set_error("gemm8: K and leading dimensions must be multiples of 64 / 16");
    return CHEM_EINVAL;
  }
  chem::ProfScope prof(label, s);
  if (epi == EPI_GELU_NEXT) {
    // 128 cells x all 416 features per block (two ring stages fit the LDS)
    if (!gemm8_fuses_next(g)) {
      chem::set_error("gemm8: the fused output layer needs the 128 x 416 tiling");
      return CHEM_EUNSUPPORTED;
    }
    return gemm8_dma16_cfg<8, 1, 26, 2>(g, epi, s);
  }
  if (g.K % 128 == 0 && g.N % 16 == 0 && ((uintptr_t)g.A8 & 15) == 0 &&
      ((uintptr_t)g.B8 & 15) == 0 && g.ldcb % 4 == 0 && g.ldcq % 4 == 0) {
    // 256 x 160 tiles (N a multiple of 160), else 128 x 208 (N of 208)
    const long mt = (g.M + 255) / 256;
    if (g.N % 160 == 0 && mt * (g.N / 160) >= 512) return gemm8_dma16_cfg<8, 2, 10>(g, epi, s);
    if (g.N % 208 == 0 && mt * 2 * (g.N / 208) >= 512) return gemm8_dma16_cfg<8, 1, 13>(g, epi, s);
  }
  if (g.tiled) {
    chem::set_error("gemm8: K-blocked operands need the direct-to-LDS tiling");
    return CHEM_EUNSUPPORTED;
  }
  constexpr int BM = 128, BN = 128;
  const long total = (long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  dim3 grid((unsigned)(((total + 7) / 8) * 8)), block(256);
  if (epi == EPI_GELU_Q8)
    hipLaunchKernelGGL((k_gemm8<2, 2, 2, 2, EPI_GELU_Q8>), grid, block, 0, s, g);
  else if (epi == EPI_GELU)
    hipLaunchKernelGGL((k_gemm8<2, 2, 2, 2, EPI_GELU>), grid, block, 0, s, g);
  else {
    chem::set_error("gemm8: unsupported epilogue");
    return CHEM_EUNSUPPORTED;
  }
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status amax(int64_t n, const void *x, bool bf16, float *part, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(k_amax, dim3(nparts), dim3(256), 0, s, n, x, bf16 ? 1 : 0, part);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status quant_e4m3(const float *src, long ld_src, int rows, int cols, uint8_t *dst,
                       int rows_p, int cols_p, float qinv, hipStream_t s) {
  const int64_t n = (int64_t)rows_p * cols_p;
  hipLaunchKernelGGL(k_quant, dim3(nblk(n, 256)), dim3(256), 0, s, src, ld_src, rows, cols, dst,
                     rows_p, cols_p, qinv);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status features(const FeatArgs &a, hipStream_t s) {
  if (a.n <= 0) return CHEM_OK;
  chem::ProfScope prof("ann_features", s);
  const bool small = a.n < (int64_t)256 * 1024;
  if (a.dinp == 32 && small)
    hipLaunchKernelGGL((k_features<32, 64>), dim3(nblk(a.n, 64)), dim3(64), 0, s, a);
  else if (a.dinp == 32)
    hipLaunchKernelGGL((k_features<32, 256>), dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_features<0, 256>), dim3(nblk(a.n, 256)), dim3(256), 0, s, a);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status targets(const TargetArgs &a, hipStream_t s) {
  if (a.n <= 0) return CHEM_OK;
  hipLaunchKernelGGL(k_targets, dim3(nblk(a.n, 64)), dim3(64), 0, s, a);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status phys_grad(const PhysArgs &a, const chem::DevMech &M, double *part, float *loss,
                      float *terms, hipStream_t s) {
  if (a.n <= 0) return CHEM_OK;
  hipLaunchKernelGGL(k_phys, dim3(PHYS_PARTS), dim3(256), 0, s, a, M, part);
  hipLaunchKernelGGL(k_phys_final, dim3(1), dim3(64), 0, s, part, PHYS_PARTS, 1.0 / (double)a.n,
                     a.w[0], a.w[1], a.w[2], loss, terms);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status l1_grad(int64_t n, int K, int doutp, const float *U, const float *Ut, u16 *Gb,
                    float *Gf, double *loss_part, int nparts, float *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_l1, dim3(nparts), dim3(256), 0, s, n, K, doutp, U, Ut, Gb, Gf, loss_part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, loss_part, nparts,
                     1.0 / ((double)n * K), loss);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status l1_grad_members(int64_t n, int G, int ldu, long gu, const float *U, const float *Ut,
                            int ldt, u16 *Gb, float *Gf, double *loss_part, int nparts,
                            float *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_l1_members, dim3(nparts), dim3(256), 0, s, n, G, ldu, gu, U, Ut, ldt, Gb,
                     Gf, loss_part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, loss_part, nparts,
                     1.0 / ((double)n * G), loss);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status take_col(int64_t n, const float *src, int lds, float *dst, int ldd, hipStream_t s) {
  if (n <= 0) return CHEM_OK;
  hipLaunchKernelGGL(k_take_col, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, lds, dst, ldd);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status tile_bf16(int N, int K, const u16 *src, u16 *dst, hipStream_t s, bool permute) {
  if (K % 32 != 0) {
    chem::set_error("tile_bf16: K must be a multiple of 32");
    return CHEM_EINVAL;
  }
  if (permute)
    hipLaunchKernelGGL((k_tile<u16, 32, true>), dim3(nblk((int64_t)N * K, 256)), dim3(256), 0, s,
                       N, K, src, dst);
  else
    hipLaunchKernelGGL((k_tile<u16, 32>), dim3(nblk((int64_t)N * K, 256)), dim3(256), 0, s, N,
                       K, src, dst);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status tile_e4m3(int rows_p, int cols_p, const uint8_t *src, uint8_t *dst, hipStream_t s) {
  if (cols_p % 128 != 0) {
    chem::set_error("tile_e4m3: the padded width must be a multiple of 128");
    return CHEM_EINVAL;
  }
  hipLaunchKernelGGL((k_tile<uint8_t, 128>), dim3(nblk((int64_t)rows_p * cols_p, 256)), dim3(256),
                     0, s, rows_p, cols_p, src, dst);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status colsum(int64_t M, int N, const float *X, long ldx, float *out, double *part,
                   hipStream_t s, int groups, long gx, long gout) {
  const int P = (int)(M < COLSUM_PARTS ? (M > 0 ? M : 1) : COLSUM_PARTS);
  const unsigned G = groups > 1 ? (unsigned)groups : 1u;
  hipLaunchKernelGGL(k_colsum_part, dim3(nblk(N, 64), P, G), dim3(64), 0, s, M, N, X, ldx, part,
                     gx);
  hipLaunchKernelGGL(k_colsum_fin, dim3(nblk(N, 256), 1, G), dim3(256), 0, s, N, P, part, out,
                     gout);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status sum_splits(int64_t n, int S, const float *part, long stride, float *out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_sum_splits, dim3(nblk(n, 256)), dim3(256), 0, s, n, S, part, stride, out);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status adam_multi(const AdamTable &t, float lr, float b1, float b2, float eps, float bc1,
                       float bc2, hipStream_t s) {
  if (t.count < 1 || t.count > ADAM_MAX) {
    chem::set_error("adam_multi: 1..%d tensors", ADAM_MAX);
    return CHEM_EINVAL;
  }
  const int64_t n = t.start[t.count];
  if (n <= 0) return CHEM_OK;
  hipLaunchKernelGGL(k_adam_multi, dim3(nblk(n, 256)), dim3(256), 0, s, t, lr, b1, b2, eps, bc1,
                     bc2);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status to_bf16(int64_t n, const float *src, u16 *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status post(const chem::DevMech &M, const PostArgs &a, hipStream_t s) {
  if (a.n <= 0) return CHEM_OK;
  if (M.E > EMAX) {
    chem::set_error("ann_step: at most %d elements supported", EMAX);
    return CHEM_EUNSUPPORTED;
  }
  chem::ProfScope prof("ann_post", s);
  const dim3 grid(nblk(a.n, 128)), block(128);
  if (M.K <= 16 && M.E <= 4)
    hipLaunchKernelGGL((k_post<16, 4>), grid, block, 0, s, M, a);
  else if (M.K <= 32 && M.E <= 4)
    hipLaunchKernelGGL((k_post<32, 4>), grid, block, 0, s, M, a);
  else if (M.K <= 32)
    hipLaunchKernelGGL((k_post<32, EMAX>), grid, block, 0, s, M, a);
  else
    hipLaunchKernelGGL((k_post<64, EMAX>), grid, block, 0, s, M, a);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status stats_partial(const StatArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(a.nblocks, 2 * a.K + 2), dim3(256), 0, s, a);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status audit_init(double *audit, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_audit_init, dim3(1), dim3(256), 0, s, audit, K);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status audit_gather(const AuditArgs &a, hipStream_t s) {
  if (a.na <= 0) return CHEM_OK;
  hipLaunchKernelGGL(k_audit_gather, dim3(nblk(a.na, 256)), dim3(256), 0, s, a);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}

chem_status audit_compare(const AuditArgs &a, hipStream_t s) {
  if (a.na <= 0) return CHEM_OK;
  hipLaunchKernelGGL(k_audit_compare, dim3(nblk(a.na, AUDIT_THREADS)), dim3(AUDIT_THREADS), 0, s,
                     a);
  CHEM_HIP(hipGetLastError());
  return CHEM_OK;
}


}  // namespace ann
