// cnn_kernels.hip -- kernels of the learned modal reconstructor (gfx950).
//
// Every product (convolutions as im2col products, fully connected layers,
// their data and weight gradients) runs on one tiled bf16 GEMM built on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation: operands staged through
// a double-buffered LDS tile by 16-byte loads, an optional deterministic
// split-K (partials added in split order), and a fused epilogue (bias,
// ReLU, beta * C, FP32 and/or bf16 output).  Activations and upstream
// gradients are carried as bf16 pairs hi + lo (~16 significant bits), so a
// product keeps the precision of FP32 operands to ~2^-17 while every
// multiply runs on the bf16 matrix cores.  Bias gradients come out of the
// weight-gradient product as one extra output column (a column of ones in
// the activation operand).  Small products (a few rows) run on a
// matrix-vector kernel that streams the weights once.  The other kernels
// are gathers and elementwise passes: im2col, col2im in gather form (each
// input element sums its own contributions in a fixed order, no atomics,
// with the ReLU mask), the MSE loss, Adam and the network-input preparation.
// The fully connected layers' data gradients take their ReLU mask in the
// product's epilogue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "cnn_launch.h"

namespace pwfs {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bool bf_pos(uint16_t h) { return h != 0 && !(h & 0x8000u); }

// Split of an FP32 value into bf16 hi + lo (hi = bf16(v), lo = bf16(v - hi)).
__device__ __forceinline__ void split_bf(float v, uint16_t* hi, uint16_t* lo, size_t i) {
  const uint16_t h = f2bf(v);
  hi[i] = h;
  lo[i] = f2bf(v - bf2f(h));
}

// Epilogue of one output element (i, j); j == N is the bias-gradient column.
__device__ __forceinline__ void epilogue(const GemmArgs& g, int i, int j, float x) {
  if (j == g.N) {
    g.bias_grad[i] = x;
    return;
  }
  if (g.bias) x += g.bias[j];
  x *= g.alpha;
  if (g.cperm) j = (j % g.cperm) * 9 + j / g.cperm;   // patch column (tap, c) -> weight column (c, tap)
  if (g.mask && !bf_pos(g.mask[(long)i * g.ldm + j])) x = 0.f;
  if (g.C && g.beta != 0.f) x = fmaf(g.beta, g.C[(long)i * g.ldc + j], x);
  if (g.relu) x = fmaxf(x, 0.f);
  if (g.C) g.C[(long)i * g.ldc + j] = x;
  if (g.Cb) {
    const long o = (long)i * g.ldcb + j;
    const uint16_t h = f2bf(x);
    g.Cb[o] = h;
    if (g.cb_lo) g.Cb[o + g.cb_lo] = f2bf(x - bf2f(h));
  }
}

// The epilogue of four consecutive outputs (i, j .. j + 3) of one row, in
// the order of epilogue(), with vector loads and stores; for outputs without
// the bias-gradient column and the patch-order remap, and 16-byte (FP32) or
// 8-byte (bf16) aligned rows (checked on the host).
__device__ __forceinline__ void epilogue4(const GemmArgs& g, int i, int j, float4 s) {
  float x[4] = {s.x, s.y, s.z, s.w};
  if (g.bias) {
    const float4 b = *reinterpret_cast<const float4*>(g.bias + j);
    x[0] += b.x; x[1] += b.y; x[2] += b.z; x[3] += b.w;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] *= g.alpha;
  if (g.mask) {
    const uint2 m = *reinterpret_cast<const uint2*>(g.mask + (long)i * g.ldm + j);
    const uint32_t mw[2] = {m.x, m.y};
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (!bf_pos((uint16_t)(mw[c >> 1] >> ((c & 1) * 16)))) x[c] = 0.f;
  }
  if (g.C && g.beta != 0.f) {
    const float4 c0 = *reinterpret_cast<const float4*>(g.C + (long)i * g.ldc + j);
    x[0] = fmaf(g.beta, c0.x, x[0]); x[1] = fmaf(g.beta, c0.y, x[1]);
    x[2] = fmaf(g.beta, c0.z, x[2]); x[3] = fmaf(g.beta, c0.w, x[3]);
  }
  if (g.relu)
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = fmaxf(x[c], 0.f);
  if (g.C) *reinterpret_cast<float4*>(g.C + (long)i * g.ldc + j) = make_float4(x[0], x[1], x[2], x[3]);
  if (g.Cb) {
    uint32_t hw[2], lw[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint16_t h0 = f2bf(x[2 * h]), h1 = f2bf(x[2 * h + 1]);
      hw[h] = (uint32_t)h0 | ((uint32_t)h1 << 16);
      lw[h] = (uint32_t)f2bf(x[2 * h] - bf2f(h0)) | ((uint32_t)f2bf(x[2 * h + 1] - bf2f(h1)) << 16);
    }
    const long o = (long)i * g.ldcb + j;
    *reinterpret_cast<uint2*>(g.Cb + o) = make_uint2(hw[0], hw[1]);
    if (g.cb_lo) *reinterpret_cast<uint2*>(g.Cb + o + g.cb_lo) = make_uint2(lw[0], lw[1]);
  }
}

// ---------------------------------------------------------------------------
// Tiled MFMA GEMM.  Block = 4 waves in a WM x WN arrangement, each wave
// owning TM x TN blocks of 32 x 32 outputs: a BM x BN tile, BM = 32 WM TM,
// BN = 32 WN TN.  K advances BK (a multiple of 16; the products use 32) at
// a time through two LDS stages (the next stage's global loads are in
// flight while the current stage is multiplied; one barrier per step).
// LDS holds every operand tile as
// [row][k] with k contiguous and a row pitch of BK + 8 bf16 (the 8 extra
// spread the 16-byte reads of eight consecutive rows over all banks), so an
// MFMA operand is one 16-byte read per lane: v_mfma_f32_32x32x16_bf16
// takes, in lane l, the 8 consecutive k of row (l mod 32) starting at
// 8 (l / 32); its 16 accumulators of lane l are
// C(8 (v / 4) + 4 (l / 32) + v mod 4, l mod 32).
//
// Operand views.  A tile of R rows (rows = i for A, j for B) by BK k comes
// from global memory in one of two layouts:
//  * k-contiguous (stride 1 along k): chunk = 8 k of one row, one 16-byte
//    load (vw 8), two 8-byte loads (vw 4) or 8 element loads (vw 1);
//  * row-contiguous (stride 1 along rows): chunk = 8 rows of one k, one
//    16-byte load (or 2 x 8 / 8 x 2 bytes), stored as loaded into an LDS
//    plane [k][row] (row pitch R + 4); an MFMA fragment then gathers its 8 k
//    of one row with 2-byte LDS reads.  Every thread takes part in the
//    staging, as for k-contiguous operands (transposing in registers left it
//    to one wave and made a k step ~3x slower).
// vw (16-, 8- or 2-byte groups) is decided on the host from the strides,
// extents and alignment, uniform per launch.  Elements past the extents are
// zero; the bias-gradient column (B row N) is 1 in the hi plane.
constexpr int pitch_of(int BK) { return BK + 8; }
constexpr int kStepK = 32;   // k depth per step of the products
// LDS plane of an R-row operand tile, in elements: k-contiguous operands
// [row][k] with pitch BK + 8 (the 16-byte fragment reads of eight
// consecutive rows cover all banks); row-contiguous ones [k][row] with pitch
// R + 4 (8-byte aligned rows; the two half-waves' k, 8 apart, fall on
// different banks).
constexpr int plane_elems(bool kc, int R, int BK) { return kc ? R * pitch_of(BK) : BK * (R + 4); }

struct OpView {
  const uint16_t* p;
  long s_row, s_k;     // element strides along the tile's rows and along k
  int rows;            // extent of rows holding data
  int ones_row;        // a row of ones at this index (hi plane), -1: none
  int vw;              // 8, 4 or 1 elements per load along the contiguous dimension
  // implicit convolution patches (conv != 0): p is the NHWC activation
  // [B][H][W][C]; a patch element (pixel (b, yo, xo), column (ky, kx, c)) is
  // p[b][2 yo + ky - 1][2 xo + kx - 1][c], 0 outside (C a multiple of 8, so
  // an 8-element chunk is 8 channels of one tap: one 16-byte load)
  int conv, H, W, C, Wo, HoWo;
};

// Address of the 8-channel chunk (pixel, column col0) of an implicit patch
// view, or NULL when the tap falls in the padding.
__device__ __forceinline__ const uint16_t* patch_chunk(const OpView& v, const uint16_t* p, uint32_t pixel,
                                                       uint32_t col0) {
  const uint32_t tap = col0 / (uint32_t)v.C, c0 = col0 - tap * (uint32_t)v.C;
  const uint32_t b = pixel / (uint32_t)v.HoWo, rem = pixel - b * (uint32_t)v.HoWo;
  const uint32_t yo = rem / (uint32_t)v.Wo, xo = rem - yo * (uint32_t)v.Wo;
  const int y = 2 * (int)yo + (int)(tap / 3) - 1, x = 2 * (int)xo + (int)(tap % 3) - 1;
  if (y < 0 || y >= v.H || x < 0 || x >= v.W) return nullptr;
  return p + (((size_t)b * v.H + y) * v.W + x) * v.C + c0;
}

struct Chunk8 { uint32_t w[4]; };

__device__ __forceinline__ uint32_t ld_u16(const uint16_t* p) { return *p; }

// 8 elements along the contiguous dimension starting at `e` (element index
// along it), `lim` the extent there; q: address of element 0.
__device__ __forceinline__ Chunk8 load8(const uint16_t* q, int e, int lim, int vw) {
  Chunk8 c;
  if (vw == 8) {
    if (e < lim) {
      const uint4 v = *reinterpret_cast<const uint4*>(q);
      c.w[0] = v.x; c.w[1] = v.y; c.w[2] = v.z; c.w[3] = v.w;
    } else {
      c.w[0] = c.w[1] = c.w[2] = c.w[3] = 0u;
    }
  } else if (vw == 4) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (e + 4 * h < lim) {
        const uint2 v = *reinterpret_cast<const uint2*>(q + 4 * h);
        c.w[2 * h] = v.x; c.w[2 * h + 1] = v.y;
      } else {
        c.w[2 * h] = c.w[2 * h + 1] = 0u;
      }
    }
  } else {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const uint32_t lo = (e + 2 * h < lim) ? ld_u16(q + 2 * h) : 0u;
      const uint32_t hi = (e + 2 * h + 1 < lim) ? ld_u16(q + 2 * h + 1) : 0u;
      c.w[h] = lo | (hi << 16);
    }
  }
  return c;
}

__device__ __forceinline__ void set_half(Chunk8& c, int r, uint32_t v) {
  const int s = (r & 1) * 16;
  c.w[r >> 1] = (c.w[r >> 1] & ~(0xffffu << s)) | (v << s);
}

// Staged global data of one operand plane for one k step: up to 4 chunks
// (k-contiguous) or one quad-chunk of 4 loads (row-contiguous) per thread,
// which bounds a tile's R rows x BK k at 8192 elements.
struct Stage {
  Chunk8 c[4];
};

template <bool KC, int R, int BK>
__device__ __forceinline__ void op_load(const OpView& v, long lo, int r0, int k0, int K, Stage& s, int tid) {
  static_assert(R * BK <= 8192, "operand tile too large for the staging registers");
  constexpr int CPR = BK / 8;   // chunks per row
  const uint16_t* p = v.p + lo;
  if constexpr (KC) {
    // R rows x CPR chunks; thread t takes chunks t, t + 256, ...
#pragma unroll
    for (int t = 0; t < (R * CPR + 255) / 256; ++t) {
      const int c = tid + 256 * t;
      if (c < R * CPR) {
        const int row = c / CPR, kk = (c % CPR) * 8;
        const int gr = r0 + row;
        const bool in = gr < v.rows;
        const int gk = k0 + kk;
        if (v.conv) {
          const uint16_t* q = (in && gk < K) ? patch_chunk(v, p, (uint32_t)gr, (uint32_t)gk) : nullptr;
          if (q) {
            const uint4 x = *reinterpret_cast<const uint4*>(q);
            s.c[t].w[0] = x.x; s.c[t].w[1] = x.y; s.c[t].w[2] = x.z; s.c[t].w[3] = x.w;
          } else {
            s.c[t].w[0] = s.c[t].w[1] = s.c[t].w[2] = s.c[t].w[3] = 0u;
          }
        } else if (in) {
          s.c[t] = load8(p + (long)gr * v.s_row + gk, gk, K, v.vw);
        } else {
          s.c[t].w[0] = s.c[t].w[1] = s.c[t].w[2] = s.c[t].w[3] = 0u;
        }
        if (gr == v.ones_row && lo == 0) {
#pragma unroll
          for (int e = 0; e < 8; ++e) set_half(s.c[t], e, gk + e < K ? 0x3f80u : 0u);
        }
      }
    }
  } else {
    // (R / 8) row groups x BK k; unit u = (row group u mod (R / 8), k u / (R / 8)),
    // thread t takes units t, t + 256, ... (a wave reads whole 128-byte rows)
    constexpr int RG = R / 8;
#pragma unroll
    for (int t = 0; t < (RG * BK + 255) / 256; ++t) {
      const int u = tid + 256 * t;
      if (u < RG * BK) {
        const int gr = r0 + (u % RG) * 8, gk = k0 + u / RG;
        if (v.conv) {
          const uint16_t* q = (gk < K && gr < v.rows) ? patch_chunk(v, p, (uint32_t)gk, (uint32_t)gr) : nullptr;
          if (q) {
            const uint4 x = *reinterpret_cast<const uint4*>(q);
            s.c[t].w[0] = x.x; s.c[t].w[1] = x.y; s.c[t].w[2] = x.z; s.c[t].w[3] = x.w;
          } else {
            s.c[t].w[0] = s.c[t].w[1] = s.c[t].w[2] = s.c[t].w[3] = 0u;
          }
        } else if (gk < K) {
          s.c[t] = load8(p + (long)gk * v.s_k + gr, gr, v.rows, v.vw);
        } else {
          s.c[t].w[0] = s.c[t].w[1] = s.c[t].w[2] = s.c[t].w[3] = 0u;
        }
        if (lo == 0) {
#pragma unroll
          for (int r = 0; r < 8; ++r)
            if (v.ones_row == gr + r) set_half(s.c[t], r, gk < K ? 0x3f80u : 0u);
        }
      }
    }
  }
}

template <bool KC, int R, int BK>
__device__ __forceinline__ void op_store(uint16_t* lds, const Stage& s, int tid) {
  constexpr int CPR = BK / 8, PITCH = pitch_of(BK);
  if constexpr (KC) {
#pragma unroll
    for (int t = 0; t < (R * CPR + 255) / 256; ++t) {
      const int c = tid + 256 * t;
      if (c < R * CPR) {
        const int row = c / CPR, kk = (c % CPR) * 8;
        *reinterpret_cast<uint4*>(lds + row * PITCH + kk) = make_uint4(s.c[t].w[0], s.c[t].w[1], s.c[t].w[2], s.c[t].w[3]);
      }
    }
  } else {
    constexpr int RG = R / 8, RP = R + 4;
#pragma unroll
    for (int t = 0; t < (RG * BK + 255) / 256; ++t) {
      const int u = tid + 256 * t;
      if (u < RG * BK) {
        uint16_t* q = lds + (u / RG) * RP + (u % RG) * 8;
        *reinterpret_cast<uint2*>(q) = make_uint2(s.c[t].w[0], s.c[t].w[1]);
        *reinterpret_cast<uint2*>(q + 4) = make_uint2(s.c[t].w[2], s.c[t].w[3]);
      }
    }
  }
}

// MFMA fragment of one lane: the 8 consecutive k from kof of tile row `row`.
template <bool KC, int R, int BK>
__device__ __forceinline__ bf16x8 frag(const uint16_t* plane, int row, int kof) {
  if constexpr (KC) {
    return *reinterpret_cast<const bf16x8*>(plane + row * pitch_of(BK) + kof);
  } else {
    constexpr int RP = R + 4;
    const uint16_t* q = plane + kof * RP + row;
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) w[h] = (uint32_t)q[(2 * h) * RP] | ((uint32_t)q[(2 * h + 1) * RP] << 16);
    bf16x8 f;
    __builtin_memcpy(&f, w, sizeof(f));
    return f;
  }
}

// Output of a wave's 32 x 32 accumulator block through LDS: 32 rows of 36
// floats (the pitch keeps float4 rows aligned), read back as 4 consecutive
// columns of one row per lane, so that a row leaves in 16-byte (FP32) or
// 8-byte (bf16) pieces instead of one element per lane and store.
constexpr int kEpiPitch = 36;
__device__ __forceinline__ float f4at(const float4& x, int q) { return q == 0 ? x.x : q == 1 ? x.y : q == 2 ? x.z : x.w; }
constexpr size_t kEpiLdsBytes = (size_t)4 * 32 * kEpiPitch * sizeof(float);   // four waves

// evec bit 0: epilogue4 may take four regular columns (no patch-order remap,
// aligned rows); bit 1: the partial rows are 16-byte aligned (Nc a multiple of 4).
template <int WM, int WN, int TM, int TN, bool AKC, bool BKC, int BK>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(GemmArgs g, OpView va, OpView vb, int kc,
                                                        float* __restrict__ part, int evec) {
  constexpr int BM = 32 * WM * TM, BN = 32 * WN * TN;
  constexpr int SA = plane_elems(AKC, BM, BK), SB = plane_elems(BKC, BN, BK);
  extern __shared__ __align__(16) uint16_t lds[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WN, wn = wave % WN;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * kc;
  const int kend = min(g.K, kbeg + kc);
  const bool alo = g.a_lo != 0, blo = g.b_lo != 0;
  // LDS stage: planes A_hi, A_lo (if any), B_hi, B_lo (if any)
  const int stage_elems = SA * (alo ? 2 : 1) + SB * (blo ? 2 : 1);
  uint16_t* st0 = lds;
  uint16_t* st1 = lds + stage_elems;
  auto a_hi = [&](uint16_t* s) { return s; };
  auto a_lo = [&](uint16_t* s) { return s + SA; };
  auto b_hi = [&](uint16_t* s) { return s + SA * (alo ? 2 : 1); };
  auto b_lo = [&](uint16_t* s) { return s + SA * (alo ? 2 : 1) + SB; };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

  Stage sa, sal, sb, sbl;
  // prologue
  op_load<AKC, BM, BK>(va, 0, i0, kbeg, kend, sa, tid);
  if (alo) op_load<AKC, BM, BK>(va, g.a_lo, i0, kbeg, kend, sal, tid);
  op_load<BKC, BN, BK>(vb, 0, j0, kbeg, kend, sb, tid);
  if (blo) op_load<BKC, BN, BK>(vb, g.b_lo, j0, kbeg, kend, sbl, tid);
  op_store<AKC, BM, BK>(a_hi(st0), sa, tid);
  if (alo) op_store<AKC, BM, BK>(a_lo(st0), sal, tid);
  op_store<BKC, BN, BK>(b_hi(st0), sb, tid);
  if (blo) op_store<BKC, BN, BK>(b_lo(st0), sbl, tid);
  __syncthreads();

  int it = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK, ++it) {
    uint16_t* cur = (it & 1) ? st1 : st0;
    uint16_t* nxt = (it & 1) ? st0 : st1;
    const bool more = k0 + BK < kend;
    if (more) {
      op_load<AKC, BM, BK>(va, 0, i0, k0 + BK, kend, sa, tid);
      if (alo) op_load<AKC, BM, BK>(va, g.a_lo, i0, k0 + BK, kend, sal, tid);
      op_load<BKC, BN, BK>(vb, 0, j0, k0 + BK, kend, sb, tid);
      if (blo) op_load<BKC, BN, BK>(vb, g.b_lo, j0, k0 + BK, kend, sbl, tid);
    }
#pragma unroll
    for (int sub = 0; sub < BK / 16; ++sub) {
      const int kof = sub * 16 + 8 * (lane >> 5);
      bf16x8 fa[TM], fb[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a)
        fa[a] = frag<AKC, BM, BK>(a_hi(cur), wm * TM * 32 + a * 32 + (lane & 31), kof);
#pragma unroll
      for (int b = 0; b < TN; ++b)
        fb[b] = frag<BKC, BN, BK>(b_hi(cur), wn * TN * 32 + b * 32 + (lane & 31), kof);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
      if (alo) {
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          const bf16x8 fl = frag<AKC, BM, BK>(a_lo(cur), wm * TM * 32 + a * 32 + (lane & 31), kof);
#pragma unroll
          for (int b = 0; b < TN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl, fb[b], acc[a][b], 0, 0, 0);
        }
      }
      if (blo) {
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const bf16x8 fl = frag<BKC, BN, BK>(b_lo(cur), wn * TN * 32 + b * 32 + (lane & 31), kof);
#pragma unroll
          for (int a = 0; a < TM; ++a) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fl, acc[a][b], 0, 0, 0);
        }
      }
    }
    if (more) {
      op_store<AKC, BM, BK>(a_hi(nxt), sa, tid);
      if (alo) op_store<AKC, BM, BK>(a_lo(nxt), sal, tid);
      op_store<BKC, BN, BK>(b_hi(nxt), sb, tid);
      if (blo) op_store<BKC, BN, BK>(b_lo(nxt), sbl, tid);
    }
    __syncthreads();
  }

  // the loop ended with a barrier: the operand stages are free
  const int Nc = g.N + (g.bias_grad ? 1 : 0);
  float* sc = reinterpret_cast<float*>(lds) + wave * 32 * kEpiPitch;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
#pragma unroll
      for (int v = 0; v < 16; ++v) sc[(8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)) * kEpiPitch + (lane & 31)] = acc[a][b][v];
      __syncthreads();
      const int c = (lane & 7) * 4;
      const int j = j0 + wn * TN * 32 + b * 32 + c;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int r = p * 8 + (lane >> 3);
        const int i = i0 + wm * TM * 32 + a * 32 + r;
        if (i >= g.M || j >= Nc) continue;
        const float4 x = *reinterpret_cast<const float4*>(sc + r * kEpiPitch + c);
        if (part) {
          float* o = part + ((size_t)blockIdx.z * g.M + i) * Nc + j;
          if ((evec & 2) && j + 3 < Nc) {
            *reinterpret_cast<float4*>(o) = x;
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (j + q < Nc) o[q] = f4at(x, q);
          }
        } else if ((evec & 1) && j + 3 < g.N) {
          epilogue4(g, i, j, x);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (j + q < Nc) epilogue(g, i, j + q, f4at(x, q));
        }
      }
      if (a + 1 < TM || b + 1 < TN) __syncthreads();
    }
}

// Sum of split-K partials, then the epilogue.  Thread = V consecutive
// outputs (V = 4: one 16-byte load per partial, when M Nc is a multiple of
// 4 so that every partial slice stays aligned), block = 256 / G threads x G
// split groups: group q adds splits q, q + G, ... in order, then the G group
// sums are added in group order (a fixed order overall; each output's
// component is summed on its own).  Many splits over few outputs (long-K
// weight gradients) take G = 16 or 64, so that each thread adds only
// splits / G partials.  VEC: the four outputs are one row's (Nc a multiple
// of 4) and take the vector epilogue.
template <int G, int V, bool VEC>
__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmArgs g, int splits, const float* __restrict__ part) {
  constexpr int EL = 256 / G;
  typedef float vec_t __attribute__((ext_vector_type(V)));
  __shared__ vec_t red[G][EL];
  const int Nc = g.N + (g.bias_grad ? 1 : 0);
  const size_t MN = (size_t)g.M * Nc, MNV = MN / V;
  const int e = threadIdx.x % EL, q = threadIdx.x / EL;
  const size_t idx = blockIdx.x * (size_t)EL + e;
  vec_t x = 0.f;
  if (idx < MNV)
    for (int z = q; z < splits; z += G) x += reinterpret_cast<const vec_t*>(part + (size_t)z * MN)[idx];
  red[q][e] = x;
  __syncthreads();
  if (q == 0 && idx < MNV) {
    vec_t s = red[0][e];
#pragma unroll
    for (int t = 1; t < G; ++t) s += red[t][e];
    const size_t o = idx * V;
    if constexpr (VEC) {
      epilogue4(g, (int)(o / Nc), (int)(o % Nc), make_float4(s[0], s[1], s[2], s[3]));
    } else {
#pragma unroll
      for (int c = 0; c < V; ++c) epilogue(g, (int)((o + c) / Nc), (int)((o + c) % Nc), s[c]);
    }
  }
}

// Small-M products C(i, j) = sum_k A[i][k] B[j][k] (both operands
// contiguous in k; a few rows of activations against a weight matrix).
// Block = W <= 8 waves over RW = 4 columns j and BT <= 16 rows i (grid over
// both); thread t takes the 8-element (16-byte) k groups t, t + 64 W, ...,
// loads the RW weight rows' and the BT activation rows' groups before any
// product, and keeps the RW x BT sums; with a split activation operand the
// lo plane's groups follow the hi plane's against the same weight groups.
// Each wave adds its 64 lanes by recursive halving (a lane keeps half of
// its sums and trades the other half at each step), the W wave sums are
// added in wave order through LDS (fixed order), then the epilogue.
// Columns and rows past the ends are clamped to the last one for loading
// (in bounds, never stored).  The weights stream from HBM once.
constexpr int kGemvMaxWaves = 8;

template <class V>
__device__ __forceinline__ uint32_t vword(const V& v, int h) {
  if constexpr (sizeof(V) == 16) return h == 0 ? v.x : h == 1 ? v.y : h == 2 ? v.z : v.w;
  else return h == 0 ? v.x : v.y;
}

// GW: k elements per load (8: 16-byte groups; 4: 8-byte groups, for K a
// multiple of 4 only, such as the first convolution's 36).
template <int BT, int GW>
__global__ __launch_bounds__(64 * kGemvMaxWaves) void gemv_bf16_kernel(GemmArgs g) {
  constexpr int RW = 4;
  constexpr int NV = RW * BT;
  constexpr int LOG2NV = NV >= 64 ? 6 : NV >= 32 ? 5 : NV >= 16 ? 4 : NV >= 8 ? 3 : NV >= 4 ? 2 : NV >= 2 ? 1 : 0;
  constexpr int SH = 6 - LOG2NV;
  static_assert((NV & (NV - 1)) == 0 && NV <= 64, "RW x BT sums: a power of two <= 64");
  __shared__ float wsum[kGemvMaxWaves][NV];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int W = (int)(blockDim.x >> 6);
  const int j0 = blockIdx.x * RW, i0 = blockIdx.y * BT;
  using V = typename std::conditional<GW == 8, uint4, uint2>::type;
  const int ng = g.K / GW;
  const int planes = g.a_lo ? 2 : 1;
  float v[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) v[e] = 0.f;
  for (int q = tid; q < ng; q += 64 * W) {
    V wr[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r)
      wr[r] = reinterpret_cast<const V*>(g.B + (long)min(j0 + r, g.N - 1) * g.sbn)[q];
    for (int pl = 0; pl < planes; ++pl) {
      V ar[BT];
      const uint16_t* Ap = g.A + (pl ? g.a_lo : 0);
#pragma unroll
      for (int b = 0; b < BT; ++b) ar[b] = reinterpret_cast<const V*>(Ap + (long)min(i0 + b, g.M - 1) * g.sam)[q];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int h = 0; h < GW / 2; ++h) {
        float wl[RW], wh[RW], al[BT], ah[BT];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const uint32_t u = vword(wr[r], h);
          wl[r] = __uint_as_float(u << 16);
          wh[r] = __uint_as_float(u & 0xffff0000u);
        }
#pragma unroll
        for (int b = 0; b < BT; ++b) {
          const uint32_t u = vword(ar[b], h);
          al[b] = __uint_as_float(u << 16);
          ah[b] = __uint_as_float(u & 0xffff0000u);
        }
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
          for (int b = 0; b < BT; ++b) {
            float& acc = v[r * BT + b];
            acc = fmaf(wl[r], al[b], acc);
            acc = fmaf(wh[r], ah[b], acc);
          }
      }
    }
  }
#pragma unroll
  for (int st = 0; st < LOG2NV; ++st) {
    const int o = 32 >> st, hh = NV >> (st + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int e = 0; e < NV / 2; ++e) {
      if (e < hh) {
        const float keep = up ? v[e + hh] : v[e];
        const float give = up ? v[e] : v[e + hh];
        v[e] = keep + __shfl_xor(give, o);
      }
    }
  }
#pragma unroll
  for (int o = 32 >> LOG2NV; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o);
  if ((lane & ((1 << SH) - 1)) == 0) wsum[wave][lane >> SH] = v[0];
  __syncthreads();
  if (tid < NV) {
    const int r = tid / BT, b = tid - r * BT;
    const int i = i0 + b, j = j0 + r;
    if (i < g.M && j < g.N) {
      float x = wsum[0][tid];
      for (int w = 1; w < W; ++w) x += wsum[w][tid];
      epilogue(g, i, j, x);
    }
  }
}

// ---------------------------------------------------------------------------
// im2col for a 3x3 stride-2 pad-1 convolution, NHWC input, patch columns in
// (ky, kx, c) order:
// cols[(b, yo, xo)][(ky * 3 + kx) C + c] = act[b][2 yo + ky - 1][2 xo + kx - 1][c] (0 outside),
// so that a tap's C channels are contiguous on both sides.  From a bf16 pair
// input (lo plane n_in elements after the hi plane) both planes are gathered
// (the lo plane of cols n_out elements after its hi plane), 8 channels per
// 16-byte move when C is a multiple of 8; from an FP32 input each value is
// rounded to bf16 (one plane): the network input's conversion and its
// im2col in one pass.  One thread per (row, tap, group of V channels).
template <int V>
__global__ __launch_bounds__(256) void im2col_pair_kernel(const uint16_t* __restrict__ act, int B, int H, int W,
                                                          int C, uint16_t* __restrict__ cols) {
  // 32-bit index arithmetic (sizes checked on the host): 64-bit divisions
  // are long emulated sequences that made this gather ALU-bound
  const uint32_t Ho = (H + 1) / 2, Wo = (W + 1) / 2, HoWo = Ho * Wo;
  const uint32_t G = C / V;                                  // channel groups per tap
  const uint32_t K9 = (uint32_t)C * 9;
  const uint32_t rows = (uint32_t)B * HoWo;
  const uint32_t total = rows * 9 * G;
  const uint32_t n_in = (uint32_t)B * H * W * C, n_out = rows * K9;
  for (uint32_t idx = blockIdx.x * 256u + threadIdx.x; idx < total; idx += gridDim.x * 256u) {
    const uint32_t t2 = idx / G, cg = idx - t2 * G;
    const uint32_t row = t2 / 9, tap = t2 - row * 9;
    const int ky = (int)tap / 3, kx = (int)tap - ky * 3;
    const uint32_t b = row / HoWo, rem = row - b * HoWo;
    const uint32_t yo = rem / Wo, xo = rem - yo * Wo;
    const int y = 2 * (int)yo + ky - 1, x = 2 * (int)xo + kx - 1;
    const bool in = y >= 0 && y < H && x >= 0 && x < W;
    const uint32_t src = in ? ((b * H + y) * W + x) * C + cg * V : 0u;
    const uint32_t dst = row * K9 + tap * C + cg * V;
    if constexpr (V == 8) {
      const uint4 z = make_uint4(0u, 0u, 0u, 0u);
      *reinterpret_cast<uint4*>(cols + dst) = in ? *reinterpret_cast<const uint4*>(act + src) : z;
      *reinterpret_cast<uint4*>(cols + dst + n_out) = in ? *reinterpret_cast<const uint4*>(act + src + n_in) : z;
    } else {
      cols[dst] = in ? act[src] : (uint16_t)0;
      cols[dst + n_out] = in ? act[src + n_in] : (uint16_t)0;
    }
  }
}

__global__ __launch_bounds__(256) void im2col_f32_kernel(const float* __restrict__ act, int B, int H, int W, int C,
                                                         uint16_t* __restrict__ cols) {
  const uint32_t Ho = (H + 1) / 2, Wo = (W + 1) / 2, HoWo = Ho * Wo;
  const uint32_t K9 = (uint32_t)C * 9;
  const uint32_t total = (uint32_t)B * HoWo * 9;
  for (uint32_t idx = blockIdx.x * 256u + threadIdx.x; idx < total; idx += gridDim.x * 256u) {
    const uint32_t row = idx / 9, tap = idx - row * 9;
    const int ky = (int)tap / 3, kx = (int)tap - ky * 3;
    const uint32_t b = row / HoWo, rem = row - b * HoWo;
    const uint32_t yo = rem / Wo, xo = rem - yo * Wo;
    const int y = 2 * (int)yo + ky - 1, x = 2 * (int)xo + kx - 1;
    const bool in = y >= 0 && y < H && x >= 0 && x < W;
    const float* src = act + (in ? ((b * H + y) * W + x) * C : 0u);
    uint16_t* dst = cols + row * K9 + tap * C;
    for (int c = 0; c < C; ++c) dst[c] = in ? f2bf(src[c]) : (uint16_t)0;
  }
}

// Gradient of im2col (gather form) fused with the ReLU mask of the layer's
// forward output act (hi plane): dz[b][y][x][c] = (act > 0) * sum over the
// taps (ky, kx) whose output pixel (yo, xo) = ((y + 1 - ky) / 2, (x + 1 - kx) / 2)
// exists, in tap order, of dcols[(b, yo, xo)][(ky * 3 + kx) C + c].  One
// thread per (pixel, group of V channels); writes the bf16 pair (lo at
// dzb + B H W C).
template <int V>
__global__ __launch_bounds__(256) void col2im_mask_kernel(const float* __restrict__ dcols, int B, int H, int W,
                                                          int C, const uint16_t* __restrict__ act,
                                                          uint16_t* __restrict__ dzb) {
  const int Ho = (H + 1) / 2, Wo = (W + 1) / 2;
  const uint32_t G = C / V;
  const uint32_t n = (uint32_t)B * H * W * C;
  const uint32_t total = (uint32_t)B * H * W * G;
  for (uint32_t idx = blockIdx.x * 256u + threadIdx.x; idx < total; idx += gridDim.x * 256u) {
    const uint32_t pix = idx / G, cg = idx - pix * G;
    const uint32_t t2 = pix / W, b = t2 / H;
    const int x = (int)(pix - t2 * W), y = (int)(t2 - b * H);
    float s[V];
#pragma unroll
    for (int v = 0; v < V; ++v) s[v] = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
      const int yy = y + 1 - ky;
      if (yy < 0 || (yy & 1) || (yy >> 1) >= Ho) continue;
      for (int kx = 0; kx < 3; ++kx) {
        const int xx = x + 1 - kx;
        if (xx < 0 || (xx & 1) || (xx >> 1) >= Wo) continue;
        const float* d = dcols + ((b * Ho + (yy >> 1)) * Wo + (xx >> 1)) * (uint32_t)(C * 9) +
                         (uint32_t)(ky * 3 + kx) * C + cg * V;
        if constexpr (V == 8) {
          const float4 u = reinterpret_cast<const float4*>(d)[0], w = reinterpret_cast<const float4*>(d)[1];
          s[0] += u.x; s[1] += u.y; s[2] += u.z; s[3] += u.w;
          s[4] += w.x; s[5] += w.y; s[6] += w.z; s[7] += w.w;
        } else {
          s[0] += d[0];
        }
      }
    }
    const uint32_t o = pix * C + cg * V;
    if constexpr (V == 8) {   // 16-byte mask load, 16-byte hi and lo stores (o and n are multiples of 8)
      const uint4 m = *reinterpret_cast<const uint4*>(act + o);
      const uint32_t mw[4] = {m.x, m.y, m.z, m.w};
      uint32_t hw[4], lw[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint16_t h[2], l[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float x = bf_pos((uint16_t)(mw[q] >> (16 * e))) ? s[2 * q + e] : 0.f;
          h[e] = f2bf(x);
          l[e] = f2bf(x - bf2f(h[e]));
        }
        hw[q] = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        lw[q] = (uint32_t)l[0] | ((uint32_t)l[1] << 16);
      }
      *reinterpret_cast<uint4*>(dzb + o) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
      *reinterpret_cast<uint4*>(dzb + n + o) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    } else {
      split_bf(bf_pos(act[o]) ? s[0] : 0.f, dzb, dzb + n, o);
    }
  }
}

// dz = (act > 0) * g as a bf16 pair (lo written at dzb + n).
// Position in the bf16 product copy of parameter i: convolution weights
// [Cout][Cin][3][3] are stored [Cout][3][3][Cin] there (the patch order of
// im2col), everything else in place.
__device__ __forceinline__ size_t wb_index(const ConvPerm& cp, size_t i) {
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const size_t len = (size_t)cp.cout[s] * cp.cin[s] * 9;
    if (i >= cp.off[s] && i < cp.off[s] + len) {
      const size_t l = i - cp.off[s];
      const size_t per_o = (size_t)cp.cin[s] * 9;
      const size_t o = l / per_o, rem = l - o * per_o;
      const size_t c = rem / 9, tap = rem - c * 9;
      return cp.off[s] + o * per_o + tap * cp.cin[s] + c;
    }
  }
  return i;
}

__global__ __launch_bounds__(256) void weights_bf16_kernel(const float* __restrict__ x, size_t n, ConvPerm cp,
                                                           uint16_t* __restrict__ y) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    y[wb_index(cp, i)] = f2bf(x[i]);
}

// Weighted MSE: gradient 2 w (p - t) / n as a bf16 pair (lo at doutb + n)
// and per-block partial sums of w (p - t)^2 (block b: elements
// [b 1024, (b + 1) 1024), fixed tree); mse_sum_kernel adds the partials in
// block order and divides by n.
constexpr int kMseBlock = 1024;

__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ pred, const float* __restrict__ target,
                                                  const float* __restrict__ weights, int n, int n_out,
                                                  uint16_t* __restrict__ doutb, float* __restrict__ part) {
  __shared__ float red[256];
  const int tid = threadIdx.x;
  const float inv = 1.f / (float)n;
  float s = 0.f;
  for (int t = 0; t < kMseBlock / 256; ++t) {
    const int i = blockIdx.x * kMseBlock + t * 256 + tid;
    if (i < n) {
      const float d = pred[i] - target[i];
      const float w = weights ? weights[i / n_out] : 1.f;
      s = fmaf(w * d, d, s);
      split_bf(2.f * w * d * inv, doutb, doutb + n, i);
    }
  }
  red[tid] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void mse_sum_kernel(const float* __restrict__ part, int nb, int n,
                                                      float* __restrict__ loss) {
  __shared__ float red[256];
  const int tid = threadIdx.x;
  float s = 0.f;
  for (int b = tid; b < nb; b += 256) s += part[b];
  red[tid] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) *loss = red[0] / (float)n;
}

// Adam on the FP32 master weights; refreshes the bf16 copy.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                                   float* __restrict__ v, uint16_t* __restrict__ wb, ConvPerm cp,
                                                   size_t i0, size_t n, float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
  for (size_t i = i0 + blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[wb_index(cp, i)] = f2bf(wi);
  }
}

__global__ __launch_bounds__(256) void fill0_kernel(float* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0.f;
}

// Network input: one block per frame.
__global__ __launch_bounds__(256) void prepare_kernel(const float* __restrict__ pupils, const float* __restrict__ ref,
                                                      const int* __restrict__ valid, int nv, int S, float* __restrict__ x) {
  __shared__ float red[2][256];
  const int tid = threadIdx.x;
  const size_t b = blockIdx.x;
  const size_t SS = (size_t)S * S;
  const float* p = pupils + b * 4 * SS;
  float s = 0.f, r = 0.f;
  for (int v = tid; v < nv; v += 256) {
    const size_t j = (size_t)valid[v];
    s += (p[j] + p[SS + j]) + (p[2 * SS + j] + p[3 * SS + j]);
    r += (ref[j] + ref[SS + j]) + (ref[2 * SS + j] + ref[3 * SS + j]);
  }
  red[0][tid] = s;
  red[1][tid] = r;
  float* xo = x + b * 4 * SS;
  for (size_t i = tid; i < 4 * SS; i += 256) xo[i] = 0.f;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      red[0][tid] += red[0][tid + st];
      red[1][tid] += red[1][tid + st];
    }
    __syncthreads();
  }
  const float n = red[0][0] / (float)nv, nr = red[1][0] / (float)nv;
  for (int v = tid; v < nv; v += 256) {
    const size_t j = (size_t)valid[v];
    for (int q = 0; q < 4; ++q) xo[j * 4 + q] = p[q * SS + j] / n - ref[q * SS + j] / nr;
  }
}

// ---------------------------------------------------------------------------
static unsigned grid_for(size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 8192); }

template <int BT, int GW>
static hipError_t launch_gemv(const GemmArgs& g, hipStream_t st) {
  const int ng = g.K / GW;
  const int waves = std::max(1, std::min(kGemvMaxWaves, (ng + 63) / 64));
  hipLaunchKernelGGL((gemv_bf16_kernel<BT, GW>), dim3((g.N + 3) / 4, (g.M + BT - 1) / BT), dim3(64 * waves), 0, st,
                     g);
  return hipGetLastError();
}

template <int GW>
static hipError_t launch_gemv_gw(const GemmArgs& g, hipStream_t st) {
  if (g.M == 1) return launch_gemv<1, GW>(g, st);
  if (g.M <= 4) return launch_gemv<4, GW>(g, st);
  if (g.M <= 8) return launch_gemv<8, GW>(g, st);
  return launch_gemv<16, GW>(g, st);
}

// Widest load group (8, 4 or 1 elements) along the contiguous dimension of
// an operand: its extent and the other stride must be multiples, the base
// (and lo plane) aligned.
static int vec_width(const uint16_t* p, long lo, long other_stride, int extent) {
  for (int w : {8, 4}) {
    const uintptr_t al = (uintptr_t)w * 2;
    if (extent % w == 0 && other_stride % w == 0 && lo % w == 0 && (uintptr_t)p % al == 0) return w;
  }
  return 1;
}

template <int WM, int WN, int TM, int TN, bool AKC, bool BKC, int BK>
static hipError_t launch_tile(const GemmArgs& g, const OpView& va, const OpView& vb, int splits, int kc, float* part,
                              hipStream_t st) {
  constexpr int BM = 32 * WM * TM, BN = 32 * WN * TN;
  const int Nc = g.N + (g.bias_grad ? 1 : 0);
  const size_t lds = std::max(kEpiLdsBytes, (size_t)2 *
                     (plane_elems(AKC, BM, BK) * (g.a_lo ? 2 : 1) + plane_elems(BKC, BN, BK) * (g.b_lo ? 2 : 1)) *
                     sizeof(uint16_t));
  auto al = [](const void* p, uintptr_t b) { return ((uintptr_t)p % b) == 0; };
  const bool e4 = !g.cperm && (!g.C || (al(g.C, 16) && g.ldc % 4 == 0)) &&
                  (!g.Cb || (al(g.Cb, 8) && g.ldcb % 4 == 0 && g.cb_lo % 4 == 0)) && (!g.bias || al(g.bias, 16)) &&
                  (!g.mask || (al(g.mask, 8) && g.ldm % 4 == 0));
  const int evec = (e4 ? 1 : 0) | (Nc % 4 == 0 && al(part, 16) ? 2 : 0);
  hipLaunchKernelGGL((gemm_mfma_kernel<WM, WN, TM, TN, AKC, BKC, BK>),
                     dim3((Nc + BN - 1) / BN, (g.M + BM - 1) / BM, splits), dim3(256), lds, st, g, va, vb, kc,
                     splits > 1 ? part : (float*)nullptr, evec);
  return hipGetLastError();
}

template <int WM, int WN, int TM, int TN, int BK>
static hipError_t launch_layout(const GemmArgs& g, const OpView& va, const OpView& vb, bool akc, bool bkc, int splits,
                                int kc, float* part, hipStream_t st) {
  if (akc && bkc) return launch_tile<WM, WN, TM, TN, true, true, BK>(g, va, vb, splits, kc, part, st);
  if (akc) return launch_tile<WM, WN, TM, TN, true, false, BK>(g, va, vb, splits, kc, part, st);
  if (bkc) return launch_tile<WM, WN, TM, TN, false, true, BK>(g, va, vb, splits, kc, part, st);
  return launch_tile<WM, WN, TM, TN, false, false, BK>(g, va, vb, splits, kc, part, st);
}

hipError_t gemm(const GemmArgs& g, float* part, size_t part_elems, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipErrorInvalidValue;
  // A few rows with both operands contiguous in k (the layers of one or a
  // few frames): the matrix-vector kernel, which streams the weights once.
  if (!g.bias_grad && g.conv_op == 0 && g.b_lo == 0 && g.sak == 1 && g.sbk == 1 &&
      (g.M <= 16 || (g.M <= 512 && (long)g.N * g.K <= 65536))) {
    if (g.K % 8 == 0 && g.sam % 8 == 0 && g.sbn % 8 == 0 && g.a_lo % 8 == 0 && (uintptr_t)g.A % 16 == 0 &&
        (uintptr_t)g.B % 16 == 0)
      return launch_gemv_gw<8>(g, st);
    if (g.K % 4 == 0 && g.sam % 4 == 0 && g.sbn % 4 == 0 && g.a_lo % 4 == 0 && (uintptr_t)g.A % 8 == 0 &&
        (uintptr_t)g.B % 8 == 0)
      return launch_gemv_gw<4>(g, st);
  }
  const int Nc = g.N + (g.bias_grad ? 1 : 0);
  // Operand views: A rows = i, B rows = j.
  const bool akc = g.conv_op == 1 || (g.conv_op != 2 && g.sak == 1);
  const bool bkc = g.conv_op != 2 && g.sbk == 1;
  if (g.conv_op == 0 && !akc && g.sam != 1) return hipErrorInvalidValue;
  if (g.conv_op == 0 && !bkc && g.sbn != 1) return hipErrorInvalidValue;
  OpView va{g.A, g.sam, g.sak, g.M, -1, 1, 0, 0, 0, 0, 0, 0};
  OpView vb{g.B, g.sbn, g.sbk, g.N, g.bias_grad ? g.N : -1, 1, 0, 0, 0, 0, 0, 0};
  va.vw = akc ? vec_width(g.A, g.a_lo, g.sam, g.K) : vec_width(g.A, g.a_lo, g.sak, g.M);
  vb.vw = bkc ? vec_width(g.B, g.b_lo, g.sbn, g.K) : vec_width(g.B, g.b_lo, g.sbk, g.N);
  if (g.conv_op) {
    // implicit patches: 16-byte chunks of 8 channels (C a multiple of 8, planes aligned)
    const uint16_t* act = g.conv_op == 1 ? g.A : g.B;
    const long lo = g.conv_op == 1 ? g.a_lo : g.b_lo;
    if (g.conv_C % 8 != 0 || (uintptr_t)act % 16 != 0 || lo % 8 != 0 || g.conv_H < 1 || g.conv_W < 1)
      return hipErrorInvalidValue;
    OpView& v = g.conv_op == 1 ? va : vb;
    v.conv = 1; v.vw = 8;
    v.H = g.conv_H; v.W = g.conv_W; v.C = g.conv_C;
    v.Wo = (g.conv_W + 1) / 2; v.HoWo = v.Wo * ((g.conv_H + 1) / 2);
    if ((g.conv_op == 1 ? g.M : g.K) % v.HoWo != 0 || (g.conv_op == 1 ? g.K : g.N) != 9 * g.conv_C)
      return hipErrorInvalidValue;
  }
  // Tile and split (measured over the training step's fourteen products at
  // batch 256): a block's time is mostly the latency of its k steps (~1 us
  // each), so many small blocks win.  64 x 64 tiles everywhere, except the
  // narrow first-layer product (32 outputs, K = 36), which takes 128 x 32.
  // Fewer than 256 tiles leave the GPU short of blocks: split K towards
  // ~768 blocks (three per CU) of at least 2 k steps (more splits cost
  // partial traffic and a longer reduction; against ~1024 blocks a batch-256
  // training step took 3.4-3.7 % less time at ~768 on two boxes, the same at
  // ~512, and within 0.5 % of ~768 at ~640 and ~896); partials must fit `part`.  Steps of 64 k were not
  // faster (a step's time grew with its depth), so steps stay 32 deep.
  const int bk = kStepK;
  const int tile = (Nc <= 32 && g.K <= 64) ? 0 : 3;   // 0: 128 x 32, 3: 64 x 64
  const int BM = tile == 3 ? 64 : 128;
  const int BN = tile == 0 ? 32 : 64;
  const long tiles = (long)((Nc + BN - 1) / BN) * ((g.M + BM - 1) / BM);
  int splits = 1;
  if (part && tiles < 256) {
    splits = (int)std::max<long>(1, std::min<long>((768 + tiles - 1) / tiles, g.K / (bk * 2)));
    while (splits > 1 && (size_t)splits * g.M * Nc > part_elems) --splits;
  }
  const int kc = ((g.K + splits - 1) / splits + bk - 1) / bk * bk;
  splits = (g.K + kc - 1) / kc;
  const hipError_t e = tile == 0 ? launch_layout<4, 1, 1, 1, kStepK>(g, va, vb, akc, bkc, splits, kc, part, st)
                                  : launch_layout<2, 2, 1, 1, kStepK>(g, va, vb, akc, bkc, splits, kc, part, st);
  if (e != hipSuccess || splits <= 1) return e;
  const size_t MN = (size_t)g.M * Nc;
  auto al = [](const void* p, uintptr_t b) { return ((uintptr_t)p % b) == 0; };
  const bool v4 = MN % 4 == 0;
  const bool vec = v4 && Nc % 4 == 0 && !g.bias_grad && !g.cperm && (!g.C || (al(g.C, 16) && g.ldc % 4 == 0)) &&
                   (!g.Cb || (al(g.Cb, 8) && g.ldcb % 4 == 0 && g.cb_lo % 4 == 0)) && (!g.bias || al(g.bias, 16)) &&
                   (!g.mask || (al(g.mask, 8) && g.ldm % 4 == 0));
  const int G = splits >= 256 ? 64 : splits >= 64 ? 16 : 4;
  const size_t per_block = (size_t)(256 / G) * (v4 ? 4 : 1);
  const dim3 grid((unsigned)((MN + per_block - 1) / per_block));
  auto launch = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, g, splits, (const float*)part); };
  if (vec) {
    if (G == 64) launch(gemm_reduce_kernel<64, 4, true>);
    else if (G == 16) launch(gemm_reduce_kernel<16, 4, true>);
    else launch(gemm_reduce_kernel<4, 4, true>);
  } else if (v4) {
    if (G == 64) launch(gemm_reduce_kernel<64, 4, false>);
    else if (G == 16) launch(gemm_reduce_kernel<16, 4, false>);
    else launch(gemm_reduce_kernel<4, 4, false>);
  } else {
    if (G == 64) launch(gemm_reduce_kernel<64, 1, false>);
    else if (G == 16) launch(gemm_reduce_kernel<16, 1, false>);
    else launch(gemm_reduce_kernel<4, 1, false>);
  }
  return hipGetLastError();
}

// The gathers index in 32 bits: every plane must hold fewer than 2^31 elements.
static bool fits32(size_t n) { return n < ((size_t)1 << 31); }

hipError_t im2col(const uint16_t* act, int B, int H, int W, int C, uint16_t* cols, hipStream_t st) {
  const size_t rows = (size_t)B * ((H + 1) / 2) * ((W + 1) / 2);
  if (!fits32(rows * 9 * C) || !fits32((size_t)B * H * W * C)) return hipErrorInvalidValue;
  if (C % 8 == 0)
    hipLaunchKernelGGL(im2col_pair_kernel<8>, dim3(grid_for(rows * 9 * (C / 8))), dim3(256), 0, st, act, B, H, W, C,
                       cols);
  else
    hipLaunchKernelGGL(im2col_pair_kernel<1>, dim3(grid_for(rows * 9 * C)), dim3(256), 0, st, act, B, H, W, C, cols);
  return hipGetLastError();
}

hipError_t im2col_f32(const float* act, int B, int H, int W, int C, uint16_t* cols, hipStream_t st) {
  const size_t total = (size_t)B * ((H + 1) / 2) * ((W + 1) / 2) * 9;
  if (!fits32(total * C) || !fits32((size_t)B * H * W * C)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(im2col_f32_kernel, dim3(grid_for(total)), dim3(256), 0, st, act, B, H, W, C, cols);
  return hipGetLastError();
}

hipError_t col2im_mask(const float* dcols, int B, int H, int W, int C, const uint16_t* act, uint16_t* dzb,
                       hipStream_t st) {
  const size_t pix = (size_t)B * H * W;
  if (!fits32(pix * C) || !fits32((size_t)B * ((H + 1) / 2) * ((W + 1) / 2) * 9 * C)) return hipErrorInvalidValue;
  if (C % 8 == 0)
    hipLaunchKernelGGL(col2im_mask_kernel<8>, dim3(grid_for(pix * (C / 8))), dim3(256), 0, st, dcols, B, H, W, C, act,
                       dzb);
  else
    hipLaunchKernelGGL(col2im_mask_kernel<1>, dim3(grid_for(pix * C)), dim3(256), 0, st, dcols, B, H, W, C, act, dzb);
  return hipGetLastError();
}

hipError_t weights_bf16(const float* x, size_t n, const ConvPerm& cp, uint16_t* y, hipStream_t st) {
  hipLaunchKernelGGL(weights_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, n, cp, y);
  return hipGetLastError();
}

size_t mse_partials(int n) { return (size_t)(n + kMseBlock - 1) / kMseBlock; }

hipError_t mse(const float* pred, const float* target, const float* weights, int n, int n_out, uint16_t* doutb,
               float* part, hipStream_t st) {
  hipLaunchKernelGGL(mse_kernel, dim3((int)mse_partials(n)), dim3(256), 0, st, pred, target, weights, n, n_out, doutb,
                     part);
  return hipGetLastError();
}

hipError_t mse_sum(const float* part, int n, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(mse_sum_kernel, dim3(1), dim3(256), 0, st, part, (int)mse_partials(n), n, loss);
  return hipGetLastError();
}

hipError_t adam(float* w, const float* g, float* m, float* v, uint16_t* wb, const ConvPerm& cp, size_t i0, size_t n,
                float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t st) {
  if (i0 >= n) return hipSuccess;
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n - i0)), dim3(256), 0, st, w, g, m, v, wb, cp, i0, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t fill0(float* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill0_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Convolution stack of a forward pass: one block of 8 waves per frame
// instead of a gather and a product per layer.  The frame's input (rounded
// to bf16) and the activations stay in LDS; the products run on
// v_mfma_f32_32x32x16_bf16 with the activation fragments gathered straight
// from LDS (implicit patches: 8 channels of one tap per 16-byte read, or two
// taps of the 4-channel input per pair of 8-byte reads, zero in the padding)
// and the weight fragments read from the bf16 weights in patch order
// [Cout][3][3][Cin] in global memory.  Same arithmetic as the tiled products
// (pair operands as two MFMAs, FP32 accumulation, bias, ReLU, pair output),
// in another summation order.  A 32 x 32 output tile: 32 output pixels by 32
// output channels.
// Weight fragments of this lane's output channel j = 32 tn + lane % 32
// for the k steps kbeg, kbeg + 16, ... (NS of them; zero past kend and K),
// loaded once, before the activations they multiply are ready.
template <bool C4, int NS>
__device__ __forceinline__ void conv_wfrags(const uint16_t* __restrict__ wt, int K, int tn, int kbeg, int kend,
                                            int lane, uint32_t (&b)[NS][4]) {
  const uint16_t* wrow = wt + (size_t)(tn * 32 + (lane & 31)) * K;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int ks = kbeg + 16 * s, kk = ks + 8 * (lane >> 5);
    b[s][0] = b[s][1] = b[s][2] = b[s][3] = 0u;
    if constexpr (!C4) {
      if (ks < kend && kk < K) {
        const uint4 u = *reinterpret_cast<const uint4*>(wrow + kk);
        b[s][0] = u.x; b[s][1] = u.y; b[s][2] = u.z; b[s][3] = u.w;
      }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (ks < kend && kk + 4 * h < K) {
          const uint2 u = *reinterpret_cast<const uint2*>(wrow + kk + 4 * h);
          b[s][2 * h] = u.x; b[s][2 * h + 1] = u.y;
        }
      }
    }
  }
}

// Activation (A) fragment of output pixel r (valid rv) at k = kk .. kk + 7
// (patch order: k = (ky 3 + kx) C + c) from the LDS planes.  Branch-free:
// an address outside the frame is replaced by the plane's start and the
// loaded words by zero.  C: input channels (a compile-time power of two,
// or 4 for the network input, whose 8 k span two taps).
template <int C, bool PAIR>
__device__ __forceinline__ void conv_afrag(const uint16_t* in_hi, const uint16_t* in_lo, int H, int W, bool rv,
                                           int yo, int xo, int K, int kk, uint32_t (&a)[4], uint32_t (&al)[4]) {
  if constexpr (C != 4) {
    static_assert(C % 8 == 0 && (C & (C - 1)) == 0, "channel count a power of two, at least 8");
    const int tap = kk / C, c = kk % C;
    const int ky = tap / 3, kx = tap - ky * 3;
    const int y = 2 * yo + ky - 1, x = 2 * xo + kx - 1;
    const bool in = rv && kk < K && y >= 0 && y < H && x >= 0 && x < W;
    const int off = in ? (y * W + x) * C + c : 0;
    const uint4 u = *reinterpret_cast<const uint4*>(in_hi + off);
    a[0] = in ? u.x : 0u; a[1] = in ? u.y : 0u; a[2] = in ? u.z : 0u; a[3] = in ? u.w : 0u;
    if constexpr (PAIR) {
      const uint4 q = *reinterpret_cast<const uint4*>(in_lo + off);
      al[0] = in ? q.x : 0u; al[1] = in ? q.y : 0u; al[2] = in ? q.z : 0u; al[3] = in ? q.w : 0u;
    } else {
      al[0] = al[1] = al[2] = al[3] = 0u;
    }
  } else {
    // 4 channels per tap: k = kk .. kk + 7 are taps kk / 4 and kk / 4 + 1
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = kk / 4 + h;
      const int ky = t / 3, kx = t - ky * 3;
      const int y = 2 * yo + ky - 1, x = 2 * xo + kx - 1;
      const bool in = rv && t < 9 && y >= 0 && y < H && x >= 0 && x < W;
      const uint2 u = *reinterpret_cast<const uint2*>(in_hi + (in ? (y * W + x) * 4 : 0));
      a[2 * h] = in ? u.x : 0u;
      a[2 * h + 1] = in ? u.y : 0u;
    }
    al[0] = al[1] = al[2] = al[3] = 0u;
  }
}

// 32 x 32 output tile (rows i = output pixels 32 tm .., columns = the
// channels of b) over the k steps of b: activation fragments gathered from
// LDS in groups of 6 steps, then their products.
template <int C, bool PAIR, int NS>
__device__ __forceinline__ f32x16 conv_tile(const uint16_t* in_hi, const uint16_t* in_lo, int H, int W, int Wo,
                                            int M, int K, int tm, int kbeg, int kend, int lane,
                                            const uint32_t (&b)[NS][4]) {
  constexpr int G = 6;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  const int r = tm * 32 + (lane & 31);
  const bool rv = r < M;
  const int yo = rv ? r / Wo : 0, xo = rv ? r - (r / Wo) * Wo : 0;
#pragma unroll
  for (int s0 = 0; s0 < NS; s0 += G) {
    uint32_t a[G][4], al[G][4];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int ks = kbeg + 16 * (s0 + g);
      if (s0 + g < NS) conv_afrag<C, PAIR>(in_hi, in_lo, H, W, rv && ks < kend, yo, xo, K, ks + 8 * (lane >> 5), a[g], al[g]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (s0 + g < NS && kbeg + 16 * (s0 + g) < kend) {
        bf16x8 fa, fb;
        __builtin_memcpy(&fa, a[g], sizeof(fa));
        __builtin_memcpy(&fb, b[s0 + g], sizeof(fb));
        // weights as the first operand: the accumulator is the tile transposed
        // (rows = channels, columns = pixels), so a lane ends up holding four
        // consecutive channels of one pixel per group of four registers
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fb, fa, acc, 0, 0, 0);
        if constexpr (PAIR) {
          bf16x8 fl;
          __builtin_memcpy(&fl, al[g], sizeof(fl));
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fb, fl, acc, 0, 0, 0);
        }
      }
    }
  }
  return acc;
}

// Bias, ReLU and the bf16 pair of a tile's outputs (row pitch N).  Lane l
// holds pixel 32 tm + l mod 32 and, in registers 4 g .. 4 g + 3, channels
// 32 tn + 8 g + 4 (l / 32) .. + 3 (bias bq in the same order): one 8-byte
// store of each plane per group.
__device__ __forceinline__ void conv_bias4(const float* __restrict__ bias, int tn, int lane, float (&bq)[16]) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float4 u = *reinterpret_cast<const float4*>(bias + tn * 32 + 8 * g + 4 * (lane >> 5));
    bq[4 * g] = u.x; bq[4 * g + 1] = u.y; bq[4 * g + 2] = u.z; bq[4 * g + 3] = u.w;
  }
}

__device__ __forceinline__ void conv_tile_out(const f32x16& acc, int tm, int tn, int M, int N, const float (&bq)[16],
                                              uint16_t* hi, uint16_t* lo, int lane) {
  const int i = tm * 32 + (lane & 31);
  if (i >= M) return;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    uint32_t hw[2], lw[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float x0 = fmaxf(acc[4 * g + 2 * h] + bq[4 * g + 2 * h], 0.f);
      const float x1 = fmaxf(acc[4 * g + 2 * h + 1] + bq[4 * g + 2 * h + 1], 0.f);
      const uint16_t h0 = f2bf(x0), h1 = f2bf(x1);
      hw[h] = (uint32_t)h0 | ((uint32_t)h1 << 16);
      lw[h] = (uint32_t)f2bf(x0 - bf2f(h0)) | ((uint32_t)f2bf(x1 - bf2f(h1)) << 16);
    }
    const int o = i * N + tn * 32 + 8 * g + 4 * (lane >> 5);
    *reinterpret_cast<uint2*>(hi + o) = make_uint2(hw[0], hw[1]);
    *reinterpret_cast<uint2*>(lo + o) = make_uint2(lw[0], lw[1]);
  }
}

constexpr int kStackThreads = 512;
constexpr int kStackWaves = kStackThreads / 64;
constexpr int kStackSteps1 = 3;    // first convolution: K = 36
constexpr int kStackSteps2 = 18;   // second: K = 9 c1 <= 288
constexpr int kStackSteps3 = 9;    // third: a wave's share of K = 9 c2
constexpr int kStackC1 = 32;       // first layer's output channels (the second's input)

// The three convolutions of one frame (block b).  LDS (elements of 16 bits):
// the input x [S][S][4] rounded to bf16, then the first convolution's
// output pair; once the second convolution has read them (each wave keeps
// its one output tile of that layer in registers across a barrier), the
// second layer's output pair is written at the end of the LDS and the third
// layer's partial accumulators at its start.  Output: the third layer's pair
// to a3 (hi at b M3 c3, lo a3_lo on).  A wave keeps one output channel tile
// per layer (the channel tile counts divide the wave count), so its weight
// fragments and biases of all three layers are loaded once, beside the input.
// A training step also takes the first layer's patches (cols1) and the first
// and second activation pairs (a1g, a2g) to HBM for its backward pass (NULL:
// not written).
// The third layer's K is split over the waves its tiles leave free: wave w
// takes tile w mod T3 and the (w / T3)-th share of the k steps, and the
// shares are added in a fixed order.
__global__ __launch_bounds__(kStackThreads) void conv_stack_kernel(const float* __restrict__ x, int S,
                                                                  const uint16_t* __restrict__ w1,
                                                                  const float* __restrict__ b1, int c1,
                                                                  const uint16_t* __restrict__ w2,
                                                                  const float* __restrict__ b2, int c2,
                                                                  const uint16_t* __restrict__ w3,
                                                                  const float* __restrict__ b3, int c3,
                                                                  uint16_t* __restrict__ a3, long a3_lo, int lds_elems,
                                                                  uint16_t* __restrict__ cols1,
                                                                  uint16_t* __restrict__ a1g, long a1_lo,
                                                                  uint16_t* __restrict__ a2g, long a2_lo) {
  extern __shared__ __align__(16) uint16_t lds[];
  const int S1 = (S + 1) / 2, S2 = (S1 + 1) / 2, S3 = (S2 + 1) / 2;
  const int M1 = S1 * S1, M2 = S2 * S2, M3 = S3 * S3;
  const int nx = S * S * 4, n2 = M2 * c2;
  uint16_t* xin = lds;
  uint16_t* a1h = lds + ((nx + 7) & ~7);
  uint16_t* a1l = a1h + M1 * c1;
  uint16_t* a2h = lds + (lds_elems - 2 * n2);   // after the second convolution
  uint16_t* a2l = a2h + n2;
  float* part = reinterpret_cast<float*>(lds);   // after the second convolution
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const size_t b = blockIdx.x;
  const int nt1 = c1 / 32, nt2 = c2 / 32, nt3 = c3 / 32;
  const int tn1 = wave % nt1, tn2 = wave % nt2;
  const int K3 = 9 * c2, tiles3 = (M3 + 31) / 32 * nt3, nq = kStackWaves / tiles3;
  const int kq = ((K3 + 15) / 16 + nq - 1) / nq * 16;
  const int t3 = wave % tiles3, q3 = wave / tiles3;
  const bool act3 = q3 < nq;
  const int tm3 = t3 / nt3, tn3 = t3 - tm3 * nt3;
  const int kb3 = act3 ? q3 * kq : 0, ke3 = act3 ? min(K3, (q3 + 1) * kq) : 0;
  uint32_t wf1[kStackSteps1][4], wf2[kStackSteps2][4], wf3[kStackSteps3][4];
  conv_wfrags<true, kStackSteps1>(w1, 36, tn1, 0, 36, lane, wf1);
  conv_wfrags<false, kStackSteps2>(w2, 9 * kStackC1, tn2, 0, 9 * kStackC1, lane, wf2);
  conv_wfrags<false, kStackSteps3>(w3, K3, tn3, kb3, ke3, lane, wf3);
  float bias1[16], bias2[16], bias3[16];
  conv_bias4(b1, tn1, lane, bias1);
  conv_bias4(b2, tn2, lane, bias2);
  conv_bias4(b3, tn3, lane, bias3);
  {
    // float4 loads (nx a multiple of 4, x 16-byte aligned), all issued before the conversions
    constexpr int U = 4;
    const float4* xf = reinterpret_cast<const float4*>(x + b * (size_t)nx);
    const int n4 = nx / 4;
    for (int i0 = tid; i0 < n4; i0 += kStackThreads * U) {
      float4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kStackThreads;
        if (i < n4) v[u] = xf[i];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * kStackThreads;
        if (i < n4)
          *reinterpret_cast<uint2*>(xin + 4 * i) =
              make_uint2((uint32_t)f2bf(v[u].x) | ((uint32_t)f2bf(v[u].y) << 16),
                         (uint32_t)f2bf(v[u].z) | ((uint32_t)f2bf(v[u].w) << 16));
      }
    }
  }
  __syncthreads();
  if (cols1) {
    // a training step's first-layer patches [M1][9 taps][4] (its weight gradient reads them)
    uint16_t* cb = cols1 + b * (size_t)M1 * 36;
    for (int u = tid; u < M1 * 9; u += kStackThreads) {
      const int r = u / 9, tap = u - r * 9;
      const int ky = tap / 3, kx = tap - ky * 3, yo = r / S1, xo = r - yo * S1;
      const int y = 2 * yo + ky - 1, xx = 2 * xo + kx - 1;
      const bool in = y >= 0 && y < S && xx >= 0 && xx < S;
      const uint2 v = *reinterpret_cast<const uint2*>(xin + (in ? (y * S + xx) * 4 : 0));
      *reinterpret_cast<uint2*>(cb + r * 36 + tap * 4) = in ? v : make_uint2(0u, 0u);
    }
  }
  // first convolution -> LDS
  const int tiles1 = (M1 + 31) / 32 * nt1;
  for (int t = wave; t < tiles1; t += kStackWaves) {
    const int tm = t / nt1;
    const f32x16 acc = conv_tile<4, false, kStackSteps1>(xin, nullptr, S, S, S1, M1, 36, tm, 0, 36, lane, wf1);
    conv_tile_out(acc, tm, tn1, M1, c1, bias1, a1h, a1l, lane);
  }
  __syncthreads();
  if (a1g) {
    // a training step keeps the first activation pair (16-byte copies, M1 c1 a multiple of 8)
    const int n16 = M1 * c1 / 8;
    uint4* dh = reinterpret_cast<uint4*>(a1g + b * (size_t)M1 * c1);
    uint4* dl = reinterpret_cast<uint4*>(a1g + a1_lo + b * (size_t)M1 * c1);
    for (int i = tid; i < n16; i += kStackThreads) {
      dh[i] = reinterpret_cast<const uint4*>(a1h)[i];
      dl[i] = reinterpret_cast<const uint4*>(a1l)[i];
    }
  }
  // second convolution: one tile per wave (at most kStackWaves tiles), kept in registers
  const int tiles2 = (M2 + 31) / 32 * nt2;
  const int tm2 = wave / nt2;
  f32x16 acc2;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc2[v] = 0.f;
  if (wave < tiles2)
    acc2 = conv_tile<kStackC1, true, kStackSteps2>(a1h, a1l, S1, S1, S2, M2, 9 * kStackC1, tm2, 0, 9 * kStackC1, lane,
                                                   wf2);
  __syncthreads();   // x and the first activation are dead from here
  if (wave < tiles2) conv_tile_out(acc2, tm2, tn2, M2, c2, bias2, a2h, a2l, lane);
  __syncthreads();
  if (a2g) {
    const int n16 = n2 / 8;
    uint4* dh = reinterpret_cast<uint4*>(a2g + b * (size_t)n2);
    uint4* dl = reinterpret_cast<uint4*>(a2g + a2_lo + b * (size_t)n2);
    for (int i = tid; i < n16; i += kStackThreads) {
      dh[i] = reinterpret_cast<const uint4*>(a2h)[i];
      dl[i] = reinterpret_cast<const uint4*>(a2l)[i];
    }
  }
  // third convolution: shares of K, partials through LDS, output pair to HBM
  f32x16 acc3;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc3[v] = 0.f;
  if (act3) {
    if (c2 == 32)
      acc3 = conv_tile<32, true, kStackSteps3>(a2h, a2l, S2, S2, S3, M3, K3, tm3, kb3, ke3, lane, wf3);
    else
      acc3 = conv_tile<64, true, kStackSteps3>(a2h, a2l, S2, S2, S3, M3, K3, tm3, kb3, ke3, lane, wf3);
  }
  if (act3 && q3 > 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) part[((q3 * tiles3 + t3) * 16 + v) * 64 + lane] = acc3[v];
  }
  __syncthreads();
  if (act3 && q3 == 0) {
    for (int qq = 1; qq < nq; ++qq) {
#pragma unroll
      for (int v = 0; v < 16; ++v) acc3[v] += part[((qq * tiles3 + t3) * 16 + v) * 64 + lane];
    }
    uint16_t* oh = a3 + b * (size_t)M3 * c3;
    conv_tile_out(acc3, tm3, tn3, M3, c3, bias3, oh, oh + a3_lo, lane);
  }
}

// LDS of the kernel (elements of 16 bits): input and first activation pair,
// which the second activation pair (at the end) and the third layer's
// partials (at the start, floats) reuse.
static int conv_stack_lds_elems(int S, int c1, int c2, int c3) {
  const int S1 = (S + 1) / 2, S2 = (S1 + 1) / 2, S3 = (S2 + 1) / 2;
  const int tiles3 = (S3 * S3 + 31) / 32 * (c3 / 32);
  const int nq = kStackWaves / tiles3;
  const int first = ((S * S * 4 + 7) & ~7) + 2 * S1 * S1 * c1;
  const int later = 2 * nq * tiles3 * 1024 + 2 * S2 * S2 * c2;    // partials (2 elements per float) + second pair
  return (std::max(first, later) + 7) & ~7;
}

bool conv_stack_fits(int S, int c1, int c2, int c3) {
  constexpr int kMaxLdsElems = 65536 / 2;
  if (S < 2 || S > 256 || c1 != kStackC1 || (c2 != 32 && c2 != 64) || c3 < 32 || c3 % 32) return false;
  const int nt1 = c1 / 32, nt2 = c2 / 32;
  if (kStackWaves % nt1 || kStackWaves % nt2) return false;            // one channel tile per wave
  if ((9 * c1 + 15) / 16 > kStackSteps2) return false;                  // second layer's k steps
  const int S1 = (S + 1) / 2, S2 = (S1 + 1) / 2, S3 = (S2 + 1) / 2;
  if ((S2 * S2 + 31) / 32 * nt2 > kStackWaves) return false;           // second layer: one tile per wave
  const int tiles3 = (S3 * S3 + 31) / 32 * (c3 / 32);
  if (tiles3 > kStackWaves) return false;
  const int nq = kStackWaves / tiles3, ksteps3 = (9 * c2 + 15) / 16;
  if ((ksteps3 + nq - 1) / nq > kStackSteps3) return false;             // a wave's share of the third layer's
  if (2 * nq * tiles3 * 1024 + 2 * S2 * S2 * c2 > conv_stack_lds_elems(S, c1, c2, c3)) return false;
  return conv_stack_lds_elems(S, c1, c2, c3) <= kMaxLdsElems;
}

hipError_t conv_stack(const float* x, int B, int S, const uint16_t* w1, const float* b1, int c1, const uint16_t* w2,
                      const float* b2, int c2, const uint16_t* w3, const float* b3, int c3, uint16_t* a3, long a3_lo,
                      hipStream_t st, uint16_t* cols1, uint16_t* a1, long a1_lo, uint16_t* a2, long a2_lo) {
  auto al = [](const void* p, uintptr_t a) { return ((uintptr_t)p % a) == 0; };
  if (B < 1 || B > 65535 || !conv_stack_fits(S, c1, c2, c3) || !al(x, 16) || !al(w1, 8) || !al(w2, 16) ||
      !al(w3, 16) || !al(b1, 16) || !al(b2, 16) || !al(b3, 16) || !al(a3, 8) || a3_lo % 4 || !al(cols1, 8) ||
      !al(a1, 16) || a1_lo % 8 || !al(a2, 16) || a2_lo % 8)
    return hipErrorNotSupported;
  const int le = conv_stack_lds_elems(S, c1, c2, c3);
  hipLaunchKernelGGL(conv_stack_kernel, dim3(B), dim3(kStackThreads), (size_t)le * sizeof(uint16_t), st, x, S, w1, b1,
                     c1, w2, b2, c2, w3, b3, c3, a3, a3_lo, le, cols1, a1, a1_lo, a2, a2_lo);
  return hipGetLastError();
}

hipError_t prepare(const float* pupils, const float* ref, const int* valid, int nv, int B, int S, float* x,
                   hipStream_t st) {
  hipLaunchKernelGGL(prepare_kernel, dim3(B), dim3(256), 0, st, pupils, ref, valid, nv, S, x);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace pwfs
