// cnn_kernels.hip -- kernels of the learned modal reconstructor (gfx950).
//
// Every product (convolutions as im2col GEMMs, fully connected layers,
// their data and weight gradients) runs on one strided bf16 GEMM built on
// v_mfma_f32_32x32x8bf16_1k with FP32 accumulation, with an optional
// deterministic split-K (fixed-order reduction of per-split partials) and a
// fused epilogue (bias, ReLU, beta * C, FP32 and/or bf16 output).  The other
// kernels are gathers and elementwise passes: im2col, col2im in gather form
// (each input element sums its own contributions in a fixed order, no
// atomics), ReLU masks, bias-gradient column sums, the MSE loss, Adam and
// the network-input preparation from binned pupil images.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "cnn_launch.h"

namespace pwfs {
namespace cnn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bool bf_pos(uint16_t h) { return h != 0 && !(h & 0x8000u); }
__device__ __forceinline__ void split_bf(float v, uint16_t* hi, uint16_t* lo, size_t i);

// ---------------------------------------------------------------------------
// GEMM: C(i, j) = sum_k A(i, k) B(k, j), A(i, k) = A[i sam + k sak],
// B(k, j) = B[k sbk + j sbn].  Block = 4 waves, tile 64 x 64, K step 32;
// wave (wm, wn) owns the 32 x 32 sub-tile.  MFMA 32x32x8 operand layout:
// lane l holds A rows (l % 32), k = 4 (l / 32) .. +3, B columns (l % 32),
// same k; accumulator v of lane l is C(8 (v / 4) + 4 (l / 32) + v % 4, l % 32).
// With gridDim.z > 1 each z handles K range [z kc, (z+1) kc) and writes raw
// partials to part[z][M][N] (epilogue applied by gemm_reduce_kernel).
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g, int kc, float* __restrict__ part) {
  __shared__ __align__(16) uint16_t As[64][40];
  __shared__ __align__(16) uint16_t Bs[64][40];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kbeg = blockIdx.z * kc;
  const int kend = min(g.K, kbeg + kc);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    for (int e = tid; e < 2048; e += 256) {
      int ii, kk;
      if (g.sak == 1) { ii = e >> 5; kk = e & 31; } else { kk = e >> 6; ii = e & 63; }
      const int gi = i0 + ii, gk = k0 + kk;
      As[ii][kk] = (gi < g.M && gk < kend) ? g.A[(long)gi * g.sam + (long)gk * g.sak] : (uint16_t)0;
    }
    for (int e = tid; e < 2048; e += 256) {
      int jj, kk;
      if (g.sbk == 1) { jj = e >> 5; kk = e & 31; } else { kk = e >> 6; jj = e & 63; }
      const int gj = j0 + jj, gk = k0 + kk;
      Bs[jj][kk] = (gj < g.N && gk < kend) ? g.B[(long)gk * g.sbk + (long)gj * g.sbn] : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 8) {
      const bf16x4 a = *reinterpret_cast<const bf16x4*>(&As[wm * 32 + (lane & 31)][kk + 4 * (lane >> 5)]);
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(&Bs[wn * 32 + (lane & 31)][kk + 4 * (lane >> 5)]);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int j = j0 + wn * 32 + (lane & 31);
  if (j >= g.N) return;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = i0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (i >= g.M) continue;
    float x = acc[v];
    if (part) {
      part[((size_t)blockIdx.z * g.M + i) * g.N + j] = x;
      continue;
    }
    if (g.bias) x += g.bias[j];
    x *= g.alpha;
    if (g.C && g.beta != 0.f) x = fmaf(g.beta, g.C[(long)i * g.ldc + j], x);
    if (g.relu) x = fmaxf(x, 0.f);
    if (g.C) g.C[(long)i * g.ldc + j] = x;
    if (g.Cb) g.Cb[(long)i * g.ldcb + j] = f2bf(x);
  }
}

// Small-M products (at most 512 rows of A, both operands contiguous in k:
// the fully connected layers at the loop's batch sizes, the convolutions of
// one frame), C(i, j) = sum_k A[i][k] B[j][k].  Block =
// W <= 8 waves over RW = 4 columns j and BT <= 16 rows i (grid over both); thread t takes the 8-element (16-byte) k groups t, t + 64 W, ..., loads
// the RW weight rows' and the BT activation rows' groups before any product,
// and keeps the RW x BT sums.  Each wave adds its 64 lanes by recursive
// halving (a lane keeps half of its sums and trades the other half at each
// step), the W wave sums are added in wave order through LDS (fixed order),
// then the epilogue of gemm_bf16_kernel.  Columns and rows past the ends are
// clamped to the last one for loading (in bounds, never stored).  The
// weights stream from HBM once, instead of through 64 x 64 MFMA tiles that
// are 1 / 64 full at one row and need a split-K pass to fill the GPU.
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
  float v[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) v[e] = 0.f;
  for (int q = tid; q < ng; q += 64 * W) {
    V wr[RW], ar[BT];
#pragma unroll
    for (int r = 0; r < RW; ++r)
      wr[r] = reinterpret_cast<const V*>(g.B + (long)min(j0 + r, g.N - 1) * g.sbn)[q];
#pragma unroll
    for (int b = 0; b < BT; ++b)
      ar[b] = reinterpret_cast<const V*>(g.A + (long)min(i0 + b, g.M - 1) * g.sam)[q];
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
      if (g.bias) x += g.bias[j];
      x *= g.alpha;
      if (g.C && g.beta != 0.f) x = fmaf(g.beta, g.C[(long)i * g.ldc + j], x);
      if (g.relu) x = fmaxf(x, 0.f);
      if (g.C) g.C[(long)i * g.ldc + j] = x;
      if (g.Cb) g.Cb[(long)i * g.ldcb + j] = f2bf(x);
    }
  }
}

// Sum of split-K partials in split order, then the epilogue.
__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmArgs g, int splits, const float* __restrict__ part) {
  const size_t idx = blockIdx.x * (size_t)256 + threadIdx.x;
  const size_t MN = (size_t)g.M * g.N;
  if (idx >= MN) return;
  const int i = (int)(idx / g.N), j = (int)(idx % g.N);
  float x = 0.f;
  for (int z = 0; z < splits; ++z) x += part[(size_t)z * MN + idx];
  if (g.bias) x += g.bias[j];
  x *= g.alpha;
  if (g.C && g.beta != 0.f) x = fmaf(g.beta, g.C[(long)i * g.ldc + j], x);
  if (g.relu) x = fmaxf(x, 0.f);
  if (g.C) g.C[(long)i * g.ldc + j] = x;
  if (g.Cb) g.Cb[(long)i * g.ldcb + j] = f2bf(x);
}

// ---------------------------------------------------------------------------
// im2col for a 3x3 stride-2 pad-1 convolution, NHWC input:
// cols[(b, yo, xo)][c * 9 + ky * 3 + kx] = act[b][2 yo + ky - 1][2 xo + kx - 1][c] (0 outside).
// (Also from an FP32 input, rounded to bf16 as to_bf16_kernel rounds it: the
// network input's conversion and its im2col in one pass.)
__device__ __forceinline__ uint16_t as_bf16(uint16_t h) { return h; }
__device__ __forceinline__ uint16_t as_bf16(float f) { return f2bf(f); }

template <typename T>
__global__ __launch_bounds__(256) void im2col_kernel(const T* __restrict__ act, int B, int H, int W,
                                                     int C, uint16_t* __restrict__ cols) {
  const int Ho = (H + 1) / 2, Wo = (W + 1) / 2;
  const size_t K9 = (size_t)C * 9;
  const size_t total = (size_t)B * Ho * Wo * K9;
  for (size_t idx = blockIdx.x * (size_t)256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const size_t row = idx / K9;
    const int col = (int)(idx - row * K9);
    const int c = col / 9, r9 = col - c * 9, ky = r9 / 3, kx = r9 - ky * 3;
    const int b = (int)(row / ((size_t)Ho * Wo));
    const int rem = (int)(row - (size_t)b * Ho * Wo);
    const int yo = rem / Wo, xo = rem - yo * Wo;
    const int y = 2 * yo + ky - 1, x = 2 * xo + kx - 1;
    cols[idx] = (y >= 0 && y < H && x >= 0 && x < W) ? as_bf16(act[(((size_t)b * H + y) * W + x) * C + c])
                                                      : (uint16_t)0;
  }
}

// Gradient of im2col (gather form) fused with the ReLU mask of the layer's
// forward output act: dz[b][y][x][c] = (act > 0) * sum over the (ky, kx)
// whose output pixel (yo, xo) = ((y + 1 - ky) / 2, (x + 1 - kx) / 2) exists,
// in ky-major order.  Writes FP32 and bf16 hi/lo (lo at dzb + B H W C).
__global__ __launch_bounds__(256) void col2im_mask_kernel(const float* __restrict__ dcols, int B, int H, int W,
                                                          int C, const uint16_t* __restrict__ act,
                                                          float* __restrict__ dz, uint16_t* __restrict__ dzb) {
  const int Ho = (H + 1) / 2, Wo = (W + 1) / 2;
  const size_t total = (size_t)B * H * W * C;
  for (size_t idx = blockIdx.x * (size_t)256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const int c = (int)(idx % C);
    const size_t pix = idx / C;
    const int x = (int)(pix % W);
    const size_t t2 = pix / W;
    const int y = (int)(t2 % H);
    const int b = (int)(t2 / H);
    float s = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
      const int yy = y + 1 - ky;
      if (yy < 0 || (yy & 1) || (yy >> 1) >= Ho) continue;
      for (int kx = 0; kx < 3; ++kx) {
        const int xx = x + 1 - kx;
        if (xx < 0 || (xx & 1) || (xx >> 1) >= Wo) continue;
        s += dcols[(((size_t)b * Ho + (yy >> 1)) * Wo + (xx >> 1)) * (size_t)(C * 9) + c * 9 + ky * 3 + kx];
      }
    }
    const float gv = bf_pos(act[idx]) ? s : 0.f;
    dz[idx] = gv;
    split_bf(gv, dzb, dzb + total, idx);
  }
}

// Split of an FP32 value into bf16 hi + lo (hi = bf16(v), lo = bf16(v - hi)):
// a product on the pair keeps ~16 significant bits of v.
__device__ __forceinline__ void split_bf(float v, uint16_t* hi, uint16_t* lo, size_t i) {
  const uint16_t h = f2bf(v);
  hi[i] = h;
  lo[i] = f2bf(v - bf2f(h));
}

// dz = (act > 0) * g, FP32 and bf16 hi/lo (lo written at dzb + n).
__global__ __launch_bounds__(256) void relu_mask_kernel(const float* __restrict__ g, const uint16_t* __restrict__ act,
                                                        size_t n, float* __restrict__ dz, uint16_t* __restrict__ dzb) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float v = bf_pos(act[i]) ? g[i] : 0.f;
    dz[i] = v;
    split_bf(v, dzb, dzb + n, i);
  }
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ x, size_t n, uint16_t* __restrict__ y) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) y[i] = f2bf(x[i]);
}

// Column sums of dz [rows][N] (bias gradient): one block per column, fixed
// per-thread strides then a fixed tree.
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ dz, int rows, int N, float* __restrict__ out) {
  __shared__ float red[256];
  const int j = blockIdx.x, tid = threadIdx.x;
  float s = 0.f;
  for (int r = tid; r < rows; r += 256) s += dz[(size_t)r * N + j];
  red[tid] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) out[j] = red[0];
}

// Weighted MSE loss (one block): loss = sum_i w[i / n_out] (p_i - t_i)^2 / n,
// gradient 2 w (p - t) / n in FP32 and bf16 hi/lo (lo at doutb + n); w = 1
// when weights is NULL.
__global__ __launch_bounds__(1024) void mse_kernel(const float* __restrict__ pred, const float* __restrict__ target,
                                                   const float* __restrict__ weights, int n, int n_out,
                                                   float* __restrict__ dout, uint16_t* __restrict__ doutb,
                                                   float* __restrict__ loss) {
  __shared__ float red[1024];
  const int tid = threadIdx.x;
  const float inv = 1.f / (float)n;
  float s = 0.f;
  for (int i = tid; i < n; i += 1024) {
    const float d = pred[i] - target[i];
    const float w = weights ? weights[i / n_out] : 1.f;
    s = fmaf(w * d, d, s);
    const float gv = 2.f * w * d * inv;
    dout[i] = gv;
    split_bf(gv, doutb, doutb + n, i);
  }
  red[tid] = s;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0 && loss) *loss = red[0] * inv;
}

// Adam on the FP32 master weights; refreshes the bf16 copy.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                                   float* __restrict__ v, uint16_t* __restrict__ wb, size_t n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
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

hipError_t gemm(const GemmArgs& g, float* part, size_t part_elems, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipErrorInvalidValue;
  // Up to 512 rows with both operands contiguous in k (the fully connected
  // layers, and the convolutions of a single frame): the matrix-vector kernel,
  // one launch and no split-K pass (measured faster than the MFMA tiles up to
  // 16 frames; at 64 frames every convolution has more rows and keeps them).
  if (g.M <= 512 && g.sak == 1 && g.sbk == 1) {
    if (g.K % 8 == 0 && g.sam % 8 == 0 && g.sbn % 8 == 0 && (uintptr_t)g.A % 16 == 0 && (uintptr_t)g.B % 16 == 0)
      return launch_gemv_gw<8>(g, st);
    if (g.K % 4 == 0 && g.sam % 4 == 0 && g.sbn % 4 == 0 && (uintptr_t)g.A % 8 == 0 && (uintptr_t)g.B % 8 == 0)
      return launch_gemv_gw<4>(g, st);
  }
  const int bx = (g.N + 63) / 64, by = (g.M + 63) / 64;
  const long blocks = (long)bx * by;
  int splits = 1;
  if (part && blocks < 512 && g.K >= 256) {
    splits = (int)std::min<long>((512 + blocks - 1) / blocks, (g.K + 127) / 128);
    while (splits > 1 && (size_t)splits * g.M * g.N > part_elems) --splits;
  }
  const int kc = ((g.K + splits - 1) / splits + 31) / 32 * 32;
  splits = (g.K + kc - 1) / kc;
  if (splits <= 1) {
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3(bx, by, 1), dim3(256), 0, st, g, g.K, (float*)nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3(bx, by, splits), dim3(256), 0, st, g, kc, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t MN = (size_t)g.M * g.N;
  hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, g, splits,
                     (const float*)part);
  return hipGetLastError();
}

hipError_t im2col(const uint16_t* act, int B, int H, int W, int C, uint16_t* cols, hipStream_t st) {
  const size_t total = (size_t)B * ((H + 1) / 2) * ((W + 1) / 2) * C * 9;
  hipLaunchKernelGGL(im2col_kernel<uint16_t>, dim3(grid_for(total)), dim3(256), 0, st, act, B, H, W, C, cols);
  return hipGetLastError();
}

hipError_t im2col_f32(const float* act, int B, int H, int W, int C, uint16_t* cols, hipStream_t st) {
  const size_t total = (size_t)B * ((H + 1) / 2) * ((W + 1) / 2) * C * 9;
  hipLaunchKernelGGL(im2col_kernel<float>, dim3(grid_for(total)), dim3(256), 0, st, act, B, H, W, C, cols);
  return hipGetLastError();
}

hipError_t col2im_mask(const float* dcols, int B, int H, int W, int C, const uint16_t* act, float* dz,
                       uint16_t* dzb, hipStream_t st) {
  const size_t total = (size_t)B * H * W * C;
  hipLaunchKernelGGL(col2im_mask_kernel, dim3(grid_for(total)), dim3(256), 0, st, dcols, B, H, W, C, act, dz, dzb);
  return hipGetLastError();
}

hipError_t relu_mask(const float* g, const uint16_t* act, size_t n, float* dz, uint16_t* dzb, hipStream_t st) {
  hipLaunchKernelGGL(relu_mask_kernel, dim3(grid_for(n)), dim3(256), 0, st, g, act, n, dz, dzb);
  return hipGetLastError();
}

hipError_t to_bf16(const float* x, size_t n, uint16_t* y, hipStream_t st) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, n, y);
  return hipGetLastError();
}

hipError_t colsum(const float* dz, int rows, int N, float* out, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3(N), dim3(256), 0, st, dz, rows, N, out);
  return hipGetLastError();
}

hipError_t mse(const float* pred, const float* target, const float* weights, int n, int n_out, float* dout,
               uint16_t* doutb, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, st, pred, target, weights, n, n_out, dout, doutb, loss);
  return hipGetLastError();
}

hipError_t adam(float* w, const float* g, float* m, float* v, uint16_t* wb, size_t n, float lr, float b1, float b2,
                float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, st, w, g, m, v, wb, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t fill0(float* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill0_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t prepare(const float* pupils, const float* ref, const int* valid, int nv, int B, int S, float* x,
                   hipStream_t st) {
  hipLaunchKernelGGL(prepare_kernel, dim3(B), dim3(256), 0, st, pupils, ref, valid, nv, S, x);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace pwfs
