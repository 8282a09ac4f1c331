// pwfs_fstop.hip -- modulated pyramid with a circular field stop (gfx950).
//
// A focal-plane stop is a disc, not a product of an x and a y factor, so the
// separable line operator of pwfs_kernels.hip does not apply.  Per modulation
// point k the 2-D transform runs in three pruned passes on the N = 4P grid,
// in pupil coordinates (field on [0, P)^2; the embedding offset of the full
// grid only moves the output windows, which are then at rows and columns
// 3P + t (side -) and P + t (side +), t < P):
//   rows     Z[u][y] = sum_x E(x, y) r_a(x) r_b(y) w_N^{u x} for every u < N:
//            four DFT_P of E w_N^{u1 x}, u = 4 u2 + u1, one per quad;
//   columns  F(u, v) = sum_y Z[u][y] w_N^{v y} (four quads per column,
//            v = 4 v2 + v1), G = F x pyramid mask x stop, and the inverse
//            along v pruned to the two row windows:
//              c_v1[t] = (1/N) w_N^{-v1 t} sum_v2 G[4 v2 + v1] w_P^{-v2 t},
//              side - = sum_v1 (-i)^v1 c_v1,  side + = sum_v1 i^v1 c_v1
//            (w_N^{-3P v1} = (-i)^v1, w_N^{-P v1} = i^v1); the four quads of a
//            column combine through two lane swizzles;
//   output   the same inverse along u on every row of the two row windows,
//            |.|^2 summed over a chunk of modulation points into a partial
//            image [4][P][P] (q = x side + 2 y side, the separable path's order).
// The chunk sum, the binning or rebin, the detector and the slopes are those
// of the separable path.  The quad DFT keeps E = P / 4 values per lane
// (P = 32, 64, 160).
#include "pwfs_common.h"
#include "pwfs_launch.h"

#include <algorithm>
#include <cstdint>

namespace pwfs {

// Lane i reads lane i ^ 8 (ds_swizzle bit mode, inside each group of 32).
__device__ __forceinline__ float swap_oct(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x201F));
}
__device__ __forceinline__ cpx sum_quads(cpx a) {   // sum over the four quads of a 16-lane group
  a.re += swap_quads(a.re);
  a.im += swap_quads(a.im);
  a.re += swap_oct(a.re);
  a.im += swap_oct(a.im);
  return a;
}

// Rows: one quad per (pupil row y, residue u1); grid (P / 16, K, B).
template <int E>
__global__ __launch_bounds__(256) void fs_rows_kernel(const cpx* __restrict__ field, const cpx* __restrict__ rx,
                                                      const cpx* __restrict__ ry, const cpx* __restrict__ tw4n,
                                                      const cpx* __restrict__ twp, int r2max, int K,
                                                      cpx* __restrict__ Z) {
  constexpr int P = 4 * E, N = 4 * P;
  const int tid = threadIdx.x, l = tid & 3;
  const int g = blockIdx.x * 64 + (tid >> 2);
  const int y = g >> 2, u1 = g & 3;
  const int k = blockIdx.y;
  const size_t fk = (size_t)blockIdx.z * K + k;
  const cpx* frow = field + ((size_t)blockIdx.z * P + y) * (size_t)P + l;
  const cpx* ra = rx + (size_t)k * P + l;
  const cpx* tw = tw4n + (size_t)u1 * P + l;
  const cpx rb = ry[(size_t)k * P + y];
  cpx v[E];
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    v[m] = cmul(cmul(frow[4 * m], ra[4 * m]), tw[4 * m]);
  });
  fence();
  const float sA = (l & 2) ? -1.f : 1.f, sB = (l & 1) ? -1.f : 1.f;
  dft_quad<E>(v, twp + l * E, sA, sB, l == 3);
  cpx* zc = Z + fk * (size_t)N * P + y;
  const int ub = 4 * E * rev2(l) + u1;               // u = 4 (k1 + E rev(l)) + u1
  static_for<0, E>([&](auto k_) {
    constexpr int k1 = decltype(k_)::value;
    const int uu = ub + 4 * k1;
    const int uus = uu < N / 2 ? uu : uu - N;
    if (uus * uus <= r2max) zc[(size_t)uu * P] = cmul(v[k1], rb);   // columns the stop blocks are never read
  });
}

// Columns: a block holds 16 adjacent columns (4 per wave, four quads v1 per
// column); grid (N / 16, K, B).  Output W[fk][w][t][u], w = 0 for the rows
// of side -, staged through LDS so that each row segment of 16 columns is
// written at once.  A column the stop blocks entirely (u_s^2 > R^2) is zero
// and is neither read nor transformed.
template <int E>
__global__ __launch_bounds__(256) void fs_cols_kernel(const cpx* __restrict__ Z, const cpx* __restrict__ tw4n,
                                                      const cpx* __restrict__ twp, const cpx* __restrict__ twi,
                                                      const cpx* __restrict__ py, int r2max, int K,
                                                      cpx* __restrict__ W) {
  constexpr int P = 4 * E, N = 4 * P;
  __shared__ __align__(16) cpx tile[2 * P * 16];
  __shared__ __align__(16) cpx s_twp[4 * E];
  __shared__ __align__(16) cpx s_tw4n[4 * P];
  __shared__ __align__(16) cpx s_twi[4 * P];
  __shared__ __align__(16) cpx s_py[N];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l = lane & 3;
  for (int i = tid; i < 4 * E; i += 256) s_twp[i] = twp[i];
  for (int i = tid; i < 4 * P; i += 256) {
    s_tw4n[i] = tw4n[i];
    s_twi[i] = twi[i];
  }
  for (int i = tid; i < N; i += 256) s_py[i] = py[i];
  __syncthreads();
  const int qd = lane >> 2;
  const int c16 = wave * 4 + (qd >> 2);
  const int v1 = qd & 3;
  const int u = blockIdx.x * 16 + c16;
  const size_t fk = (size_t)blockIdx.z * K + blockIdx.y;
  const int us = u < N / 2 ? u : u - N;
  const int w = v1 & 1, msel = v1 >> 1;
  if (us * us > r2max) {
    // The stop blocks this whole column (the same for its four quads).
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      if ((m & 1) == msel) tile[(w * P + l + 4 * m) * 16 + c16] = cpx{0.f, 0.f};
    });
  } else {
    const cpx* zc = Z + (fk * N + u) * (size_t)P + l;
    const cpx* tw = s_tw4n + v1 * P + l;
    cpx v[E];
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      v[m] = cmul(zc[4 * m], tw[4 * m]);
    });
    fence();
    const float sA = (l & 2) ? -1.f : 1.f, sB = (l & 1) ? -1.f : 1.f;
    const bool l3 = l == 3;
    dft_quad<E>(v, s_twp + l * E, sA, sB, l3);
    // lane l, register k1: v = 4 (k1 + E rev(l)) + v1
    const cpx pu = s_py[u];
    const int vb = 4 * E * rev2(l) + v1;
    static_for<0, E>([&](auto k_) {
      constexpr int k1 = decltype(k_)::value;
      if constexpr (k1 % 8 == 0 && k1 > 0) fence();
      const int vv = vb + 4 * k1;
      const int vs = vv < N / 2 ? vv : vv - N;
      const float in = (us * us + vs * vs <= r2max) ? 1.f : 0.f;
      const cpx g = cmul(v[k1], cmul(s_py[vv], pu));
      v[k1] = {in * g.re, in * g.im};
    });
    fence();
    asm volatile("" ::: "memory");   // the quad twiddles are read again from LDS, not kept in registers
    idft_quad<E>(v, s_twp + l * E, sA, sB, l3);
    // lane l, register m: t = l + 4 m
    const cpx* ti = s_twi + v1 * P + l;
    const float s1 = (v1 & 1) ? -1.f : 1.f;
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      if constexpr (m % 8 == 0 && m > 0) fence();
      const cpx d = cmul(v[m], ti[4 * m]);
      const cpx a = sum_quads(d);
      const cpx b = sum_quads(cpx{s1 * d.re, s1 * d.im});
      if ((m & 1) == msel) tile[(w * P + l + 4 * m) * 16 + c16] = w ? b : a;
    });
  }
  __syncthreads();
  cpx* wb = W + fk * (size_t)(2 * P) * N + (size_t)blockIdx.x * 16;
  for (int i = tid; i < 2 * P * 16; i += 256) wb[(size_t)(i >> 4) * N + (i & 15)] = tile[i];
}

// Output rows: one quad per (row r of the two row windows, residue u1), a
// block holds 16 rows; loops over a chunk of modulation points; grid
// (2P / 16, n_chunks, B).  Works on conjugates (the forward quad DFT of the
// conjugated row is the conjugate of the inverse); |.|^2 is unchanged.
template <int E>
__global__ __launch_bounds__(256) void fs_out_kernel(const cpx* __restrict__ W, const cpx* __restrict__ twp,
                                                     const cpx* __restrict__ twi, int K, int k_chunk, int n_chunks,
                                                     float* __restrict__ partial) {
  constexpr int P = 4 * E, N = 4 * P;
  __shared__ __align__(16) cpx s_twp[4 * E];
  __shared__ __align__(16) cpx s_twi[4 * P];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l = lane & 3;
  for (int i = tid; i < 4 * E; i += 256) s_twp[i] = twp[i];
  for (int i = tid; i < 4 * P; i += 256) s_twi[i] = twi[i];
  __syncthreads();
  const int qd = lane >> 2;
  const int r = blockIdx.x * 16 + wave * 4 + (qd >> 2);
  const int u1 = qd & 3;
  const int chunk = blockIdx.y;
  const size_t fr = blockIdx.z;
  const int kb = chunk * k_chunk, ke = min(kb + k_chunk, K);
  const float sA = (l & 2) ? -1.f : 1.f, sB = (l & 1) ? -1.f : 1.f;
  const bool l3 = l == 3;
  const float s1 = (u1 & 1) ? -1.f : 1.f;
  const int xw = u1 & 1, msel = u1 >> 1;             // this quad keeps side xw, registers k1 = 2 j + msel
  const cpx* ti = s_twi + u1 * P + E * rev2(l);       // t = k1 + E rev(l)
  float acc[E / 2];
  static_for<0, E / 2>([&](auto j_) { acc[decltype(j_)::value] = 0.f; });
  for (int k = kb; k < ke; ++k) {
    // Tables are read from LDS in every iteration (kept out of registers).
    asm volatile("" ::: "memory");
    const cpx* row = W + ((fr * K + k) * (size_t)(2 * P) + r) * N + 4 * l + u1;   // u = 16 m + 4 l + u1
    cpx v[E];
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      const cpx c = row[16 * m];
      v[m] = cpx{c.re, -c.im};
    });
    fence();
    dft_quad<E>(v, s_twp + l * E, sA, sB, l3);
    static_for<0, E / 2>([&](auto j_) {
      constexpr int j = decltype(j_)::value;
      if constexpr (j % 4 == 0 && j > 0) fence();
      const cpx d0 = cmulc(v[2 * j], ti[2 * j]);
      const cpx d1 = cmulc(v[2 * j + 1], ti[2 * j + 1]);
      const cpx a0 = sum_quads(d0), a1 = sum_quads(d1);
      const cpx b0 = sum_quads(cpx{s1 * d0.re, s1 * d0.im}), b1 = sum_quads(cpx{s1 * d1.re, s1 * d1.im});
      const cpx x0 = xw ? b0 : a0, x1 = xw ? b1 : a1;
      const cpx x = msel ? x1 : x0;
      acc[j] = fmaf(x.re, x.re, fmaf(x.im, x.im, acc[j]));
    });
  }
  const int yw = r >= P ? 1 : 0;
  const int trow = r - yw * P;
  float* dst = partial + ((fr * n_chunks + chunk) * 4 + (size_t)(xw + 2 * yw)) * (size_t)P * P + (size_t)trow * P +
               E * rev2(l) + msel;
  static_for<0, E / 2>([&](auto j_) {
    constexpr int j = decltype(j_)::value;
    dst[2 * j] = acc[j];
  });
}

template <int E>
static hipError_t launch_fs_e(const MeasureArgs& a, hipStream_t st) {
  constexpr int P = 4 * E, N = 4 * P;
  hipError_t e;
  if ((e = launch_k(fs_rows_kernel<E>, dim3(P / 16, a.K, a.B), dim3(256), 0, st, nullptr, a.tev[1],
                    (const cpx*)a.field, a.fs_rx, a.fs_ry, a.fs_tw4n, a.fs_twp, a.fs_r2max, a.K, a.fs_Z)) != hipSuccess)
    return e;
  if ((e = launch_k(fs_cols_kernel<E>, dim3(N / 16, a.K, a.B), dim3(256), 0, st, a.tev[2], nullptr,
                    (const cpx*)a.fs_Z, a.fs_tw4n, a.fs_twp, a.fs_twi, a.fs_py, a.fs_r2max, a.K, a.fs_W)) != hipSuccess)
    return e;
  return launch_k(fs_out_kernel<E>, dim3(2 * P / 16, a.n_chunks, a.B), dim3(256), 0, st, nullptr, a.tev[3],
                  (const cpx*)a.fs_W, a.fs_twp, a.fs_twi, a.K, a.k_chunk, a.n_chunks, a.partial);
}

hipError_t launch_fstop_passes(const MeasureArgs& a, hipStream_t st) {
  switch (a.P) {
    case 32: return launch_fs_e<8>(a, st);
    case 64: return launch_fs_e<16>(a, st);
    case 160: return launch_fs_e<40>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pwfs
