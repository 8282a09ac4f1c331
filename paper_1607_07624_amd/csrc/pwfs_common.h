// pwfs_common.h -- device helpers shared by the pyramid line kernels (gfx950):
// scheduling fences, the quad DFT and its inverse, the quad-lane half-band projection
// and line operator, the row-pass intermediate index and LDS staging copies.
#pragma once

#include "pwfs_dft.h"

#include <cstdint>

namespace pwfs {

// Scheduling fence: keeps the machine scheduler from hoisting the table and
// field loads of later phases over the register-resident transforms.
__device__ __forceinline__ void fence() { __builtin_amdgcn_sched_barrier(0); }

// Global-address-space views (builtin vector types, which copy across address
// spaces) for pointers that pass an empty asm: a pointer laundered that way
// in the generic space would give flat accesses, and one pending flat access
// turns every later wait into a full drain of the memory counter.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const u32x4 g_u32x4;
typedef __attribute__((address_space(1))) f32x2 g_f32x2;

// LDS copies of the pyramid tables are padded so that a ds_read of a quad's
// four lanes (mix table, rows of 2E values) or of a team's two quads (input
// and output tables, halves of P values) spreads over distinct banks: both
// 2E and P complex values are multiples of the bank-set width here.
template <int E>
struct TabLds {
  static constexpr int P = 4 * E;
  static constexpr int QO = P + 4;        // offset of quad 1's half of an input / output table
  static constexpr int MS = 2 * E + 2;    // per-lane row stride of the mix table
};

// Half-band projection of the E samples held by this lane (see header), up to
// a factor 1/2 that the output table absorbs.  The forward twiddle w_l =
// w_P^{l k}, the quad mix and the conjugate twiddle are folded into
//   V_l = v_l + (A_l / 2) v_{l+1} + (B_l / 2) v_{l-1},
//   A_l = (1 - i) conj(w_l) w_{l+1},  B_l = (1 + i) conj(w_l) w_{l-1}   (lanes mod 4),
// mid[(l * E + k) * 2 + {0, 1}] = {A_l(k) / 2, B_l(k) / 2}.
template <int E>
__device__ __forceinline__ void half_band(cpx (&v)[E], const cpx* __restrict__ mid, int l) {
  Dft<E, +1>::run(v);
  fence();
  const cpx* ml = mid + l * TabLds<E>::MS;
  static_assert(E % 2 == 0, "mixes in pairs");
  static_for<0, E / 2>([&](auto h_) {
    constexpr int k = 2 * decltype(h_)::value;
    if constexpr (k % 8 == 0 && k > 0) fence();
    mix3_quad2(v[k], ml[2 * k], ml[2 * k + 1], v[k + 1], ml[2 * k + 2], ml[2 * k + 3]);   // lanes l + 1, l - 1
  });
  fence();
  Dft<E, -1>::run(v);
  fence();
}

// Full 1-D pyramid operator for one line.
//   load_in(m)  = f(x) w_N^{(2q+1) x} at x = l + 4 m (tilted input times this
//                 quad's twist, one complex product from a combined table);
//   load_x(m), load_t(m): the untilted sample at x = l + 4 m and this quad's
//                 finishing factor, minus the tilt for quad 0 and zero for
//                 quad 1, so that y_H + x t is y_H - f = -y_L or y_H;
//   outw[q * P + j] = (4/N) w_N^{-(2q+1) j}  (2/N times the 2 the half-band step leaves out).
// On return quad 0 holds -y_L(l + 4 m) and quad 1 holds y_H(l + 4 m) in v[m]
// (the sign of a whole pupil window drops out of every intensity).
template <int E, typename LoadIn, typename LoadX, typename LoadT>
__device__ __forceinline__ void line_op(cpx (&v)[E], LoadIn&& load_in, LoadX&& load_x, LoadT&& load_t,
                                        const cpx* __restrict__ mid, const cpx* __restrict__ outw,
                                        int q, int l) {
  constexpr int P = 4 * E;
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    if constexpr (m % 8 == 0 && m > 0) fence();
    v[m] = load_in(m);
  });
  fence();
  half_band<E>(v, mid, l);
  const cpx* ow = outw + q * TabLds<E>::QO + l;
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    if constexpr (m % 8 == 0 && m > 0) fence();
    cpx w = cmul(v[m], ow[4 * m]);
    w.re += swap_quads(w.re);
    w.im += swap_quads(w.im);
    v[m] = cfma(load_x(m), load_t(m), w);
  });
}

// DFT_P (P = 4E) held by a quad, lane l holding x = l + 4 m (m < E): in-lane
// DFT_E, twiddle twl[k1] = w_P^{l k1}, DFT_4 across the quad (two DPP
// butterflies); afterwards lane l holds u = k1 + E rev(l), rev = (0, 2, 1, 3).
template <int E>
__device__ __forceinline__ void dft_quad(cpx (&v)[E], const cpx* __restrict__ twl, float sA, float sB, bool l3) {
  Dft<E, +1>::run(v);
  fence();
  static_for<0, E>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    if constexpr (k % 8 == 0 && k > 0) fence();
    v[k] = quad_dft4_fwd(cmul(v[k], twl[k]), sA, sB, l3);
  });
}

__device__ __forceinline__ int rev2(int l) { return l == 1 ? 2 : (l == 2 ? 1 : l); }

// Inverse of dft_quad's steps: from lane l holding X[k1 + E rev(l)] in
// register k1 to lane l holding sum_u X[u] w_P^{-u t} at t = l + 4 m in
// register m (unnormalised): DFT_4^-1 across the quad, conjugate twiddle,
// in-lane inverse DFT_E.
template <int E>
__device__ __forceinline__ void idft_quad(cpx (&v)[E], const cpx* __restrict__ twl, float sA, float sB, bool l3) {
  static_for<0, E>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    if constexpr (k % 8 == 0 && k > 0) fence();
    v[k] = cmulc(quad_dft4_inv(v[k], sA, sB, l3), twl[k]);
  });
  fence();
  Dft<E, -1>::run(v);
}

__device__ __forceinline__ size_t rw_index(int xp, int y, int P) {
  return ((size_t)(xp >> 3) * (size_t)(P >> 2) + (size_t)(y >> 2)) * 32u + (size_t)((xp & 7) * 4 + (y & 3));
}

// Block-cooperative copy of n16 16-byte words (global -> LDS).
__device__ __forceinline__ void copy16(void* __restrict__ dst, const void* __restrict__ src, int n16,
                                       int tid, int nthreads) {
  uint4* d = reinterpret_cast<uint4*>(dst);
  const uint4* s = reinterpret_cast<const uint4*>(src);
  for (int i = tid; i < n16; i += nthreads) d[i] = s[i];
}

// Block copy of exactly 256 N 16-byte words: every load is issued before the
// first LDS write, so a thread waits for one memory round trip, not N.
template <int N>
__device__ __forceinline__ void copy16_n(void* __restrict__ dst, const void* __restrict__ src, int tid) {
  uint4* d = reinterpret_cast<uint4*>(dst);
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4 r[N];
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = s[tid + 256 * i];
  fence();
#pragma unroll
  for (int i = 0; i < N; ++i) d[tid + 256 * i] = r[i];
}

// Table [2][P] (quad 0 half, quad 1 half) -> LDS with quad 1 at TabLds::QO.
template <int E>
__device__ __forceinline__ void stage_quads(cpx* __restrict__ dst, const cpx* __restrict__ src, int tid) {
  constexpr int P = 4 * E;
  copy16(dst, src, P / 2, tid, 256);
  copy16(dst + TabLds<E>::QO, src + P, P / 2, tid, 256);
}

// Mix table [4][2E] -> LDS rows of stride TabLds::MS.
template <int E>
__device__ __forceinline__ void stage_mid(cpx* __restrict__ dst, const cpx* __restrict__ src, int tid) {
  for (int i = tid; i < 4 * E; i += 256) {
    const int l = i / E, r = i - l * E;
    reinterpret_cast<uint4*>(dst + l * TabLds<E>::MS)[r] = reinterpret_cast<const uint4*>(src + l * 2 * E)[r];
  }
}

}  // namespace pwfs
