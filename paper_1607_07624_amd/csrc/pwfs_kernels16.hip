// pwfs_kernels16.hip -- pyramid line kernels for long lines, P = 16 E (P = 128, 480), gfx950.
#include "pwfs_common.h"
#include "pwfs_field.h"
#include "pwfs_launch.h"

#include <algorithm>
#include <cstdint>

namespace pwfs {

// ===========================================================================
// Long lines, P = 16 E (P = 128, 480; at P = 160 an alternative to the quad
// form for small batches).  The four lanes of the quad form above
// become four 4-lane subgroups: a projection is held by a row of 16 lanes,
// lane 4 l1 + l2 holding the samples x = l1 + 4 l2 + 16 m (m < E), so that
// "outer lane" l1 holds x = l1 + 4 m' with m' = l2 + 4 m as before.  Its
// DFT over m' (length 4E) is done by the subgroup in four steps:
//   in-lane DFT_E over m  ->  twiddle w_{4E}^{l2 k1}  ->  DFT_4 across the
//   subgroup (two DPP radix-2 butterflies; lane l2 ends with t' = k1 + E rev(l2))
// then the folded 3-tap mix of the quad form runs between outer lanes
// l1 +- 1, i.e. lanes +-4 of the row (DPP row rotations), with its
// coefficients tabulated per (lane, k1); then the same four steps inverted.
// A line takes 32 lanes, the two projections exchanging halves with
// ds_swizzle (lane ^ 16).

template <int E>
struct Tab16 {
  static constexpr int P = 16 * E;
  static constexpr int QO = P + 16;   // offset of projection 1's half of an input / output table (other bank half)
  static constexpr int MS = 2 * E + 2;  // per-lane row stride of the mix table
  static constexpr int TS = E + 1;    // per-l2 row stride of the subgroup twiddles
  static constexpr int LDP = P + 16;  // field row stride in the row pass (two rows per wave on opposite bank halves)
  static constexpr int GS = 40;       // y-group stride of the staged columns (column pass)
};

// mid [16][E][2] = (A/2, B/2) for lane 4 l1 + l2 at t' = k1 + E rev(l2);
// tw [4][E] = w_{4E}^{l2 k1}; outw [2][P].
template <int E>
__device__ __forceinline__ void stage_tables16(cpx* __restrict__ s_mid, cpx* __restrict__ s_tw,
                                               cpx* __restrict__ s_out, const cpx* __restrict__ mid,
                                               const cpx* __restrict__ tw, const cpx* __restrict__ outw, int tid,
                                               int nthreads) {
  using T = Tab16<E>;
  for (int i = tid; i < 16 * E; i += nthreads) {
    const int row = i / E, k = i - row * E;
    reinterpret_cast<uint4*>(s_mid + row * T::MS)[k] = reinterpret_cast<const uint4*>(mid + row * 2 * E)[k];
  }
  for (int i = tid; i < 4 * E; i += nthreads) {
    const int row = i / E, k = i - row * E;
    s_tw[row * T::TS + k] = tw[row * E + k];
  }
  copy16(s_out, outw, T::P / 2, tid, nthreads);
  copy16(s_out + T::QO, outw + T::P, T::P / 2, tid, nthreads);
}

// Half-band projection held by a 16-lane row (see above), up to the factor
// 1/2 that the output table absorbs.  ml: this lane's mix row, tl: its twiddles.
template <int E>
__device__ __forceinline__ void half_band16(cpx (&v)[E], const cpx* __restrict__ ml, const cpx* __restrict__ tl,
                                            float sA, float sB, bool l3) {
  Dft<E, +1>::run(v);
  fence();
  static_for<0, E>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    if constexpr (k % 8 == 0 && k > 0) fence();
    v[k] = quad_dft4_fwd(cmul(v[k], tl[k]), sA, sB, l3);
  });
  fence();
  static_for<0, E>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    if constexpr (k % 8 == 0 && k > 0) fence();
    v[k] = mix3_row4(v[k], ml[2 * k], ml[2 * k + 1]);   // outer lanes l1 + 1, l1 - 1
  });
  fence();
  static_for<0, E>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    if constexpr (k % 8 == 0 && k > 0) fence();
    v[k] = cmulc(quad_dft4_inv(v[k], sA, sB, l3), tl[k]);
  });
  fence();
  Dft<E, -1>::run(v);
  fence();
}

// Full 1-D pyramid operator of one line held by a 32-lane team.
//   load_in(m) = f(x) w_N^{(2q+1) x} at x = l1 + 4 l2 + 16 m; load_x(m), load_t(m):
//   the untilted sample and this projection's finishing factor (minus the tilt
//   for projection 0, zero for projection 1); ow = outw + q QO + l1 + 4 l2.
// On return projection 0 holds -y_L(x) and projection 1 holds y_H(x) in v[m].
template <int E, typename LoadIn, typename LoadX, typename LoadT>
__device__ __forceinline__ void line_op16(cpx (&v)[E], LoadIn&& load_in, LoadX&& load_x, LoadT&& load_t,
                                          const cpx* __restrict__ ml, const cpx* __restrict__ tl,
                                          const cpx* __restrict__ ow, float sA, float sB, bool l3) {
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    if constexpr (m % 8 == 0 && m > 0) fence();
    v[m] = load_in(m);
  });
  fence();
  half_band16<E>(v, ml, tl, sA, sB, l3);
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    if constexpr (m % 8 == 0 && m > 0) fence();
    cpx w = cmul(v[m], ow[16 * m]);
    w.re += swap_halves(w.re);
    w.im += swap_halves(w.im);
    v[m] = cfma(load_x(m), load_t(m), w);
  });
}

// Row pass, long lines.  Block = 4 waves = 8 pupil rows of one frame (two
// 32-lane teams per wave), looping over a chunk of distinct x tilts.  With
// kField the block forms the field of its 8 rows from the OPD and the
// amplitude itself (pupil_field, the arithmetic of field_kernel) instead of
// reading it from a field pass: at n_pupil 128 and 160 the 1,024-1,280
// sincos per block cost less than a separate launch, which matters for the
// single-frame calls this form serves; at 480 the field pass stays.
template <int E, bool kField>
__global__ __launch_bounds__(256) void row_pass16_kernel(
    const cpx* __restrict__ fieldg, const float* __restrict__ opd, const float* __restrict__ amp, double kphase,
    int fp32_phase, const cpx* __restrict__ in_a, const cpx* __restrict__ f_a, const cpx* __restrict__ mid,
    const cpx* __restrict__ tw, const cpx* __restrict__ outw, cpx* __restrict__ Rw, int n_a, int a_chunk) {
  using T = Tab16<E>;
  constexpr int P = T::P;
  __shared__ __align__(16) cpx field[8 * T::LDP];
  __shared__ __align__(16) cpx s_in[2 * T::QO];
  __shared__ __align__(16) cpx s_f[2 * T::QO];   // [projection 0: -tilt | projection 1: 0]
  __shared__ __align__(16) cpx s_mid[16 * T::MS];
  __shared__ __align__(16) cpx s_tw[4 * T::TS];
  __shared__ __align__(16) cpx s_out[2 * T::QO];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int team = lane >> 5, q = (lane >> 4) & 1, l16 = lane & 15, l1 = l16 >> 2, l2 = l16 & 3;
  const int yb = blockIdx.x * 8;
  const int a0 = blockIdx.y * a_chunk;
  const size_t fr = blockIdx.z;
  // Up to n_pupil 170 the tilt tables (3 P / 2 16-byte words) take one word
  // per thread and are loaded one x tilt ahead, as in the 8-lane row pass;
  // at n_pupil 480 the extra registers would cost a wave per SIMD, so those
  // tables are copied at the top of each tilt.
  constexpr int H = P / 2;
  constexpr bool kPrefetch = 3 * H <= 256;
  const int tw3 = tid % (3 * H);
  const int tab_part = tw3 / H, tab_w = tw3 - (tw3 / H) * H;
  u32x4* const tab_dst = reinterpret_cast<u32x4*>(
      tab_part == 0 ? s_in : (tab_part == 1 ? s_in + T::QO : s_f)) + tab_w;
  auto tab_src = [&](int ia) {
    const cpx* base = tab_part < 2 ? in_a + (size_t)ia * 2 * P + tab_part * P : f_a + (size_t)ia * P;
    return (g_u32x4*)base + tab_w;
  };
  u32x4 tab_next = {0u, 0u, 0u, 0u};
  // First tilt's word: issued before the field rows, whose wait covers it
  // (a0 < n_a for every block of the grid).
  if constexpr (kPrefetch) tab_next = *tab_src(a0);
  // 8 field rows (contiguous in HBM, 4 P 16-byte words) -> LDS rows of stride
  // LDP; every load is issued before the first LDS write.
  {
    constexpr int NW = 4 * P;
    constexpr int NPT = (NW + 255) / 256;
    // The tail's surplus lanes load word NW - 1 again and store nothing: every
    // element of w is defined, so w stays in registers.
    if constexpr (kField) {
      // Word e = pixels 2 e and 2 e + 1 of the 8 rows (row e / (P / 2)).
      const float* po = opd + (fr * (size_t)P + yb) * (size_t)P;
      const float* pa = amp + (size_t)yb * P;
      float o[NPT][2], am[NPT][2];
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int e = min(tid + 256 * i, NW - 1);
        o[i][0] = po[2 * e];
        o[i][1] = po[2 * e + 1];
        am[i][0] = pa[2 * e];
        am[i][1] = pa[2 * e + 1];
      }
      fence();
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int e = tid + 256 * i;
        if (e < NW) {
          const int r = e / (P / 2), c2 = e - r * (P / 2);
          cpx* f = field + r * T::LDP + 2 * c2;
          f[0] = pupil_field(o[i][0], am[i][0], kphase, fp32_phase);
          f[1] = pupil_field(o[i][1], am[i][1], kphase, fp32_phase);
        }
      }
    } else {
      const uint4* src = reinterpret_cast<const uint4*>(fieldg + (fr * (size_t)P + yb) * (size_t)P);
      uint4 w[NPT];
#pragma unroll
      for (int i = 0; i < NPT; ++i) w[i] = src[min(tid + 256 * i, NW - 1)];
      fence();
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int e = tid + 256 * i;
        if (e < NW) {
          const int r = e / (P / 2), c2 = e - r * (P / 2);
          *reinterpret_cast<uint4*>(field + r * T::LDP + 2 * c2) = w[i];
        }
      }
    }
  }
  stage_tables16<E>(s_mid, s_tw, s_out, mid, tw, outw, tid, 256);
  for (int i = tid; i < P; i += 256) s_f[T::QO + i] = cpx{0.f, 0.f};
  const int a1 = min(a0 + a_chunk, n_a);
  const int r = wave * 2 + team;                  // row within the block
  const int y = yb + r;
  const int xl = l1 + 4 * l2;                     // this lane's samples: x = xl + 16 m
  const cpx* frow = field + r * T::LDP + xl;
  const cpx* ml = s_mid + l16 * T::MS;
  const cpx* tl = s_tw + l2 * T::TS;
  const cpx* ow = s_out + q * T::QO + xl;
  const cpx* tin = s_in + q * T::QO + xl;
  const cpx* tf = s_f + q * T::QO + xl;
  const float sA = (l2 & 2) ? -1.f : 1.f, sB = (l2 & 1) ? -1.f : 1.f;
  const bool l3 = l2 == 3;
  auto tab_ptr = tab_src(min(a0 + 1, a1 - 1));   // global address space: global loads
  // The first word is consumed here, on every path into the loop, so the
  // loop's own wait counts only the one load in flight across its stores.
  if constexpr (kPrefetch) asm volatile("" ::"v"(tab_next.x), "v"(tab_next.y), "v"(tab_next.z), "v"(tab_next.w));
  for (int ia = a0; ia < a1; ++ia) {
    __syncthreads();
    if constexpr (kPrefetch) {
      *tab_dst = tab_next;
      tab_next = *tab_ptr;
    } else {
      copy16(s_in, in_a + (size_t)ia * 2 * P, P / 2, tid, 256);
      copy16(s_in + T::QO, in_a + (size_t)ia * 2 * P + P, P / 2, tid, 256);
      copy16(s_f, f_a + (size_t)ia * P, P / 2, tid, 256);
    }
    __syncthreads();
    cpx v[E];
    line_op16<E>(v, [&](int m) { return cmul(frow[16 * m], tin[16 * m]); }, [&](int m) { return frow[16 * m]; },
                 [&](int m) { return tf[16 * m]; }, ml, tl, ow, sA, sB, l3);
    // Element (x' = qP + xl + 16 m, y): consecutive m are 16 P apart in the
    // intermediate layout (two 8-column groups); addresses formed just in time.
    // Global (not flat) stores: the pointer is in the global address space
    // before it passes the asm.
    g_f32x2* out = (g_f32x2*)Rw + (fr * (size_t)n_a + ia) * (size_t)(2 * P * P) + rw_index(q * P + xl, y, P);
    // Next tilt's table address, formed before the stores (registers written
    // after them could be ones a store still reads, which costs a full wait).
    if constexpr (kPrefetch) {
      tab_ptr = tab_src(min(ia + 2, a1 - 1));
      asm volatile("" : "+v"(tab_ptr));
    }
    fence();
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      g_f32x2* o = out + (size_t)m * 16 * P;
      asm volatile("" : "+v"(o));
      *o = f32x2{v[m].re, v[m].im};
    });
  }
}

// Column pass, long lines.  Block = CB / 2 waves = CB = 8 adjacent columns x'
// of one frame (one 32-lane team per column) and one chunk of modulation
// points; a block never straddles the two pupil windows.  When the binning
// divides 8 the block bins b x b itself; otherwise (b = 5) it writes
// row-binned sums per column and a reduction kernel finishes the bins.  The CB columns of one distinct x
// tilt are gathered from the intermediate into LDS as [y/4][column][y%4]
// with a y-group stride of 40 values (conflict-free reads); each team
// accumulates |E|^2 of its column over the chunk in registers, then the
// block bins b x b through LDS and writes its part of the chunk's pupils.
template <int E, int CB>
__global__ __launch_bounds__(32 * CB, 2) void col_pass16_kernel(
    const cpx* __restrict__ Rw, const cpx* __restrict__ in_b, const cpx* __restrict__ f_b,
    const int* __restrict__ k_order, const int* __restrict__ k_ia, const cpx* __restrict__ mid,
    const cpx* __restrict__ tw, const cpx* __restrict__ outw, float* __restrict__ partial, int n_a, int K,
    int k_chunk, int n_chunks, int n_bin) {
  using T = Tab16<E>;
  constexpr int P = T::P;
  constexpr int NT = 32 * CB;
  constexpr int G = P / 4;                        // y groups of 4 rows
  static_assert(4 * CB <= T::GS, "staged columns exceed the y-group stride");
  __shared__ __align__(16) cpx s_col[G * T::GS];
  __shared__ __align__(16) cpx s_in[2 * T::QO];
  __shared__ __align__(16) cpx s_f[2 * T::QO];   // [projection 0: -tilt | projection 1: 0]
  __shared__ __align__(16) cpx s_mid[16 * T::MS];
  __shared__ __align__(16) cpx s_tw[4 * T::TS];
  __shared__ __align__(16) cpx s_out[2 * T::QO];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int team = lane >> 5, q = (lane >> 4) & 1, l16 = lane & 15, l1 = l16 >> 2, l2 = l16 & 3;
  const int X0 = blockIdx.x * CB;
  const int chunk = blockIdx.y;
  const size_t fr = blockIdx.z;
  float acc[E];
  static_for<0, E>([&](auto m_) { acc[decltype(m_)::value] = 0.f; });
  stage_tables16<E>(s_mid, s_tw, s_out, mid, tw, outw, tid, NT);
  for (int i = tid; i < P; i += NT) s_f[T::QO + i] = cpx{0.f, 0.f};
  const int kb = chunk * k_chunk;
  const int ke = min(kb + k_chunk, K);
  const cpx* frame = Rw + fr * (size_t)n_a * (size_t)(2 * P * P);
  const int c = wave * 2 + team;                  // column within the block
  const int xl = l1 + 4 * l2;                     // this lane's rows: y = xl + 16 m
  const cpx* colp = s_col + l2 * T::GS + c * 4 + l1;   // row y = xl + 16 m at colp[4 m GS]
  const cpx* ml = s_mid + l16 * T::MS;
  const cpx* tl = s_tw + l2 * T::TS;
  const cpx* ow = s_out + q * T::QO + xl;
  const cpx* tin = s_in + q * T::QO + xl;
  const cpx* tf = s_f + q * T::QO + xl;
  const float sA = (l2 & 2) ? -1.f : 1.f, sB = (l2 & 1) ? -1.f : 1.f;
  const bool l3 = l2 == 3;
  int cur_ia = -1;
  for (int kk = kb; kk < ke; ++kk) {
    const int k = k_order[kk];
    const int ia = k_ia[k];
    __syncthreads();
    if (ia != cur_ia) {
      // (y group g, column c, half h) <- 4 values (y = 4g .. 4g+3) of column X0 + c,
      // two 16-byte words; all loads issued before the LDS writes.
      constexpr int NW = G * CB * 2;
      constexpr int NPT = (NW + NT - 1) / NT;
      const cpx* src = frame + (size_t)ia * (size_t)(2 * P * P);
      uint4 w[NPT];
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int u = min(tid + NT * i, NW - 1);   // tail lanes reload the last word
        const int g = u / (2 * CB), rem = u - g * (2 * CB), cc = rem >> 1, h = rem & 1;
        w[i] = *reinterpret_cast<const uint4*>(src + rw_index(X0 + cc, 4 * g, P) + 2 * h);
      }
      fence();
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int u = tid + NT * i;
        if (u < NW) {
          const int g = u / (2 * CB), rem = u - g * (2 * CB), cc = rem >> 1, h = rem & 1;
          *reinterpret_cast<uint4*>(s_col + g * T::GS + cc * 4 + 2 * h) = w[i];
        }
      }
      cur_ia = ia;
    }
    copy16(s_in, in_b + (size_t)k * 2 * P, P / 2, tid, NT);
    copy16(s_in + T::QO, in_b + (size_t)k * 2 * P + P, P / 2, tid, NT);
    copy16(s_f, f_b + (size_t)k * P, P / 2, tid, NT);
    __syncthreads();
    cpx v[E];
    line_op16<E>(v, [&](int m) { return cmul(colp[4 * m * T::GS], tin[16 * m]); },
                 [&](int m) { return colp[4 * m * T::GS]; }, [&](int m) { return tf[16 * m]; }, ml, tl, ow, sA, sB,
                 l3);
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      acc[m] += fmaf(v[m].re, v[m].re, v[m].im * v[m].im);
    });
  }
  __syncthreads();
  // tile[c][q][row] (CB 2 P floats, within s_col), then b x b binning.
  float* tile = reinterpret_cast<float*>(s_col);
  float* my = tile + (c * 2 + q) * P + xl;
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    my[16 * m] = acc[m];
  });
  __syncthreads();
  const int S = P / n_bin;
  if (CB % n_bin == 0) {
    // whole bins in the block: b x b sums straight into the chunk's pupils
    const int nbc = CB / n_bin;
    const int xw = X0 >= P ? 1 : 0;
    const int ix0 = (X0 - xw * P) / n_bin;
    float* dst = partial + (fr * (size_t)n_chunks + chunk) * (size_t)(4 * S * S);
    for (int o = tid; o < nbc * 2 * S; o += NT) {
      const int bc = o / (2 * S);
      const int rem = o - bc * 2 * S;
      const int qq = rem / S;
      const int iy = rem - qq * S;
      float sum = 0.f;
      for (int dx = 0; dx < n_bin; ++dx) {
        const float* gp = tile + ((bc * n_bin + dx) * 2 + qq) * P + iy * n_bin;
        for (int dy = 0; dy < n_bin; ++dy) sum += gp[dy];
      }
      dst[(size_t)(xw + 2 * qq) * S * S + (size_t)iy * S + ix0 + bc] = sum;
    }
  } else {
    // bins straddle blocks: row-binned sums per column, [qq][x'][iy], finished
    // by pupil_reduce_cols_kernel
    float* dst = partial + (fr * (size_t)n_chunks + chunk) * (size_t)(4 * P * S);
    for (int o = tid; o < CB * 2 * S; o += NT) {
      const int c = o / (2 * S);
      const int rem = o - c * 2 * S;
      const int qq = rem / S;
      const int iy = rem - qq * S;
      const float* gp = tile + (c * 2 + qq) * P + iy * n_bin;
      float sum = 0.f;
      for (int dy = 0; dy < n_bin; ++dy) sum += gp[dy];
      dst[(size_t)qq * (2 * P * S) + (size_t)(X0 + c) * S + iy] = sum;
    }
  }
}

// Pupil images from per-column partials [frame][chunk][qy][x'][iy]: pixel
// (q, iy, ix) = (1/K) sum over chunks (in order) and the b columns of the bin.
__global__ __launch_bounds__(256) void pupil_reduce_cols_kernel(const float* __restrict__ partial, int n_chunks,
                                                                int P, int S, int n_bin, float inv_k,
                                                                float* __restrict__ pupils) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const size_t fr = blockIdx.y;
  const int SS = S * S;
  if (i >= 4 * SS) return;
  const int q = i / SS, rem = i - q * SS, iy = rem / S, ix = rem - iy * S;
  const int xw = q & 1, qy = q >> 1;
  const size_t per_chunk = (size_t)4 * P * S;
  const float* pp = partial + fr * (size_t)n_chunks * per_chunk + (size_t)qy * (2 * P * S) +
                    (size_t)(xw * P + ix * n_bin) * S + iy;
  float s = 0.f;
  for (int c = 0; c < n_chunks; ++c) {
    const float* pc = pp + (size_t)c * per_chunk;
    for (int dx = 0; dx < n_bin; ++dx) s += pc[(size_t)dx * S];
  }
  pupils[fr * 4 * (size_t)SS + i] = s * inv_k;
}

template <int E>
static hipError_t launch_rows16_e(const MeasureArgs& a, hipStream_t st) {
  constexpr bool kField = E <= 10;                // the field formed in the row pass (n_pupil 128, 160)
  if (a.a_chunk < 1 || a.n_a < 1) return hipErrorInvalidValue;   // every block needs a0 < n_a
  if constexpr (!kField) {
    hipError_t e = launch_field(a, st);
    if (e != hipSuccess) return e;
  }
  dim3 grid(a.P / 8, (a.n_a + a.a_chunk - 1) / a.a_chunk, a.B);
  return launch_k(row_pass16_kernel<E, kField>, grid, dim3(256), 0, st, kField ? a.tev[0] : nullptr, a.tev[1],
                  a.field, a.opd, a.amp, a.kphase, a.fp32_phase, a.in_a, a.f_a, a.mid, a.tw16, a.outw, a.Rw, a.n_a,
                  a.a_chunk);
}

template <int E, int CB>
static hipError_t launch_cols16_e(const MeasureArgs& a, hipStream_t st) {
  dim3 grid(2 * a.P / CB, a.n_chunks, a.B);
  return launch_k(col_pass16_kernel<E, CB>, grid, dim3(32 * CB), 0, st, a.tev[2], a.tev[3], a.Rw, a.in_b, a.f_b,
                  a.k_order, a.k_ia, a.mid, a.tw16, a.outw, a.partial, a.n_a, a.K, a.k_chunk, a.n_chunks, a.n_bin);
}

hipError_t launch_rows_long(const MeasureArgs& a, hipStream_t st) {
  switch (a.P) {
    case 128: return launch_rows16_e<8>(a, st);
    case 160: return launch_rows16_e<10>(a, st);
    case 480: return launch_rows16_e<30>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cols_long(const MeasureArgs& a, hipStream_t st) {
  switch (a.P) {
    case 128: return launch_cols16_e<8, 8>(a, st);
    case 160: return launch_cols16_e<10, 8>(a, st);
    case 480: return launch_cols16_e<30, 8>(a, st);
    default: return hipErrorInvalidValue;
  }
}

bool partials_by_column(int P, int n_bin) { return (P == 128 || P == 480) && 8 % n_bin != 0; }

// First kernel of the finish: takes its start event; `stop` when it is also the last.
hipError_t launch_reduce_cols(const MeasureArgs& a, float* out, hipStream_t st, hipEvent_t stop) {
  const int S = a.P / a.n_bin;
  return launch_k(pupil_reduce_cols_kernel, dim3((4 * S * S + 255) / 256, a.B), dim3(256), 0, st, a.tev[4], stop,
                  (const float*)a.partial, a.n_chunks, a.P, S, a.n_bin, 1.0f / (float)a.K, out);
}

}  // namespace pwfs
