// pwfs_kernels.hip -- HIP kernels of the modulated pyramid sensor (gfx950).
//
// The 2-D operator "tilt -> FFT -> four-face mask -> inverse FFT" is
// separable: the mask exp(-2 pi i Delta (|u| + |v|) / N) and the tilt ramp
// factor into x and y parts, so every modulation point's output field is
// T_y [r_b . T_x [r_a . E]] with the 1-D operator T = IFFT diag(m) FFT.
// The kernels use two passes over the field:
//   row pass    T_x on each pupil row, once per distinct x tilt a
//               (k and K-k share a), written to an HBM intermediate;
//   column pass y tilt + T_y on each needed column, |E|^2, sum over the
//               modulation points of a chunk, b x b binning.
// and a small slopes kernel sums the chunks, normalises and subtracts the
// reference slopes.
//
// The 1-D operator restricted to what is kept.  With N = 4P and Delta = N/4
// the input occupies P samples at offset o = (N-P)/2 and the output is
// needed in two windows of P samples, at o - Delta (y_L) and o + Delta
// (y_H).  Splitting the N frequencies by residue mod 4, the even residues
// pass straight through and the odd residues see a +-1 step, which leaves
//   y_H(j) = (2/N) [w^-j b_1(j) + w^-3j b_3(j)],   y_L(j) = f(j) - y_H(j),
//   b_r = IDFT_P [ 1_{t < P/2} . DFT_P (f . w^{r x}) ],   w = exp(-2 pi i / N),
// i.e. two half-band projections of length P per line instead of a pair of
// length-N transforms.
//
// Lane mapping.  A line is handled by a team of 8 lanes: lanes 0-3 (quad 0)
// compute b_1, lanes 4-7 (quad 1) compute b_3.  Lane l of a quad holds the
// E = P/4 samples x = l + 4 m.  The half-band projection is
//   in-lane DFT_E over m  ->  twiddle w_P^{l k}  ->  quad 3-tap mix
//   V_l = 2 Y_l + (1 - i) Y_{l+1} + (1 + i) Y_{l-1}   (DPP quad_perm)
//   ->  conj twiddle  ->  in-lane inverse DFT_E,
// the exact four-step form of "keep frequencies t < P/2" with no LDS round
// trip.  The two quads then exchange their halves with one ds_swizzle.
//
// Intermediate layout (row pass -> column pass), complex64:
//   Rw[frame][a][x'/8][y/4][x'%8][y%4], x' in [0, 2P) (y_L then y_H), y in [0, P)
// so that both the row pass's stores and the column pass's loads touch
// 128-256 contiguous bytes per instruction.
#include "pwfs_common.h"
#include "pwfs_field.h"
#include "pwfs_launch.h"

#include <algorithm>
#include <cstdint>
#include <type_traits>

namespace pwfs {

// ---------------------------------------------------------------------------
// Pupil field A exp(i phi) of every pixel (pupil_field); once per frame.
__global__ __launch_bounds__(256) void field_kernel(const float* __restrict__ opd, const float* __restrict__ amp,
                                                    double kphase, int fp32_phase, int PP, size_t n,
                                                    cpx* __restrict__ field) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    field[i] = pupil_field(opd[i], amp[i % PP], kphase, fp32_phase);
}

// Row pass.  Block = 4 waves = 32 pupil rows of one frame (8 rows per wave),
// looping over a chunk of distinct x tilts.  The pupil field of the 32 rows
// is staged once in LDS; the tilt tables of each x tilt and the constant
// pyramid tables are staged in LDS and shared by the four waves.
//   in_a[ia][q][x] = r_a(x) w_N^{(2q+1) x},  f_a[ia][x] = r_a(x).
template <int E>
__global__ __launch_bounds__(256) void row_pass_kernel(
    const cpx* __restrict__ fieldg, const cpx* __restrict__ in_a, const cpx* __restrict__ f_a,
    const cpx* __restrict__ mid, const cpx* __restrict__ outw, cpx* __restrict__ Rw, int n_a, int a_chunk) {
  constexpr int P = 4 * E;
  constexpr int LDP = P + 4;
  __shared__ __align__(16) cpx field[32 * LDP];
  __shared__ __align__(16) cpx s_in[2 * P + 4];
  __shared__ __align__(16) cpx s_f[2 * TabLds<E>::QO];   // [quad 0: -tilt | quad 1: 0]
  __shared__ __align__(16) cpx s_mid[4 * TabLds<E>::MS];
  __shared__ __align__(16) cpx s_out[2 * P + 4];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int t = lane >> 3, q = (lane >> 2) & 1, l = lane & 3;
  const int yb = blockIdx.x * 32;
  const int a0 = blockIdx.y * a_chunk;
  const size_t fr = blockIdx.z;
  // Tilt tables, 3 P / 2 16-byte words (in_a quad 0 half, in_a quad 1 half,
  // f_a), loaded one x tilt ahead so that the load latency hides behind the
  // current tilt's transforms.  Thread t moves word t mod 3 P / 2 (threads
  // past the table repeat a word: same value, same address), and the last
  // tilt reloads itself, so there is no branch and the wait before the LDS
  // write covers that one load, not the stores of the previous tilt.
  constexpr int H = P / 2;
  const int tw = tid % (3 * H);
  const int tab_part = tw / H, tab_w = tw - (tw / H) * H;
  u32x4* const tab_dst = reinterpret_cast<u32x4*>(
      tab_part == 0 ? s_in : (tab_part == 1 ? s_in + TabLds<E>::QO : s_f)) + tab_w;
  auto tab_src = [&](int ia) {
    const cpx* base = tab_part < 2 ? in_a + (size_t)ia * 2 * P + tab_part * P : f_a + (size_t)ia * P;
    return (g_u32x4*)base + tab_w;
  };
  // First tilt's word: issued before the field rows, whose wait covers it
  // (a0 < n_a for every block of the grid).
  u32x4 tab_next = *tab_src(a0);
  // 32 field rows (contiguous in HBM) -> LDS rows of stride LDP, 16 bytes per move.
  // 32 P / 2 = 256 (P / 16) words per block, all loads issued before the LDS writes.
  const uint4* src = reinterpret_cast<const uint4*>(fieldg + (fr * (size_t)P + yb) * (size_t)P);
  {
    constexpr int NW = P / 16;
    uint4 w[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = src[tid + 256 * i];
    fence();
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int e = tid + 256 * i;
      const int r = e / (P / 2), c2 = e - r * (P / 2);
      *reinterpret_cast<uint4*>(field + r * LDP + 2 * c2) = w[i];
    }
  }
  stage_mid<E>(s_mid, mid, tid);
  stage_quads<E>(s_out, outw, tid);
  for (int i = tid; i < P; i += 256) s_f[TabLds<E>::QO + i] = cpx{0.f, 0.f};
  const int a1 = min(a0 + a_chunk, n_a);
  const int r = wave * 8 + t;                     // row within the block
  const cpx* frow = field + r * LDP + l;
  const int y = yb + r;
  auto tab_ptr = tab_src(min(a0 + 1, a1 - 1));   // global address space: global loads
  // The first word is consumed here, on every path into the loop, so the
  // loop's own wait counts only the one load in flight across its stores.
  asm volatile("" ::"v"(tab_next.x), "v"(tab_next.y), "v"(tab_next.z), "v"(tab_next.w));
  for (int ia = a0; ia < a1; ++ia) {
    __syncthreads();
    *tab_dst = tab_next;
    tab_next = *tab_ptr;
    __syncthreads();
    const cpx* tin = s_in + q * TabLds<E>::QO + l;
    const cpx* tf = s_f + q * TabLds<E>::QO + l;
    cpx v[E];
    line_op<E>(v, [&](int m) { return cmul(frow[4 * m], tin[4 * m]); }, [&](int m) { return frow[4 * m]; },
               [&](int m) { return tf[4 * m]; }, s_mid, s_out, q, l);
    // Element (x' = qP + l + 4m, y) sits at base + (m >> 1) 8P + (m & 1) 16
    // (see rw_index); each address is formed just before its store so the
    // compiler does not keep E 64-bit addresses live across the transforms.
    // The pointer is in the global address space before it passes the asm,
    // so the stores are global, not flat: a pending flat access would turn
    // the wait for the next tilt's table load into a wait for these stores.
    g_f32x2* out = (g_f32x2*)Rw + (fr * (size_t)n_a + ia) * (size_t)(2 * P * P) + rw_index(q * P + l, y, P);
    // Next tilt's table address, formed before the stores: registers written
    // after them could be ones a store still reads, which costs a full wait.
    tab_ptr = tab_src(min(ia + 2, a1 - 1));
    asm volatile("" : "+v"(tab_ptr));
    fence();
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      g_f32x2* o = out + (size_t)((m >> 1) * 8 * P + (m & 1) * 16);
      asm volatile("" : "+v"(o));
      *o = f32x2{v[m].re, v[m].im};
    });
  }
}

// ---------------------------------------------------------------------------
// Column pass.  Block = 4 waves = 32 adjacent columns x' of one frame (8 per
// wave) and one chunk of modulation points.  In the intermediate layout the
// 32 columns form one contiguous block of 32P complex values, staged in LDS
// once per distinct x tilt (k and K-k are adjacent in the modulation order
// and share it).  Each team accumulates |E|^2 of its column over the chunk
// in registers.  With G = 4 (binning a multiple of 4) the four rows
// 4m..4m+3, held by the four lanes of a quad, are summed by a DPP quad
// reduction as they are accumulated and lane l keeps the row groups
// m = 4i + l; with G = 2 (even binning) lane pairs sum rows 4m + {0, 1} and
// 4m + {2, 3} and each lane keeps every other m; G = 1 keeps every row.  The
// block then finishes the b x b binning through LDS and writes its part of
// the chunk's four pupil images.
//   in_b[k][q][y] = r_b(y) w_N^{(2q+1) y},  f_b[k][y] = -r_b(y).
template <int E, int G>
__global__ __launch_bounds__(256) void col_pass_kernel(
    const cpx* __restrict__ Rw, const cpx* __restrict__ in_b, const cpx* __restrict__ f_b,
    const int* __restrict__ k_order, const int* __restrict__ k_ia, const cpx* __restrict__ mid,
    const cpx* __restrict__ outw, float* __restrict__ partial, int n_a, int K, int k_chunk,
    int n_chunks, int n_bin) {
  constexpr int P = 4 * E;
  static_assert(G == 1 || G == 2 || G == 4, "row groups of 1, 2 or 4 lanes");
  constexpr int NA = E / G;                      // accumulators per lane
  __shared__ __align__(16) cpx s_col[32 * P];
  __shared__ __align__(16) cpx s_in[2 * P + 4];
  __shared__ __align__(16) cpx s_f[2 * TabLds<E>::QO];   // [quad 0: -tilt | quad 1: 0]
  __shared__ __align__(16) cpx s_mid[4 * TabLds<E>::MS];
  __shared__ __align__(16) cpx s_out[2 * P + 4];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int t = lane >> 3, q = (lane >> 2) & 1, l = lane & 3;
  const int X0 = blockIdx.x * 32;
  const int chunk = blockIdx.y;
  const size_t fr = blockIdx.z;
  float acc[NA];
  static_for<0, NA>([&](auto m_) { acc[decltype(m_)::value] = 0.f; });
  stage_mid<E>(s_mid, mid, tid);
  stage_quads<E>(s_out, outw, tid);
  for (int i = tid; i < P; i += 256) s_f[TabLds<E>::QO + i] = cpx{0.f, 0.f};
  const int kb = chunk * k_chunk;
  const int ke = min(kb + k_chunk, K);
  const cpx* frame = Rw + fr * (size_t)n_a * (size_t)(2 * P * P) + (size_t)(X0 >> 3) * (size_t)(8 * P);
  const int c = wave * 8 + t;                      // column within the block
  const cpx* col = s_col + wave * 8 * P + t * 4 + l;   // element (x' = X0 + c, y = l + 4m) at col[32 m]
  const cpx* tin = s_in + q * TabLds<E>::QO + l;
  const cpx* tf = s_f + q * TabLds<E>::QO + l;
  // Lane l keeps the groups m = G i + (l mod G): one FMA with a 0/1 mask per
  // group instead of a select and an add.
  float keepm[G];
  static_for<0, G>([&](auto j_) { keepm[decltype(j_)::value] = ((l & (G - 1)) == decltype(j_)::value) ? 1.f : 0.f; });
  int cur_ia = -1;
  for (int kk = kb; kk < ke; ++kk) {
    const int k = k_order[kk];
    const int ia = k_ia[k];
    __syncthreads();
    if (ia != cur_ia) {
      copy16_n<P / 16>(s_col, frame + (size_t)ia * (size_t)(2 * P * P), tid);   // 16 P words
      cur_ia = ia;
    }
    stage_quads<E>(s_in, in_b + (size_t)k * 2 * P, tid);
    copy16(s_f, f_b + (size_t)k * P, P / 2, tid, 256);
    __syncthreads();
    cpx v[E];
    line_op<E>(v, [&](int m) { return cmul(col[32 * m], tin[4 * m]); }, [&](int m) { return col[32 * m]; },
               [&](int m) { return tf[4 * m]; }, s_mid, s_out, q, l);
    // |E|^2 of all E samples first, then each DPP round over all of them: a
    // DPP read of e[m] then follows the VALU write of e[m] by many
    // instructions, so it needs no wait states.
    float e[E];
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      e[m] = fmaf(v[m].re, v[m].re, v[m].im * v[m].im);
    });
    if constexpr (G >= 2) {
      static_for<0, E>([&](auto m_) {
        constexpr int m = decltype(m_)::value;
        e[m] += quad_perm<0xB1>(e[m]);             // lanes (0,1), (2,3)
      });
    }
    if constexpr (G == 4) {
      static_for<0, E>([&](auto m_) {
        constexpr int m = decltype(m_)::value;
        e[m] += quad_perm<0x4E>(e[m]);             // lanes (0,2), (1,3)
      });
    }
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      if constexpr (G == 4) acc[m >> 2] = fmaf(keepm[m & 3], e[m], acc[m >> 2]);
      else if constexpr (G == 2) acc[m >> 1] = fmaf(keepm[m & 1], e[m], acc[m >> 1]);
      else acc[m] += e[m];
    });
  }
  __syncthreads();
  float* tile = reinterpret_cast<float*>(s_col);
  const int S = P / n_bin;
  const int nbc = 32 / n_bin;
  const int xw = X0 >= P ? 1 : 0;
  const int ix0 = (X0 - xw * P) / n_bin;
  float* dst = partial + (fr * (size_t)n_chunks + chunk) * (size_t)(4 * S * S);
  if constexpr (G > 1) {
    // tile[c][q][g]: sum over rows G g .. G g + G - 1 of column c, window q;
    // lane l holds the groups g = 4 i + slot.
    const int slot = G == 4 ? l : 2 * (l & 1) + (l >> 1);
    float* my = tile + (c * 2 + q) * (P / G) + slot;
    static_for<0, NA>([&](auto i_) {
      constexpr int i = decltype(i_)::value;
      my[4 * i] = acc[i];
    });
    __syncthreads();
    const int gpb = n_bin / G;                     // row groups per bin
    for (int o = tid; o < nbc * 2 * S; o += 256) {
      const int bc = o / (2 * S);
      const int rem = o - bc * 2 * S;
      const int qq = rem / S;
      const int iy = rem - qq * S;
      float sum = 0.f;
      for (int dx = 0; dx < n_bin; ++dx) {
        const float* g = tile + ((bc * n_bin + dx) * 2 + qq) * (P / G) + iy * gpb;
        for (int dg = 0; dg < gpb; ++dg) sum += g[dg];
      }
      dst[(size_t)(xw + 2 * qq) * S * S + (size_t)iy * S + ix0 + bc] = sum;
    }
  } else {
    // tile[c][q][row]
    float* my = tile + (c * 2 + q) * P + l;
    static_for<0, NA>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      my[4 * m] = acc[m];
    });
    __syncthreads();
    for (int o = tid; o < nbc * 2 * S; o += 256) {
      const int bc = o / (2 * S);
      const int rem = o - bc * 2 * S;
      const int qq = rem / S;
      const int iy = rem - qq * S;
      float sum = 0.f;
      for (int dx = 0; dx < n_bin; ++dx) {
        const float* g = tile + ((bc * n_bin + dx) * 2 + qq) * P + iy * n_bin;
        for (int dy = 0; dy < n_bin; ++dy) sum += g[dy];
      }
      dst[(size_t)(xw + 2 * qq) * S * S + (size_t)iy * S + ix0 + bc] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// Pupil reduction: sum of the chunk partials in chunk order (fixed order,
// loads issued four at a time), scaled by 1/K.  One thread per binned pixel.
__global__ __launch_bounds__(256) void pupil_reduce_kernel(const float* __restrict__ partial, int n_chunks,
                                                           int n4ss, float inv_k, float* __restrict__ pupils) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const size_t fr = blockIdx.y;
  if (i >= n4ss) return;
  const size_t stride = (size_t)n4ss;
  const float* pp = partial + fr * (size_t)n_chunks * stride + i;
  float s = 0.f;
  int c = 0;
  for (; c + 4 <= n_chunks; c += 4) {
    const float a = pp[(size_t)c * stride], b = pp[(size_t)(c + 1) * stride];
    const float d = pp[(size_t)(c + 2) * stride], e = pp[(size_t)(c + 3) * stride];
    s += a;
    s += b;
    s += d;
    s += e;
  }
  for (; c < n_chunks; ++c) s += pp[(size_t)c * stride];
  pupils[fr * stride + i] = s * inv_k;
}

// Slopes.  One block of 1024 threads per frame: mean total flux over the
// valid subapertures (fixed-order tree), then reference-subtracted slopes.
// The four intensities of a thread's first two subapertures (all of them up
// to 2048 valid ones) stay in registers between the two passes, so the
// second pass does not repeat the dependent index-then-pixel loads.
__global__ __launch_bounds__(1024) void slopes_kernel(const float* __restrict__ pupils, int S,
                                                      const int* __restrict__ valid, int nv,
                                                      const float* __restrict__ sref, int norm_mode,
                                                      float* __restrict__ slopes) {
  constexpr int KEEP = 2;
  __shared__ float red[1024];
  const int tid = threadIdx.x;
  const size_t fr = blockIdx.x;
  const size_t SS = (size_t)S * S;
  const float* pp = pupils + fr * 4 * SS;
  float ik[KEEP][4];
#pragma unroll
  for (int r = 0; r < KEEP; ++r) {
    const int v = tid + 1024 * r;
    const size_t j = (size_t)valid[min(v, nv - 1)];   // clamped for loading, used only when v < nv
#pragma unroll
    for (int c = 0; c < 4; ++c) ik[r][c] = pp[c * SS + j];
  }
  float loc = 0.f;
  if (norm_mode == 0) {
#pragma unroll
    for (int r = 0; r < KEEP; ++r)
      if (tid + 1024 * r < nv) loc += (ik[r][0] + ik[r][1]) + (ik[r][2] + ik[r][3]);
    for (int v = tid + 1024 * KEEP; v < nv; v += 1024) {
      const size_t j = (size_t)valid[v];
      loc += (pp[j] + pp[SS + j]) + (pp[2 * SS + j] + pp[3 * SS + j]);
    }
  }
  red[tid] = loc;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  const float mean_flux = red[0] / (float)nv;
  float* so = slopes + fr * 2 * (size_t)nv;
  auto emit = [&](int v, float i0, float i1, float i2, float i3) {
    const float n = norm_mode ? ((i0 + i1) + (i2 + i3)) : mean_flux;
    so[v] = ((i1 + i3) - (i0 + i2)) / n - sref[v];
    so[nv + v] = ((i2 + i3) - (i0 + i1)) / n - sref[nv + v];
  };
#pragma unroll
  for (int r = 0; r < KEEP; ++r)
    if (tid + 1024 * r < nv) emit(tid + 1024 * r, ik[r][0], ik[r][1], ik[r][2], ik[r][3]);
  for (int v = tid + 1024 * KEEP; v < nv; v += 1024) {
    const size_t j = (size_t)valid[v];
    emit(v, pp[j], pp[SS + j], pp[2 * SS + j], pp[3 * SS + j]);
  }
}

// ---------------------------------------------------------------------------
// m = alpha R s + beta m for B <= 16.  Block = W <= 10 waves over RW rows of
// R and BT slope vectors; thread t of the block takes the float4 (or scalar)
// columns j = t, t + 64 W, ... (one pass when the row has at most 640 of
// them), loads the RW row pieces and the BT vector pieces of a column before
// any product, and keeps the RW x BT partial sums (NV of them, a power of two
// <= 64).  Each wave then sums its 64 lanes by recursive halving: at the step
// of distance o a lane keeps one half of its sums (the upper half when lane
// bit o is set), adds the partner's copy of that half and hands over the
// other, so after log2 NV steps lane l holds sum number l >> (6 - log2 NV) of
// its group of 64 / NV lanes, and a butterfly over the group completes it
// (63 exchanges for NV = 64 instead of 6 x 64).  The W wave sums are added in
// wave order through LDS: a fixed summation order, bitwise reproducible.
// Rows and vectors past the ends are clamped to the last one for loading (in
// bounds, never stored).
constexpr int kReconMaxWaves = 10;

template <int BT, int RW, int VEC>
__global__ __launch_bounds__(64 * kReconMaxWaves) void recon_kernel(const float* __restrict__ R, int M, int ns,
                                                                    const float* __restrict__ s, int B,
                                                                    float alpha, float beta,
                                                                    float* __restrict__ m) {
  constexpr int NV = RW * BT;
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "RW x BT sums: a power of two <= 64");
  constexpr int LOG2NV = NV >= 64 ? 6 : NV >= 32 ? 5 : NV >= 16 ? 4 : NV >= 8 ? 3 : NV >= 4 ? 2 : NV >= 2 ? 1 : 0;
  constexpr int SH = 6 - LOG2NV;
  using V = typename std::conditional<VEC == 4, float4, float>::type;
  __shared__ float part[kReconMaxWaves][NV];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int W = (int)(blockDim.x >> 6);
  const int i0 = blockIdx.x * RW;
  const int b0 = blockIdx.y * BT;
  const int nb = min(BT, B - b0);
  const int nv = ns / VEC;
  float v[NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) v[e] = 0.f;
  for (int j = tid; j < nv; j += 64 * W) {
    V r[RW], x[BT];
#pragma unroll
    for (int rr = 0; rr < RW; ++rr)
      r[rr] = reinterpret_cast<const V*>(R + (size_t)min(i0 + rr, M - 1) * (size_t)ns)[j];
#pragma unroll
    for (int bb = 0; bb < BT; ++bb)
      x[bb] = reinterpret_cast<const V*>(s + (size_t)(b0 + min(bb, nb - 1)) * (size_t)ns)[j];
    fence();
#pragma unroll
    for (int rr = 0; rr < RW; ++rr)
#pragma unroll
      for (int bb = 0; bb < BT; ++bb) {
        float& acc = v[rr * BT + bb];
        if constexpr (VEC == 4) {
          acc = fmaf(r[rr].x, x[bb].x, acc);
          acc = fmaf(r[rr].y, x[bb].y, acc);
          acc = fmaf(r[rr].z, x[bb].z, acc);
          acc = fmaf(r[rr].w, x[bb].w, acc);
        } else {
          acc = fmaf(r[rr], x[bb], acc);
        }
      }
  }
  static_for<0, LOG2NV>([&](auto st_) {
    constexpr int st = decltype(st_)::value;
    constexpr int o = 32 >> st, h = NV >> (st + 1);
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int e = 0; e < h; ++e) {
      const float keep = up ? v[e + h] : v[e];
      const float give = up ? v[e] : v[e + h];
      v[e] = keep + __shfl_xor(give, o);
    }
  });
#pragma unroll
  for (int o = 32 >> LOG2NV; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o);
  if ((lane & ((1 << SH) - 1)) == 0) part[wave][lane >> SH] = v[0];
  __syncthreads();
  if (tid < NV) {
    const int rr = tid / BT, bb = tid - rr * BT;
    const int i = i0 + rr;
    if (i < M && bb < nb) {
      float tot = part[0][tid];
      for (int w = 1; w < W; ++w) tot += part[w][tid];
      float* mm = m + (size_t)(b0 + bb) * M + i;
      *mm = beta != 0.f ? fmaf(alpha, tot, beta * *mm) : alpha * tot;
    }
  }
}

// ---------------------------------------------------------------------------
// Batched m = alpha R s + beta m for B > 16 frames: a dense FP32 product
// C[b][i] = sum_k s[b][k] R[i][k] on v_mfma_f32_32x32x2f32 (FP32 operands,
// fixed order).  Block = 4 waves, tile 64 frames x 64 rows of
// R, K step 32 through LDS; lane l feeds A(b = l % 32, k = l / 32) and
// B(i = l % 32, k = l / 32); accumulator v of lane l is
// C(8 (v / 4) + 4 (l / 32) + v % 4, l % 32).
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void recon_mfma_kernel(const float* __restrict__ R, int M, int ns,
                                                          const float* __restrict__ s, int B, float alpha,
                                                          float beta, float* __restrict__ m) {
  __shared__ float As[64][33];
  __shared__ float Bs[64][33];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int b0 = blockIdx.y * 64, i0 = blockIdx.x * 64;
  // The MFMA accumulator is reset for every 32-wide K tile and the tiles are
  // summed with ordinary FP32 adds (round to nearest): the matrix core's own
  // accumulation rounding is biased, so it is confined to 32 terms.
  f32x16_t acc, tile;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int k0 = 0; k0 < ns; k0 += 32) {
    for (int e = tid; e < 2048; e += 256) {
      const int r = e >> 5, kk = e & 31;
      const int gk = k0 + kk;
      const int gb = b0 + r, gi = i0 + r;
      As[r][kk] = (gb < B && gk < ns) ? s[(size_t)gb * ns + gk] : 0.f;
      Bs[r][kk] = (gi < M && gk < ns) ? R[(size_t)gi * ns + gk] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 16; ++v) tile[v] = 0.f;
#pragma unroll
    for (int kk = 0; kk < 32; kk += 2) {
      const float a = As[wm * 32 + (lane & 31)][kk + (lane >> 5)];
      const float b = Bs[wn * 32 + (lane & 31)][kk + (lane >> 5)];
      tile = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, tile, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] += tile[v];
    __syncthreads();
  }
  const int i = i0 + wn * 32 + (lane & 31);
  if (i >= M) return;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int b = b0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (b >= B) continue;
    float* mm = m + (size_t)b * M + i;
    *mm = beta != 0.f ? fmaf(alpha, acc[v], beta * *mm) : alpha * acc[v];
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
hipError_t launch_field_raw(const float* opd, const float* amp, double kphase, int P, int B, cpx* field,
                            hipStream_t st) {
  const size_t n = (size_t)B * P * P;
  const unsigned fb = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(field_kernel, dim3(fb), dim3(256), 0, st, opd, amp, kphase, 0, P * P, n, field);
  return hipGetLastError();
}

hipError_t launch_field(const MeasureArgs& a, hipStream_t st) {
  const size_t n = (size_t)a.B * a.P * a.P;
  const unsigned fb = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  return launch_k(field_kernel, dim3(fb), dim3(256), 0, st, a.tev[0], nullptr, a.opd, a.amp, a.kphase, a.fp32_phase,
                  a.P * a.P, n, a.field);
}

template <int E>
static hipError_t launch_rows(const MeasureArgs& a, hipStream_t st) {
  if (a.a_chunk < 1 || a.n_a < 1) return hipErrorInvalidValue;   // every block needs a0 < n_a
  hipError_t e = launch_field(a, st);
  if (e != hipSuccess) return e;
  dim3 grid(a.P / 32, (a.n_a + a.a_chunk - 1) / a.a_chunk, a.B);
  return launch_k(row_pass_kernel<E>, grid, dim3(256), 0, st, nullptr, a.tev[1], a.field, a.in_a, a.f_a, a.mid,
                  a.outw, a.Rw, a.n_a, a.a_chunk);
}

template <int E>
static hipError_t launch_cols(const MeasureArgs& a, hipStream_t st) {
  dim3 grid(2 * a.P / 32, a.n_chunks, a.B);
  auto* kern = a.n_bin % 4 == 0 ? col_pass_kernel<E, 4> : a.n_bin % 2 == 0 ? col_pass_kernel<E, 2>
                                                                           : col_pass_kernel<E, 1>;
  return launch_k(kern, grid, dim3(256), 0, st, a.tev[2], a.tev[3], a.Rw, a.in_b, a.f_b, a.k_order, a.k_ia, a.mid,
                  a.outw, a.partial, a.n_a, a.K, a.k_chunk, a.n_chunks, a.n_bin);
}

hipError_t launch_finish(const MeasureArgs& a, int Sb, hipStream_t st);

// Non-integer detector rebin: each P x P window [B][4][P][P] to S x S pixels
// of pitch P / S.  Positions in units of 1 / S: pupil pixel y spans
// [y S, (y + 1) S), detector pixel j spans [j P, (j + 1) P); their overlap is
// an exact integer, and pixel (j, i) = sum_y,x ov_y ov_x img[y][x] / S^2, the
// integral of the piecewise-constant window over the pixel in pupil-pixel
// area units.
__global__ __launch_bounds__(256) void rebin_kernel(const float* __restrict__ in, int P, int S,
                                                    float* __restrict__ out) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  const size_t fr = blockIdx.y;
  if (o >= 4 * S * S) return;
  const int q = o / (S * S), rem = o - q * S * S, j = rem / S, i = rem - j * S;
  const float* img = in + (fr * 4 + q) * (size_t)P * P;
  const int y0 = (j * P) / S, y1 = ((j + 1) * P + S - 1) / S;
  const int x0 = (i * P) / S, x1 = ((i + 1) * P + S - 1) / S;
  float acc = 0.f;
  for (int y = y0; y < y1; ++y) {
    const int wy = min((y + 1) * S, (j + 1) * P) - max(y * S, j * P);
    float row = 0.f;
    for (int x = x0; x < x1; ++x) {
      const int wx = min((x + 1) * S, (i + 1) * P) - max(x * S, i * P);
      row = fmaf((float)wx, img[(size_t)y * P + x], row);
    }
    acc = fmaf((float)wy, row, acc);
  }
  out[fr * 4 * (size_t)S * S + o] = acc / (float)(S * S);
}

hipError_t launch_measure(const MeasureArgs& args, hipStream_t st, hipEvent_t* ev) {
  MeasureArgs a = args;
  for (int i = 0; i < 6; ++i) a.tev[i] = ev ? ev[i] : nullptr;
  hipError_t e = hipSuccess;
  if (a.fs_on) {
    if ((e = launch_field(a, st)) != hipSuccess) return e;
    if ((e = launch_fstop_passes(a, st)) != hipSuccess) return e;
    return launch_finish(a, a.P, st);
  }
  if (a.lines16) {
    e = launch_rows_long(a, st);
  } else {
    switch (a.P) {
      case 32: e = launch_rows<8>(a, st); break;
      case 64: e = launch_rows<16>(a, st); break;
      case 160: e = launch_rows<40>(a, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  if (a.lines16) {
    e = launch_cols_long(a, st);
  } else {
    switch (a.P) {
      case 32: e = launch_cols<8>(a, st); break;
      case 64: e = launch_cols<16>(a, st); break;
      case 160: e = launch_cols<40>(a, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  return launch_finish(a, a.P / a.n_bin, st);
}

// After the passes: chunk sum of the partial images (Sb x Sb per window),
// optional rebin, detector and slopes.  The first kernel takes the finish's
// start event, the last one its stop event.
hipError_t launch_finish(const MeasureArgs& a, int Sb, hipStream_t st) {
  hipError_t e = hipSuccess;
  const int S = a.rebin_S > 0 ? a.rebin_S : Sb;
  const int n4ss = 4 * S * S;
  const int last = a.slopes ? 3 : a.det_on ? 2 : a.rebin_S > 0 ? 1 : 0;
  auto stop_if = [&](int i) { return i == last ? a.tev[5] : nullptr; };
  // With a detector the noiseless images go to the intensity scratch and the
  // detector writes the pixels that the slopes use.
  float* images = a.det_on ? a.intensity : a.pupils;
  float* reduced = a.rebin_S > 0 ? a.fullres : images;
  if (!a.fs_on && partials_by_column(a.P, a.n_bin)) {
    // (its start event: see launch_reduce_cols)
    if ((e = launch_reduce_cols(a, reduced, st, stop_if(0))) != hipSuccess) return e;
  } else {
    const int n4bb = 4 * Sb * Sb;
    if ((e = launch_k(pupil_reduce_kernel, dim3((n4bb + 255) / 256, a.B), dim3(256), 0, st, a.tev[4], stop_if(0),
                      (const float*)a.partial, a.n_chunks, n4bb, 1.0f / (float)a.K, reduced)) != hipSuccess)
      return e;
  }
  if (a.rebin_S > 0) {
    if ((e = launch_k(rebin_kernel, dim3((n4ss + 255) / 256, a.B), dim3(256), 0, st, nullptr, stop_if(1),
                      (const float*)a.fullres, a.P, S, images)) != hipSuccess)
      return e;
  }
  if (a.det_on) {
    if ((e = launch_detector(a.intensity, a.pupils, n4ss, a.B, a.frame0, a.det_gain, a.det_ron, a.det_seed, st,
                             stop_if(2))) != hipSuccess)
      return e;
  }
  if (a.slopes) {
    if ((e = launch_k(slopes_kernel, dim3(a.B), dim3(1024), 0, st, nullptr, stop_if(3), (const float*)a.pupils, S,
                      a.valid, a.nv, a.sref, a.norm_mode, a.slopes)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

__global__ void fill_kernel(float* __restrict__ p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill(float* p, size_t n, float v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

template <int BT, int RW>
static void launch_recon_bt(const float* R, int M, int ns, const float* s, int B, float alpha, float beta,
                            float* m, hipStream_t st) {
  const bool vec = (ns % 4 == 0) && ((uintptr_t)R % 16 == 0) && ((uintptr_t)s % 16 == 0);
  const int nv = vec ? ns / 4 : ns;
  const int waves = std::max(1, std::min(kReconMaxWaves, (nv + 63) / 64));
  dim3 grid((M + RW - 1) / RW, (B + BT - 1) / BT);
  if (vec)
    hipLaunchKernelGGL((recon_kernel<BT, RW, 4>), grid, dim3(64 * waves), 0, st, R, M, ns, s, B, alpha, beta, m);
  else
    hipLaunchKernelGGL((recon_kernel<BT, RW, 1>), grid, dim3(64 * waves), 0, st, R, M, ns, s, B, alpha, beta, m);
}

hipError_t launch_recon(const float* R, int M, int ns, const float* s, int B, float alpha,
                        float beta, float* m, hipStream_t st) {
  if (B > 16) {
    hipLaunchKernelGGL(recon_mfma_kernel, dim3((M + 63) / 64, (B + 63) / 64), dim3(256), 0, st, R, M, ns, s, B,
                       alpha, beta, m);
    return hipGetLastError();
  }
  // Four rows per block at every batch size: the block's 4 x BT sums come
  // out of the halving steps in one pass.
  if (B <= 1)
    launch_recon_bt<1, 4>(R, M, ns, s, B, alpha, beta, m, st);
  else if (B <= 4)
    launch_recon_bt<4, 4>(R, M, ns, s, B, alpha, beta, m, st);
  else if (B <= 8)
    launch_recon_bt<8, 4>(R, M, ns, s, B, alpha, beta, m, st);
  else
    launch_recon_bt<16, 4>(R, M, ns, s, B, alpha, beta, m, st);
  return hipGetLastError();
}

}  // namespace pwfs
