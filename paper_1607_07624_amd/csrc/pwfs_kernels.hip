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
#include "pwfs_dft.h"
#include "pwfs_launch.h"

#include <algorithm>

namespace pwfs {

// Scheduling fence: keeps the machine scheduler from hoisting the table and
// field loads of later phases over the register-resident transforms.
__device__ __forceinline__ void fence() { __builtin_amdgcn_sched_barrier(0); }

// Opaque copy of a wave-uniform pointer: stops loop-invariant code motion
// from hoisting whole tables out of the modulation loop into registers.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Half-band projection of the E samples held by this lane (see header).
// mid[l * E + k] = w_P^{l k}.
template <int E>
__device__ __forceinline__ void half_band(cpx (&v)[E], const cpx* __restrict__ mid, int l) {
  Dft<E, +1>::run(v);
  fence();
  const cpx* ml = mid + l * E;
  static_for<0, E>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    if constexpr (k % 8 == 0 && k > 0) fence();
    const cpx w = ml[k];
    const cpx y = cmul(v[k], w);
    const float pr = quad_perm<0x39>(y.re), pim = quad_perm<0x39>(y.im);  // lane l+1
    const float nr = quad_perm<0x93>(y.re), nim = quad_perm<0x93>(y.im);  // lane l-1
    const float sr = pr + nr, si = pim + nim;
    const float dr = nr - pr, di = nim - pim;
    const cpx V = {fmaf(2.f, y.re, sr - di), fmaf(2.f, y.im, si + dr)};
    v[k] = cmulc(V, w);
  });
  fence();
  Dft<E, -1>::run(v);
  fence();
}

// Full 1-D pyramid operator for one line.  load_f(m) returns f(l + 4 m) for
// this lane's line (f = tilted input field).  On return quad 0 holds
// y_L(l + 4 m) and quad 1 holds y_H(l + 4 m) in v[m].
//   twist[q * P + x] = w_N^{(2q+1) x},  outw[q * P + j] = (2/N) w_N^{-(2q+1) j}.
template <int E, typename LoadF>
__device__ __forceinline__ void line_op(cpx (&v)[E], LoadF&& load_f, const cpx* __restrict__ twist,
                                        const cpx* __restrict__ mid, const cpx* __restrict__ outw,
                                        int q, int l) {
  constexpr int P = 4 * E;
  const cpx* tw = twist + q * P + l;
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    if constexpr (m % 8 == 0 && m > 0) fence();
    v[m] = cmul(load_f(m), tw[4 * m]);
  });
  fence();
  half_band<E>(v, mid, l);
  const cpx* ow = outw + q * P + l;
  const float keep = (q == 0) ? 1.f : 0.f;   // quad 0 adds f back (y_L = f - y_H)
  const float sgn = (q == 0) ? -1.f : 1.f;
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    if constexpr (m % 8 == 0 && m > 0) fence();
    cpx w = cmul(v[m], ow[4 * m]);
    w.re += swap_quads(w.re);
    w.im += swap_quads(w.im);
    const cpx f = load_f(m);
    v[m] = {fmaf(sgn, w.re, keep * f.re), fmaf(sgn, w.im, keep * f.im)};
  });
}

__device__ __forceinline__ size_t rw_index(int xp, int y, int P) {
  return ((size_t)(xp >> 3) * (size_t)(P >> 2) + (size_t)(y >> 2)) * 32u + (size_t)((xp & 7) * 4 + (y & 3));
}

// ---------------------------------------------------------------------------
// Row pass.  Block = one wave = 8 pupil rows of one frame, looping over a
// chunk of distinct x tilts.  The pupil field A exp(i phi) of the 8 rows is
// staged once in LDS; the phase is formed and range-reduced in FP64.
template <int E>
__global__ __launch_bounds__(64) void row_pass_kernel(
    const float* __restrict__ opd, const float* __restrict__ amp, double kphase,
    const cpx* __restrict__ ramp_a, const cpx* __restrict__ twist, const cpx* __restrict__ mid,
    const cpx* __restrict__ outw, cpx* __restrict__ Rw, int n_a, int a_chunk) {
  constexpr int P = 4 * E;
  constexpr int LDP = P + 4;
  __shared__ cpx field[8 * LDP];
  const int lane = threadIdx.x;
  const int t = lane >> 3, q = (lane >> 2) & 1, l = lane & 3;
  const int y0 = blockIdx.x * 8;
  const int a0 = blockIdx.y * a_chunk;
  const size_t fr = blockIdx.z;
  const float* op = opd + fr * (size_t)P * P;
  constexpr double two_pi = 6.283185307179586476925286766559;
  constexpr double inv_two_pi = 0.15915494309189533576888376337251;
  for (int i = lane; i < 8 * P; i += 64) {
    const int r = i / P, x = i - r * P;
    const int y = y0 + r;
    const double th = (double)op[y * P + x] * kphase;
    const double red = fma(-rint(th * inv_two_pi), two_pi, th);
    float s, c;
    sincosf((float)red, &s, &c);
    const float A = amp[y * P + x];
    field[r * LDP + x] = {A * c, A * s};
  }
  __syncthreads();
  const int a1 = min(a0 + a_chunk, n_a);
  const cpx* frow = field + t * LDP + l;
  const int y = y0 + t;
  for (int ia = a0; ia < a1; ++ia) {
    const cpx* ra = ramp_a + (size_t)ia * P + l;
    auto load_f = [&](int m) { return cmul(frow[4 * m], ra[4 * m]); };
    cpx v[E];
    line_op<E>(v, load_f, opaque(twist), opaque(mid), opaque(outw), q, l);
    cpx* out = Rw + (fr * (size_t)n_a + ia) * (size_t)(2 * P * P);
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      out[rw_index(q * P + l + 4 * m, y, P)] = v[m];
    });
  }
}

// ---------------------------------------------------------------------------
// Column pass.  Block = one wave = 8 adjacent columns x' of one frame and
// one chunk of modulation points.  Each team accumulates |E|^2 of its
// column over the chunk in registers; the wave then bins b x b through LDS
// and writes its part of the chunk's four pupil images.
template <int E>
__global__ __launch_bounds__(64) void col_pass_kernel(
    const cpx* __restrict__ Rw, const cpx* __restrict__ ramp_b, const int* __restrict__ k_order,
    const int* __restrict__ k_ia, const cpx* __restrict__ twist, const cpx* __restrict__ mid,
    const cpx* __restrict__ outw, float* __restrict__ partial, int n_a, int K, int k_chunk,
    int n_chunks, int n_bin) {
  constexpr int P = 4 * E;
  __shared__ float tile[8 * 2 * P];
  const int lane = threadIdx.x;
  const int t = lane >> 3, q = (lane >> 2) & 1, l = lane & 3;
  const int X0 = blockIdx.x * 8;
  const int chunk = blockIdx.y;
  const size_t fr = blockIdx.z;
  const int xp = X0 + t;
  float acc[E];
  static_for<0, E>([&](auto m_) { acc[decltype(m_)::value] = 0.f; });
  const int kb = chunk * k_chunk;
  const int ke = min(kb + k_chunk, K);
  // Column xp, rows y = l + 4 m: base of the (x'/8, y/4 = m) tiles for this lane.
  const size_t col_off = (size_t)(xp >> 3) * (size_t)(P >> 2) * 32u + (size_t)((xp & 7) * 4 + l);
  for (int kk = kb; kk < ke; ++kk) {
    const int k = k_order[kk];
    const cpx* src = Rw + (fr * (size_t)n_a + k_ia[k]) * (size_t)(2 * P * P) + col_off;
    const cpx* rb = ramp_b + (size_t)k * P + l;
    auto load_f = [&](int m) { return cmul(src[32 * m], rb[4 * m]); };
    cpx v[E];
    line_op<E>(v, load_f, opaque(twist), opaque(mid), opaque(outw), q, l);
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      acc[m] = fmaf(v[m].re, v[m].re, fmaf(v[m].im, v[m].im, acc[m]));
    });
  }
  float* my = tile + (t * 2 + q) * P + l;
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    my[4 * m] = acc[m];
  });
  __syncthreads();
  const int S = P / n_bin;
  const int nbc = 8 / n_bin;
  const int xw = X0 >= P ? 1 : 0;
  const int ix0 = (X0 - xw * P) / n_bin;
  float* dst = partial + (fr * (size_t)n_chunks + chunk) * (size_t)(4 * S * S);
  for (int o = lane; o < nbc * 2 * S; o += 64) {
    const int bc = o / (2 * S);
    const int rem = o - bc * 2 * S;
    const int qq = rem / S;
    const int iy = rem - qq * S;
    float s = 0.f;
    for (int dx = 0; dx < n_bin; ++dx) {
      const float* col = tile + ((bc * n_bin + dx) * 2 + qq) * P + iy * n_bin;
      for (int dy = 0; dy < n_bin; ++dy) s += col[dy];
    }
    dst[(size_t)(xw + 2 * qq) * S * S + (size_t)iy * S + ix0 + bc] = s;
  }
}

// ---------------------------------------------------------------------------
// Slopes.  One block per frame: sum the chunk partials (fixed order),
// scale by 1/K, optionally write the pupils, then the flux normalisation
// (fixed-order tree) and the reference-subtracted slopes.  The partials are
// re-read in the second sweep rather than staged, so any pupil size fits.
__device__ __forceinline__ float chunk_sum(const float* __restrict__ pp, int n_chunks, size_t stride,
                                           size_t idx, float inv_k) {
  float s = 0.f;
  for (int c = 0; c < n_chunks; ++c) s += pp[(size_t)c * stride + idx];
  return s * inv_k;
}

__global__ __launch_bounds__(256) void slopes_kernel(
    const float* __restrict__ partial, int n_chunks, int S, float inv_k,
    const int* __restrict__ valid, int nv, const float* __restrict__ sref, int norm_mode,
    float* __restrict__ pupils, float* __restrict__ slopes) {
  __shared__ float red[256];
  const int tid = threadIdx.x;
  const size_t fr = blockIdx.x;
  const size_t SS = (size_t)S * S;
  const size_t stride = 4 * SS;
  const float* pp = partial + fr * (size_t)n_chunks * stride;
  if (pupils) {
    float* po = pupils + fr * stride;
    for (size_t i = tid; i < stride; i += 256) po[i] = chunk_sum(pp, n_chunks, stride, i, inv_k);
  }
  if (!slopes) return;
  float loc = 0.f;
  if (norm_mode == 0) {
    for (int v = tid; v < nv; v += 256) {
      const size_t j = (size_t)valid[v];
      const float i0 = chunk_sum(pp, n_chunks, stride, j, inv_k);
      const float i1 = chunk_sum(pp, n_chunks, stride, SS + j, inv_k);
      const float i2 = chunk_sum(pp, n_chunks, stride, 2 * SS + j, inv_k);
      const float i3 = chunk_sum(pp, n_chunks, stride, 3 * SS + j, inv_k);
      loc += (i0 + i1) + (i2 + i3);
    }
  }
  red[tid] = loc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  const float mean_flux = red[0] / (float)nv;
  float* so = slopes + fr * 2 * (size_t)nv;
  for (int v = tid; v < nv; v += 256) {
    const size_t j = (size_t)valid[v];
    const float i0 = chunk_sum(pp, n_chunks, stride, j, inv_k);
    const float i1 = chunk_sum(pp, n_chunks, stride, SS + j, inv_k);
    const float i2 = chunk_sum(pp, n_chunks, stride, 2 * SS + j, inv_k);
    const float i3 = chunk_sum(pp, n_chunks, stride, 3 * SS + j, inv_k);
    const float n = norm_mode ? ((i0 + i1) + (i2 + i3)) : mean_flux;
    so[v] = ((i1 + i3) - (i0 + i2)) / n - sref[v];
    so[nv + v] = ((i2 + i3) - (i0 + i1)) / n - sref[nv + v];
  }
}

// ---------------------------------------------------------------------------
// m = alpha R s + beta m.  One wave per row of R; lanes stride the row
// (coalesced), each lane keeps BT batch accumulators, butterfly reduction.
template <int BT>
__global__ __launch_bounds__(256) void recon_kernel(const float* __restrict__ R, int M, int ns,
                                                     const float* __restrict__ s, int B, float alpha,
                                                     float beta, float* __restrict__ m) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wave;
  if (i >= M) return;
  const int b0 = blockIdx.y * BT;
  const int nb = min(BT, B - b0);
  float acc[BT];
#pragma unroll
  for (int bb = 0; bb < BT; ++bb) acc[bb] = 0.f;
  const float* Ri = R + (size_t)i * ns;
  const float* sb = s + (size_t)b0 * ns;
  for (int j = lane; j < ns; j += 64) {
    const float r = Ri[j];
#pragma unroll
    for (int bb = 0; bb < BT; ++bb)
      if (bb < nb) acc[bb] = fmaf(r, sb[(size_t)bb * ns + j], acc[bb]);
  }
#pragma unroll
  for (int bb = 0; bb < BT; ++bb) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[bb] += __shfl_xor(acc[bb], off);
  }
  if (lane == 0) {
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) {
      if (bb < nb) {
        float* mm = m + (size_t)(b0 + bb) * M + i;
        *mm = beta != 0.f ? fmaf(alpha, acc[bb], beta * *mm) : alpha * acc[bb];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
template <int E>
static hipError_t launch_rows(const MeasureArgs& a, hipStream_t st) {
  dim3 grid(a.P / 8, (a.n_a + a.a_chunk - 1) / a.a_chunk, a.B);
  hipLaunchKernelGGL(row_pass_kernel<E>, grid, dim3(64), 0, st, a.opd, a.amp, a.kphase, a.ramp_a,
                     a.twist, a.mid, a.outw, a.Rw, a.n_a, a.a_chunk);
  return hipGetLastError();
}

template <int E>
static hipError_t launch_cols(const MeasureArgs& a, hipStream_t st) {
  dim3 grid(2 * a.P / 8, a.n_chunks, a.B);
  hipLaunchKernelGGL(col_pass_kernel<E>, grid, dim3(64), 0, st, a.Rw, a.ramp_b, a.k_order, a.k_ia,
                     a.twist, a.mid, a.outw, a.partial, a.n_a, a.K, a.k_chunk, a.n_chunks, a.n_bin);
  return hipGetLastError();
}

hipError_t launch_measure(const MeasureArgs& a, hipStream_t st, hipEvent_t* ev) {
  hipError_t e = hipSuccess;
  if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
  switch (a.P / 4) {
    case 8: e = launch_rows<8>(a, st); break;
    case 16: e = launch_rows<16>(a, st); break;
    case 40: e = launch_rows<40>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
  switch (a.P / 4) {
    case 8: e = launch_cols<8>(a, st); break;
    case 16: e = launch_cols<16>(a, st); break;
    case 40: e = launch_cols<40>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
  const int S = a.P / a.n_bin;
  hipLaunchKernelGGL(slopes_kernel, dim3(a.B), dim3(256), 0, st, a.partial, a.n_chunks, S,
                     1.0f / (float)a.K, a.valid, a.nv, a.sref, a.norm_mode, a.pupils, a.slopes);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[3], st)) != hipSuccess) return e;
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

hipError_t launch_recon(const float* R, int M, int ns, const float* s, int B, float alpha,
                        float beta, float* m, hipStream_t st) {
  const int gx = (M + 3) / 4;
  if (B <= 1) {
    hipLaunchKernelGGL(recon_kernel<1>, dim3(gx, B), dim3(256), 0, st, R, M, ns, s, B, alpha, beta, m);
  } else if (B <= 4) {
    hipLaunchKernelGGL(recon_kernel<4>, dim3(gx, 1), dim3(256), 0, st, R, M, ns, s, B, alpha, beta, m);
  } else {
    hipLaunchKernelGGL(recon_kernel<8>, dim3(gx, (B + 7) / 8), dim3(256), 0, st, R, M, ns, s, B,
                       alpha, beta, m);
  }
  return hipGetLastError();
}

}  // namespace pwfs
