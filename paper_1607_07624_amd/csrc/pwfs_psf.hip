// pwfs_psf.hip -- PSF camera of the residual wavefront (gfx950).
//
// PSF[v][u] = |FFT2(A exp(i phi))|^2 / (sum A)^2 on the N = pad P grid, zero
// frequency at (N/2, N/2).  The zero-padded transform of a line of P samples
// splits by the residue of the output index,
//   X[pad u2 + u1] = DFT_P( f[x] w_N^{u1 x} )[u2],   u1 < pad, u2 < P,
// so a line is `pad` DFTs of length P = 4E.  A DFT_P is held by a quad, lane
// l holding x = l + 4 m (m < E): in-lane DFT_E, twiddle w_P^{l k1}, DFT_4
// across the quad (two DPP butterflies), after which lane l holds
// u2 = k1 + E rev(l), rev = (0, 2, 1, 3).  A wave holds 16 quads.
//   row pass     each pupil row (the other rows are zero) -> Z[frame][u][y];
//   column pass  each column u -> |X|^2, scaled and shifted to the centred
//                image; with `accumulate` each lane sums its pixels over the
//                frames in order and adds them to the caller's image.
// The Strehl ratio |sum A exp(i phi)|^2 / (sum A)^2 (the PSF at the centre)
// is a separate fixed-order FP64 sum per frame.
#include "pwfs_common.h"
#include "pwfs_launch.h"

#include <algorithm>
#include <cstdint>

namespace pwfs {

// twpad [pad][P] = w_N^{u1 x};  twp [4][E] = w_P^{l k1}.
template <int E>
__global__ __launch_bounds__(256) void psf_row_kernel(const cpx* __restrict__ field, const cpx* __restrict__ twpad,
                                                      const cpx* __restrict__ twp, cpx* __restrict__ Z, int pad) {
  constexpr int P = 4 * E;
  constexpr int RG = P / 16;                        // groups of 16 rows
  const int N = pad * P;
  const int lane = threadIdx.x & 63;
  const int wg = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int u1 = wg / RG;
  if (u1 >= pad) return;                            // no barriers in this kernel
  const int y = (wg - u1 * RG) * 16 + (lane >> 2);
  const int l = lane & 3;
  const size_t fr = blockIdx.y;
  const cpx* frow = field + (fr * P + y) * (size_t)P + l;
  const cpx* tw = twpad + (size_t)u1 * P + l;
  cpx v[E];
  static_for<0, E>([&](auto m_) {
    constexpr int m = decltype(m_)::value;
    v[m] = cmul(frow[4 * m], tw[4 * m]);
  });
  fence();
  const float sA = (l & 2) ? -1.f : 1.f, sB = (l & 1) ? -1.f : 1.f;
  dft_quad<E>(v, twp + l * E, sA, sB, l == 3);
  cpx* zc = Z + fr * (size_t)N * P + y;
  const int base = pad * E * rev2(l) + u1;          // u = pad (k1 + E rev(l)) + u1
  static_for<0, E>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    zc[(size_t)(base + pad * k) * P] = v[k];
  });
}

template <int E>
__global__ __launch_bounds__(256) void psf_col_kernel(const cpx* __restrict__ Z, const cpx* __restrict__ twpad,
                                                      const cpx* __restrict__ twp, float* __restrict__ psf, int pad,
                                                      int B, int accumulate, float inv_norm) {
  constexpr int P = 4 * E;
  const int N = pad * P;
  const int CG = N / 16;                            // groups of 16 columns
  const int lane = threadIdx.x & 63;
  const int wg = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int v1 = wg / CG;
  if (v1 >= pad) return;
  const int u = (wg - v1 * CG) * 16 + (lane >> 2);
  const int l = lane & 3;
  const cpx* tw = twpad + (size_t)v1 * P + l;
  const float sA = (l & 2) ? -1.f : 1.f, sB = (l & 1) ? -1.f : 1.f;
  const int vbase = pad * E * rev2(l) + v1;         // v = pad (k1 + E rev(l)) + v1
  const int us = (u + N / 2) % N;
  float acc[E];
  static_for<0, E>([&](auto k_) { acc[decltype(k_)::value] = 0.f; });
  const int b0 = accumulate ? 0 : (int)blockIdx.y;
  const int b1 = accumulate ? B : b0 + 1;
  for (int b = b0; b < b1; ++b) {
    const cpx* zc = Z + (size_t)b * N * P + (size_t)u * P + l;
    cpx v[E];
    static_for<0, E>([&](auto m_) {
      constexpr int m = decltype(m_)::value;
      v[m] = cmul(zc[4 * m], tw[4 * m]);
    });
    fence();
    dft_quad<E>(v, twp + l * E, sA, sB, l == 3);
    if (accumulate) {
      static_for<0, E>([&](auto k_) {
        constexpr int k = decltype(k_)::value;
        acc[k] += fmaf(v[k].re, v[k].re, v[k].im * v[k].im);
      });
    } else {
      float* img = psf + (size_t)b * N * N;
      static_for<0, E>([&](auto k_) {
        constexpr int k = decltype(k_)::value;
        const int vs = (vbase + pad * k + N / 2) % N;
        img[(size_t)vs * N + us] = fmaf(v[k].re, v[k].re, v[k].im * v[k].im) * inv_norm;
      });
    }
  }
  if (accumulate) {
    static_for<0, E>([&](auto k_) {
      constexpr int k = decltype(k_)::value;
      const int vs = (vbase + pad * k + N / 2) % N;
      float* o = psf + (size_t)vs * N + us;
      *o = fmaf(acc[k], inv_norm, *o);
    });
  }
}

// Strehl ratio per frame: fixed-order FP64 sums of the field.
__global__ __launch_bounds__(256) void strehl_kernel(const cpx* __restrict__ field, int PP, double inv_norm,
                                                     float* __restrict__ sr) {
  __shared__ double sre[256], sim[256];
  const int tid = threadIdx.x;
  const size_t fr = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int i = tid; i < PP; i += 256) {
    const cpx c = field[fr * PP + i];
    re += (double)c.re;
    im += (double)c.im;
  }
  sre[tid] = re;
  sim[tid] = im;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      sre[tid] += sre[tid + st];
      sim[tid] += sim[tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) sr[fr] = (float)((sre[0] * sre[0] + sim[0] * sim[0]) * inv_norm);
}

template <int E>
static hipError_t launch_psf_e(const PsfArgs& a, hipStream_t st) {
  constexpr int P = 4 * E;
  const int N = a.pad * P;
  hipLaunchKernelGGL(psf_row_kernel<E>, dim3((P / 16 * a.pad + 3) / 4, a.B), dim3(256), 0, st, a.field, a.twpad,
                     a.twp, a.Z, a.pad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(psf_col_kernel<E>, dim3((N / 16 * a.pad + 3) / 4, a.accumulate ? 1 : a.B), dim3(256), 0, st,
                     a.Z, a.twpad, a.twp, a.psf, a.pad, a.B, a.accumulate, a.inv_norm);
  return hipGetLastError();
}

hipError_t launch_psf(const PsfArgs& a, hipStream_t st) {
  hipError_t e = launch_field_raw(a.opd, a.amp, a.kphase, a.P, a.B, a.field, st);
  if (e != hipSuccess) return e;
  if (a.psf) {
    switch (a.P) {
      case 32: e = launch_psf_e<8>(a, st); break;
      case 64: e = launch_psf_e<16>(a, st); break;
      case 160: e = launch_psf_e<40>(a, st); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  if (a.strehl) {
    hipLaunchKernelGGL(strehl_kernel, dim3(a.B), dim3(256), 0, st, a.field, a.P * a.P, (double)a.inv_norm_d,
                       a.strehl);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace pwfs
