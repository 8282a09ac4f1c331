// pwfs_sh.hip -- Shack-Hartmann sensor (gfx950).
//
// For each valid subaperture (s x s pupil pixels) the field is zero-padded to
// M = pad s and  spot[v][u] = |sum_{y,x} E[y][x] w_M^{(v - M/2) y + (u - M/2) x}|^2,
// w_M = exp(-2 pi i / M) (the zero frequency at (M/2, M/2)); the centroid is
// the centre of gravity over the M x M box in spot pixels, minus the flat
// reference.  One wave per (frame, subaperture): the wave stages its s x s
// field in LDS, each lane computes spot pixels u + M v = lane + 64 i by the
// direct DFT (s^2 products against a twiddle table), and the wave reduces
// the three moments with a fixed butterfly.
#include "pwfs_common.h"
#include "pwfs_launch.h"

#include <cstdint>

namespace pwfs {

__global__ __launch_bounds__(256) void sh_kernel(const cpx* __restrict__ field, int P, int S, int s, int M,
                                                 const int* __restrict__ valid, int nv, const cpx* __restrict__ twm,
                                                 const float* __restrict__ sref, float* __restrict__ spots,
                                                 float* __restrict__ slopes) {
  __shared__ cpx s_e[4][64];
  __shared__ cpx s_tw[32];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const size_t fr = blockIdx.y;
  if (tid < M) s_tw[tid] = twm[tid];
  const int vi = blockIdx.x * 4 + wave;
  const bool active = vi < nv;
  if (active && lane < s * s) {
    const int j = valid[vi];
    const int iy = j / S, ix = j - iy * S;
    const int y = lane / s, x = lane - y * s;
    s_e[wave][lane] = field[(fr * P + (size_t)(iy * s + y)) * P + ix * s + x];
  }
  __syncthreads();
  if (!active) return;
  const int MM = M * M;
  float m0 = 0.f, mx = 0.f, my = 0.f;
  for (int p = lane; p < MM; p += 64) {
    const int v = p / M, u = p - v * M;
    const int cu = u - M / 2, cv = v - M / 2;
    float re = 0.f, im = 0.f;
    for (int y = 0; y < s; ++y) {
      const int ty = ((cv * y) % M + M) % M;
      for (int x = 0; x < s; ++x) {
        const int t = (ty + ((cu * x) % M + M)) % M;
        const cpx e = s_e[wave][y * s + x], w = s_tw[t];
        re = fmaf(e.re, w.re, fmaf(-e.im, w.im, re));
        im = fmaf(e.re, w.im, fmaf(e.im, w.re, im));
      }
    }
    const float I = fmaf(re, re, im * im);
    if (spots) spots[(fr * nv + vi) * (size_t)MM + p] = I;
    m0 += I;
    mx = fmaf(I, (float)cu, mx);
    my = fmaf(I, (float)cv, my);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m0 += __shfl_xor(m0, off);
    mx += __shfl_xor(mx, off);
    my += __shfl_xor(my, off);
  }
  if (lane == 0 && slopes) {
    float* so = slopes + fr * 2 * (size_t)nv;
    so[vi] = mx / m0 - sref[vi];
    so[nv + vi] = my / m0 - sref[nv + vi];
  }
}

hipError_t launch_sh(const ShArgs& a, hipStream_t st) {
  hipError_t e = launch_field_raw(a.opd, a.amp, a.kphase, a.P, a.B, a.field, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sh_kernel, dim3((a.nv + 3) / 4, a.B), dim3(256), 0, st, a.field, a.P, a.S, a.s, a.M, a.valid,
                     a.nv, a.twm, a.sref, a.spots, a.slopes);
  return hipGetLastError();
}

}  // namespace pwfs
