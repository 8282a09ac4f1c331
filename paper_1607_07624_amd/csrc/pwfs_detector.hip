// pwfs_detector.hip -- detector step (photon and readout noise) of the pyramid sensor, gfx950.
#include "pwfs_launch.h"

#include <cstdint>

namespace pwfs {

// ---------------------------------------------------------------------------
// Detector (the paper's CCD step: photon noise, readout noise, quantum
// efficiency folded into the gain).  One thread per binned pixel:
//   lam = gain * I (FP64 product of FP32 values), k ~ Poisson(lam),
//   pixel = k + ron z, z ~ N(0, 1).
// Counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11), key =
// seed, counter = (pixel, frame low word, frame high word, draw word d).  The
// count multiplies uniforms u = (x + 1/2) 2^-32 in FP64 (draw words d = 0, 1,
// ... in order, four uniforms each) until the product falls to exp(-lam/n) or
// below, for each of n = ceil(lam / 500) equal pieces; above lam = 1e4 it is
// floor(lam + sqrt(lam) z' + 1/2) clipped at 0.  z and z' are Box-Muller
// deviates of the draw word 2^31 (uniform pairs 1-2 and 3-4).  Only IEEE
// products and one FP64 exp take the integer decision.
__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double u01(uint32_t x) { return ((double)x + 0.5) * 2.3283064365386963e-10; }

__global__ __launch_bounds__(256) void detector_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                       int npix, uint64_t frame0, float gain, float ron,
                                                       uint64_t seed) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const size_t b = blockIdx.y;
  if (j >= npix) return;
  const uint64_t f = frame0 + b;
  const uint32_t flo = (uint32_t)f, fhi = (uint32_t)(f >> 32);
  const uint32_t klo = (uint32_t)seed, khi = (uint32_t)(seed >> 32);
  const double lam = (double)gain * (double)in[b * (size_t)npix + j];
  uint32_t w[4] = {(uint32_t)j, flo, fhi, 0x80000000u};
  philox4x32_10(w, klo, khi);
  constexpr double two_pi = 6.283185307179586476925286766559;
  const double z = sqrt(-2.0 * log(u01(w[0]))) * cos(two_pi * u01(w[1]));
  double k = 0.0;  // whole numbers, exact in FP64 up to 2^53
  if (lam > 1.0e4) {
    const double z2 = sqrt(-2.0 * log(u01(w[2]))) * cos(two_pi * u01(w[3]));
    k = fmax(0.0, floor(lam + sqrt(lam) * z2 + 0.5));
  } else if (lam > 0.0) {
    const double npieces = ceil(lam / 500.0);
    const double L = exp(-(lam / npieces));
    double p = 1.0, piece = 0.0;
    uint32_t t = 0;
    uint32_t buf[4] = {0u, 0u, 0u, 0u};
    while (piece < npieces) {
      if ((t & 3u) == 0u) {
        buf[0] = (uint32_t)j;
        buf[1] = flo;
        buf[2] = fhi;
        buf[3] = t >> 2;
        philox4x32_10(buf, klo, khi);
      }
      const uint32_t x = (t & 3u) == 0u ? buf[0] : (t & 3u) == 1u ? buf[1] : (t & 3u) == 2u ? buf[2] : buf[3];
      ++t;
      p *= u01(x);
      if (p <= L) {
        piece += 1.0;
        p = 1.0;
      } else {
        k += 1.0;
      }
    }
  }
  out[b * (size_t)npix + j] = (float)(k + (double)ron * z);
}

hipError_t launch_detector(const float* intensity, float* pixels, int npix, int B, uint64_t frame0, float gain,
                           float ron, uint64_t seed, hipStream_t st, hipEvent_t stop) {
  if (B == 0) return hipSuccess;
  return launch_k(detector_kernel, dim3((npix + 255) / 256, B), dim3(256), 0, st, nullptr, stop, intensity, pixels,
                  npix, frame0, gain, ron, seed);
}

}  // namespace pwfs
