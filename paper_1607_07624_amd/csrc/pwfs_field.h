// pwfs_field.h -- the pupil field A exp(i phi) of one pixel, shared by the
// field kernel and the row passes that form the field in their prologue.
#ifndef PWFS_FIELD_H
#define PWFS_FIELD_H

#include "pwfs_dft.h"

namespace pwfs {

// phi = 2 pi opd 1e-9 / lambda (kphase = 2 pi 1e-9 / lambda) formed and
// reduced modulo 2 pi in FP64, then FP32 sincos.  fp32_phase (precision
// study only): the phase formed in FP32 and passed to sincosf unreduced.
__device__ __forceinline__ cpx pupil_field(float opd, float A, double kphase, int fp32_phase) {
  constexpr double two_pi = 6.283185307179586476925286766559;
  constexpr double inv_two_pi = 0.15915494309189533576888376337251;
  float sn, cs;
  if (fp32_phase) {
    sincosf(opd * (float)kphase, &sn, &cs);
  } else {
    const double th = (double)opd * kphase;
    const double red = fma(-rint(th * inv_two_pi), two_pi, th);
    sincosf((float)red, &sn, &cs);
  }
  return {A * cs, A * sn};
}

}  // namespace pwfs

#endif  // PWFS_FIELD_H
