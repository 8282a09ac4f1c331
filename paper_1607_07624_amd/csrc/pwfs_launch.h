// pwfs_launch.h -- argument bundle between the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>

namespace pwfs {

struct cpx;

struct MeasureArgs {
  // geometry
  int P, n_bin, K, n_a, nv, norm_mode;
  // batch slice and work split
  int B, a_chunk, k_chunk, n_chunks;
  double kphase;  // 2 pi 1e-9 / lambda
  int fp32_phase; // precision study: form and reduce the phase in FP32
  int lines16;    // 32-lane teams (16-lane projections): always for P = 128, 480; optional at P = 160
  // inputs / outputs
  const float* opd;
  float* pupils;       // [B][4][S][S]: the caller's buffer or the plan's scratch
  float* slopes;       // [B][2 nv] or NULL
  // plan tables
  const float* amp;
  const cpx* in_a;     // [n_a][2][P]  r_a(x) w_N^{(2q+1)x}
  const cpx* f_a;      // [n_a][P]     -r_a(x) (finishing factor of the low-face projection)
  const cpx* in_b;     // [K][2][P]    r_b(y) w_N^{(2q+1)y}
  const cpx* f_b;      // [K][P]       -r_b(y)
  const cpx* mid;      // [4][P/4][2] folded mix coefficients (A/2, B/2) per lane; 32-lane teams: [16][E][2]
  const cpx* tw16;     // 32-lane teams only: [4][E] subgroup twiddles w_{4E}^{l2 k1}
  const cpx* outw;     // [2][P]
  const int* k_order;  // [K]
  const int* k_ia;     // [K]
  const int* valid;    // [nv]
  const float* sref;   // [2 nv]
  // workspace
  cpx* field;          // [B][P][P]    A exp(i phi)
  cpx* Rw;             // [B][n_a][2P][P]
  float* partial;      // [B][n_chunks][4][S][S] (per-column [B][n_chunks][2][2P][S], see below)
  // detector (det_on == 0: the pupils are the noiseless intensity)
  int det_on;
  float det_gain, det_ron;   // electrons per unit intensity, readout noise (e- RMS)
  uint64_t det_seed, frame0; // Philox key, frame index of the slice's first frame
  float* intensity;          // [B][4][S][S] scratch for the noiseless images when det_on
  // rebin_S > 0 (detector window, or the field-stop path): the chunk sum goes
  // to fullres [B][4][P][P], then each window is resampled to rebin_S pixels
  float* fullres;
  // circular field stop (fs_on): general 2-D path of pwfs_fstop.hip; the
  // modulation chunks of its output pass reuse k_chunk / n_chunks
  int fs_on, fs_r2max, rebin_S;
  const cpx* fs_rx;    // [K][P]  r_a(x)
  const cpx* fs_ry;    // [K][P]  r_b(y)
  const cpx* fs_tw4n;  // [4][P]  w_N^{u1 x}
  const cpx* fs_twp;   // [4][E]  w_P^{l k1}
  const cpx* fs_twi;   // [4][P]  (-i)^{v1} w_N^{-v1 t} / N
  const cpx* fs_py;    // [N]     exp(-2 pi i Delta |v_s| / N)
  cpx* fs_Z;           // [B][K][N][P]
  cpx* fs_W;           // [B][K][2P][N]
  // timing (all NULL unless timed): start and stop of the row segment (field
  // and row pass), the column segment and the finish (chunk sum to slopes),
  // bound to the first and last kernel of each (launch_k)
  hipEvent_t tev[6];
};

// Kernel launch with optional timing events bound to the kernel itself
// (hipExtLaunchKernelGGL): `start` takes the kernel's start time and `stop`
// its end time, so no marker packets are queued between the kernels of a
// call and the events measure kernel execution only.
template <typename... KArgs, typename... Args>
inline hipError_t launch_k(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t st,
                           hipEvent_t start, hipEvent_t stop, Args... args) {
  if (start || stop)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, start, stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
  return hipGetLastError();
}

// PSF camera: field at the science wavelength, zero-padded 2-D transform,
// |.|^2 / (sum A)^2 centred (or accumulated over the frames), Strehl ratios.
struct PsfArgs {
  int P, pad, B, accumulate;
  double kphase;       // 2 pi 1e-9 / lambda
  float inv_norm;      // 1 / (sum A)^2
  double inv_norm_d;
  const float* opd;    // [B][P][P] nm
  const float* amp;    // [P][P]
  const cpx* twpad;    // [pad][P]  w_N^{u1 x}
  const cpx* twp;      // [4][P/4]  w_P^{l k1}
  cpx* field;          // [B][P][P]
  cpx* Z;              // [B][N][P]
  float* psf;          // [B][N][N], or [N][N] accumulated; may be NULL
  float* strehl;       // [B] or NULL
};

// Shack-Hartmann: field, per-subaperture zero-padded spots, centroids.
struct ShArgs {
  int P, S, s, M, nv, B;
  double kphase;
  const float* opd;    // [B][P][P] nm
  const float* amp;    // [P][P]
  const int* valid;    // [nv] j = iy S + ix
  const cpx* twm;      // [M] w_M^k
  const float* sref;   // [2 nv]
  cpx* field;          // [B][P][P]
  float* spots;        // [B][nv][M][M] or NULL
  float* slopes;       // [B][2 nv] or NULL
};

// ev: NULL, or six events that take the start and end times of the row
// segment, the column segment and the finish (MeasureArgs::tev).
hipError_t launch_measure(const MeasureArgs& a, hipStream_t stream, hipEvent_t* ev);
// The three passes of the field-stop path (pwfs_fstop.hip), after the field;
// its row transforms end the row segment, its column and output passes form
// the column segment.
hipError_t launch_fstop_passes(const MeasureArgs& a, hipStream_t stream);
// Pieces of launch_measure: the pupil field (one frame slice), and the row and
// column passes of the long-line kernels (P = 128, 480).
hipError_t launch_field(const MeasureArgs& a, hipStream_t stream);
hipError_t launch_field_raw(const float* opd, const float* amp, double kphase, int P, int B, cpx* field,
                            hipStream_t stream);
hipError_t launch_psf(const PsfArgs& a, hipStream_t stream);
hipError_t launch_sh(const ShArgs& a, hipStream_t stream);
hipError_t launch_rows_long(const MeasureArgs& a, hipStream_t stream);
hipError_t launch_cols_long(const MeasureArgs& a, hipStream_t stream);
// Long lines with a binning that does not divide 8 columns: the column pass
// writes per-column partials [B][n_chunks][2][2P][S], finished here.
bool partials_by_column(int P, int n_bin);
hipError_t launch_reduce_cols(const MeasureArgs& a, float* pupils, hipStream_t stream, hipEvent_t stop);
hipError_t launch_fill(float* p, size_t n, float v, hipStream_t stream);
hipError_t launch_detector(const float* intensity, float* pixels, int npix, int B, uint64_t frame0, float gain,
                           float ron, uint64_t seed, hipStream_t stream, hipEvent_t stop = nullptr);
hipError_t launch_recon(const float* R, int M, int ns, const float* s, int B, float alpha, float beta,
                        float* m, hipStream_t stream);

}  // namespace pwfs
