/*
 * pwfs.h -- C ABI of the modulated pyramid wavefront-sensor library.
 *
 * The operations follow the sensor chain of the paper's SCAO example
 * (Sec. 4, main file, Tab. 2): the pyramid turns the pupil electric field
 * into pupil-plane intensity with circular modulation (pyr.in_ef ->
 * pyr.out_i), the detector integrates it into pixels (ccd.in_i ->
 * out_pixels), the slope computer turns pixels into slopes using the
 * sub-aperture indices and a slope reference vector (sc.in_pixels ->
 * out_slopes; Tab. 1 "slopec"), and the modal reconstructor multiplies the
 * slopes by the reconstruction matrix (rec.in_slopes -> out_modes;
 * Tab. 1 "modalrec"), whose output feeds the integrator (Tab. 1
 * "control").  Pyramid parameters: Tab. 1 "pyramid" (modulation radius in
 * lambda/D, wavelength).
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - FFT grid N x N, pupil P x P embedded at offset (N-P)/2, circular pupil
 *     of diameter P centred at (P-1)/2 (pixel inside iff r^2 <= (P/2)^2,
 *     optional central obstruction removing r < eps P / 2);
 *   - phase = 2 pi opd[nm] 1e-9 / lambda;
 *   - K modulation points at angles 2 pi k / K, radius r_mod N / P focal
 *     pixels; intensity is the mean over the K points;
 *   - pyramid mask exp(-2 pi i Delta (|u| + |v|) / N) on signed frequency
 *     indices, apex on frequency bin 0, Delta = N / 4; optionally times a
 *     circular field stop (field_stop_lod);
 *   - pupil q = (x side +) + 2 (y side +), each binned b x b to S x S,
 *     S = P / b, stored [q][iy][ix] row-major; or, with det_window = S > 0
 *     (and b = 1), each P x P window resampled to S x S detector pixels of
 *     pitch P / S pupil pixels (a non-integer rebin: detector pixel (j, i)
 *     integrates the piecewise-constant window over
 *     [j P/S, (j+1) P/S) x [i P/S, (i+1) P/S), in pixel-area units);
 *   - valid subapertures: pupil fill fraction of the b x b block (of the
 *     detector pixel's footprint with det_window) >= 0.5, listed as
 *     j = iy * S + ix in ascending order (pwfs_set_valid replaces the list);
 *   - slopes: sx = [(I1 + I3) - (I0 + I2)] / n, sy = [(I2 + I3) - (I0 + I1)] / n
 *     with n the mean total flux over valid subapertures of the same frame
 *     (norm_mode 0) or each subaperture's own total flux (norm_mode 1);
 *     layout [sx over valid ; sy over valid] minus the reference slopes
 *     (slopes of a flat wavefront, measured when the plan is made).
 *
 * Memory: every pointer documented as "device" is a device allocation on
 * the device that was current when the plan was made, owned by the
 * caller; "host" pointers are ordinary host memory.  Streams are
 * hipStream_t passed as void* (NULL = default stream).  All calls return
 * PWFS_OK or a negative status; argument checks run on the host before
 * anything is launched.  There is no CPU fallback: without a usable
 * device the plan call fails with PWFS_ERR_NO_DEVICE.
 */
#ifndef PWFS_H
#define PWFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pwfs_plan_s* pwfs_plan_t;

enum {
  PWFS_OK = 0,
  PWFS_ERR_INVALID_ARG = -1,   /* NULL pointer, non-positive size, inconsistent geometry */
  PWFS_ERR_UNSUPPORTED = -2,   /* geometry outside what the kernels implement            */
  PWFS_ERR_NO_DEVICE = -3,     /* no HIP device visible                                  */
  PWFS_ERR_OUT_OF_MEMORY = -4, /* device allocation failed                               */
  PWFS_ERR_HIP = -5            /* a HIP runtime call or kernel launch failed             */
};

typedef struct {
  int32_t n_fft;      /* N: FFT grid side.  Must equal 4 * n_pupil.                        */
  int32_t n_pupil;    /* P: pupil window in pixels: 32, 64, 128, 160 or 480.               */
  int32_t n_bin;      /* b: detector binning, P % b == 0, b in {1, 2, 4, 8} (or 5, P 480). */
  int32_t n_mod;      /* K: modulation points, 1 <= K <= 1024.                            */
  int32_t face_shift; /* Delta in pixels; 0 selects N / 4 (the only supported value).     */
  int32_t norm_mode;  /* 0: global mean flux over valid subapertures; 1: per subaperture. */
  int32_t batch_max;  /* largest batch the workspace is sized for (larger batches are     */
                      /* processed in slices of batch_max frames).                         */
  int32_t flags;      /* 0 for the default FP64-generated tables and FP64 phase formation.  */
                      /* Precision study only: bit 0 generates the tilt-ramp, twist and   */
                      /* pyramid tables in FP32, bit 1 forms and reduces the phase in     */
                      /* FP32; other bits must be 0.                                       */
  double diameter_m;      /* D (informational: the sensor works in pixels)                */
  double wavelength_m;    /* lambda                                                       */
  double mod_radius_lod;  /* r_mod in lambda / D, >= 0                                    */
  double obstruction;     /* central obstruction, fraction of D, 0 <= eps < 1              */
  int32_t det_window;     /* 0: integer binning by n_bin.  S > 0: each pupil window of P   */
                          /* pixels is resampled to S detector pixels (2 <= S <= P, n_bin */
                          /* must be 1).  The paper's detector (output_resolution 80,     */
                          /* pupils of pup_diam 30 pixels whose centres are pup_dist 36   */
                          /* apart) is S = pup_dist = 36 with a pupil of diameter         */
                          /* P pup_diam / pup_dist pupil pixels: the four windows fill    */
                          /* the central 72 x 72 pixels of the 80 x 80 frame.             */
  int32_t reserved;       /* must be 0                                                    */
  double field_stop_lod;  /* 0: no field stop.  > 0: diameter, in lambda / D (the unit of  */
                          /* mod_radius_lod), of a circular focal-plane stop: the field is */
                          /* kept where u_s^2 + v_s^2 <= R^2, R = field_stop_lod N / (2P)  */
                          /* focal pixels (the paper's pyramid "fov").  The disc is not    */
                          /* separable, so such a plan runs a general 2-D path (three      */
                          /* pruned transform passes per modulation point, about 5 x the   */
                          /* work); n_pupil must be 32, 64 or 160; fixed work split.       */
} pwfs_config_t;

/* Build a plan (the pyramid object of Sec. 4 with the parameters of Tab. 1
 * "pyramid", plus the calibration Sec. 4 requires before a run: the
 * sub-aperture indices and the slope reference of the slope computer, Tab. 1
 * "slopec" pupdata and sn): validates cfg, generates the FP64 tables (tilt
 * ramps, pyramid twiddles), uploads them as FP32, allocates the workspace for
 * batch_max frames and measures the reference slopes of a flat wavefront
 * (synchronises the default stream once).  pupil_amp_host: P * P floats,
 * row-major [y][x], or NULL for the circular pupil described above.
 * On success *out owns every device buffer until pwfs_destroy. */
int pwfs_plan(const pwfs_config_t* cfg, const float* pupil_amp_host, pwfs_plan_t* out);

/* Sizes of a plan: number of valid subapertures, S = P / b and the bytes
 * of device workspace held.  Any output pointer may be NULL. */
int pwfs_plan_info(pwfs_plan_t plan, int32_t* n_valid, int32_t* n_sub, size_t* workspace_bytes);

/* Copy the valid-subaperture list (n_valid int32, ascending j = iy*S+ix)
 * into host memory. */
int pwfs_get_valid(pwfs_plan_t plan, int32_t* idx_host);

/* Replace the valid-subaperture list with n host indices (strictly
 * ascending, each in [0, S * S)), e.g. from a pupil acquisition on a
 * detector frame (the paper's calibration: a flat-wavefront frame taken with
 * a large modulation radius, thresholded).  Reallocates the list and the
 * reference, then measures the reference slopes of a flat wavefront again
 * (noiseless, detector bypassed).  Synchronises the device; must not overlap
 * any other call on this plan.  PWFS_ERR_INVALID_ARG for an empty, unsorted
 * or out-of-range list (the plan keeps its previous list). */
int pwfs_set_valid(pwfs_plan_t plan, const int32_t* idx_host, int32_t n);

/* Copy the current reference slopes (2 * n_valid floats) into host memory. */
int pwfs_get_reference(pwfs_plan_t plan, float* sref_host);

/* Replace the reference slopes with 2 * n_valid floats from device memory
 * (stream-ordered copy), or with zeros when d_sref is NULL. */
int pwfs_set_reference(pwfs_plan_t plan, const float* d_sref, void* stream);

/* Modulated pyramid measurement of B frames: the chain pyr.in_ef ->
 * pyr.out_i -> sc.out_slopes of the paper's main file (Sec. 4, Tab. 2), i.e.
 * the pyramid propagation from wavefront to detector plane that Sec. 6 runs
 * on the GPU, then the slope computer (Tab. 1 "slopec").
 *   d_opd_nm  device, B * P * P float, [frame][y][x], optical path in nm.
 *   d_pupils  device, B * 4 * S * S float, binned pupil images (mean over
 *             modulation points of |E|^2, pupil-plane pixels summed b x b,
 *             unit input amplitude), or NULL to skip writing them.
 *   d_slopes  device, B * 2 * n_valid float, reference-subtracted slopes,
 *             or NULL to skip them.
 * Asynchronous on `stream`.  A plan holds one workspace: calls on the same
 * plan must not overlap on different streams. */
int pwfs_measure(pwfs_plan_t plan, const float* d_opd_nm, int32_t B,
                 float* d_pupils, float* d_slopes, void* stream);

/* pwfs_measure without allocation, for callers that cannot allocate device
 * memory or must not touch the plan's workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, slices, schedules, kernels and results (bit for bit) as
 * pwfs_measure; the workspace regions (row-pass intermediate, chunk
 * partials, pupil field, internal images, detector and field-stop buffers)
 * come from one static device array of PWFS_STATIC_SCRATCH_BYTES per GPU,
 * held until the process ends.  A slice of min(B, batch_max) frames must
 * fit in it (10.2 MB of intermediate per frame at n_pupil 160, i.e. one or
 * two frames per slice; ~0.2 MB at n_pupil 32), else PWFS_ERR_UNSUPPORTED
 * with the bytes needed in pwfs_last_error().  Calls no hipMalloc or
 * hipFree.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, or two host threads) race and give
 * undefined results.  No region needs to start at zero (each call writes
 * every element it reads), so the array's contents between calls do not
 * matter. */
#define PWFS_STATIC_SCRATCH_BYTES (32u << 20)
int pwfs_measure_static(pwfs_plan_t plan, const float* d_opd_nm, int32_t B,
                        float* d_pupils, float* d_slopes, void* stream);

/* Copy the pupil amplitude used by the plan (P * P floats, [y][x]) into
 * host memory. */
int pwfs_get_pupil(pwfs_plan_t plan, float* amp_host);

/* Per-kernel timing of pwfs_measure.  With enable != 0 every later
 * pwfs_measure on this plan binds HIP events to its kernels on the caller's
 * stream (hipExtLaunchKernel: an event takes a kernel's own start or end
 * time, no marker is queued between kernels): start and end of the row
 * segment (pupil field and row pass), of the column pass (the field-stop
 * path: its column and output passes) and of the finish (chunk sum to
 * slopes).  The previous record is discarded; enable == 0 stops recording.
 * pwfs_timing_read waits for the recorded events and returns the summed
 * segment durations in milliseconds and the number of pwfs_measure batch
 * slices recorded.  Any output pointer may be NULL. */
int pwfs_timing_enable(pwfs_plan_t plan, int enable);
int pwfs_timing_read(pwfs_plan_t plan, double* ms_row, double* ms_col, double* ms_slopes,
                     int64_t* n_slices);

/* Detector (the paper's CCD object, Sec. 4, Tab. 1 "ccd": it integrates the
 * intensity over the exposure into pixels with photon noise and readout noise;
 * the quantum efficiency, band, source magnitude and exposure enter through
 * the photo-electron budget).  With a detector set, pwfs_measure passes the
 * binned images through it: d_pupils receives detector pixels (electrons) and
 * the slopes are computed from them (the reference slopes stay the noiseless
 * flat-wavefront ones).
 *   electrons_per_frame  mean photo-electrons that a flat wavefront deposits in
 *                        the four binned pupil images (flux x band x collecting
 *                        area x exposure x QE); the gain is this budget divided
 *                        by the sum of the plan's flat-wavefront images;
 *                        0 removes the detector (noiseless images).
 *   readout_noise_e      Gaussian readout noise per binned pixel, electrons RMS.
 *   seed                 key of the random numbers.
 * Pixel = k + ron z with k ~ Poisson(gain I) and z ~ N(0, 1), drawn from the
 * counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 * SC'11) with key = seed and counter = (pixel index within the frame, frame
 * index low word, frame index high word, draw word): the noise of a frame
 * depends only on (seed, frame index, pixel), not on batching or schedule.
 * The count multiplies uniforms (x + 1/2) 2^-32 in FP64 (draw words 0, 1, ...)
 * until the product falls to exp(-lam / n) or below, for each of
 * n = ceil(lam / 500) equal pieces of lam = gain I; above lam = 1e4 it is the
 * normal approximation floor(lam + sqrt(lam) z' + 1/2), clipped at 0.  z and
 * z' are Box-Muller deviates of draw word 2^31.
 * Frame indices: pwfs_measure gives its B frames the indices f, f+1, ...,
 * f+B-1 with f the plan's frame counter, then advances the counter by B;
 * pwfs_set_detector resets it to 0, pwfs_set_frame_counter sets it.
 * PWFS_ERR_INVALID_ARG for a negative or non-finite budget or noise. */
typedef struct {
  double electrons_per_frame;
  double readout_noise_e;
  uint64_t seed;
} pwfs_detector_t;

int pwfs_set_detector(pwfs_plan_t plan, const pwfs_detector_t* det /* NULL = noiseless */);
/* Gain (electrons per unit intensity, 0 without a detector) and the next frame index. */
int pwfs_get_detector(pwfs_plan_t plan, float* gain, uint64_t* next_frame);
int pwfs_set_frame_counter(pwfs_plan_t plan, uint64_t frame);

/* The detector alone: d_pixels [B][4][S][S] from noiseless images
 * d_intensity [B][4][S][S] (device), frame b using index frame0 + b.
 * Requires a detector set on the plan (PWFS_ERR_INVALID_ARG otherwise).
 * Asynchronous on `stream`; does not touch the plan's frame counter. */
int pwfs_detect(pwfs_plan_t plan, const float* d_intensity, int32_t B, uint64_t frame0, float* d_pixels,
                void* stream);

/* Shack-Hartmann sensor (the paper's second sensor type, Sec. 1 and Sec. 6;
 * the geometry is fixed by this library): n_sub x n_sub square subapertures
 * of s = n_pupil / n_sub pixels; valid subapertures by the sensor's
 * fill-fraction rule (>= 0.5).  For each the field E = A exp(i phi) is
 * zero-padded to M = pad s and
 *   spot[v][u] = |sum_{y,x} E[y][x] exp(-2 pi i ((v - M/2) y + (u - M/2) x) / M)|^2
 * (one spot pixel = lambda / (pad d)); the slopes are the centre of gravity
 * over the M x M box, [cx over valid ; cy over valid] in spot pixels, minus
 * the slopes of a flat wavefront (measured at creation).  Supported: s <= 8,
 * pad 2 or 4, pad s <= 32, n_pupil <= 1024.  d_spots [B][n_valid][M][M] and
 * d_slopes [B][2 n_valid] (device, either may be NULL).  Asynchronous on
 * `stream`; a sensor may not run on two streams at once. */
typedef struct pwfs_sh_s* pwfs_sh_t;
typedef struct {
  int32_t n_pupil;
  int32_t n_sub;
  int32_t pad;
  int32_t batch_max;
  double wavelength_m;
  double obstruction;
} pwfs_sh_config_t;

int pwfs_sh_create(const pwfs_sh_config_t* cfg, const float* pupil_amp_host, pwfs_sh_t* out);
int pwfs_sh_info(pwfs_sh_t sh, int32_t* n_valid, int32_t* spot_side);
int pwfs_sh_get_valid(pwfs_sh_t sh, int32_t* idx_host);
int pwfs_sh_get_reference(pwfs_sh_t sh, float* sref_host);
int pwfs_sh_measure(pwfs_sh_t sh, const float* d_opd_nm, int32_t B, float* d_spots, float* d_slopes, void* stream);
void pwfs_sh_destroy(pwfs_sh_t sh);

/* PSF camera (the paper's PSF object, Sec. 4, Tab. 1 "psf": the image of
 * the residual wavefront at a science wavelength with a padding factor, its
 * Strehl ratio, and its integration over the run).
 *   PSF[v][u] = |FFT2(A exp(i phi))[v - N/2][u - N/2]|^2 / (sum A)^2
 * on the N x N grid, N = pad * n_pupil (one lambda/D = pad pixels), the pupil
 * field zero-padded, phi = 2 pi opd[nm] 1e-9 / wavelength, frequency indices
 * modulo N, zero frequency at (N/2, N/2): a flat wavefront gives exactly 1 there
 * and the value at (N/2, N/2) is the Strehl ratio.  Supported: n_pupil 32,
 * 64 or 160, pad 2, 4 or 8.  The pupil amplitude is the same circle as the
 * sensor plan's (or the caller's P x P host array). */
typedef struct pwfs_psf_s* pwfs_psf_t;
typedef struct {
  int32_t n_pupil;
  int32_t pad;
  int32_t batch_max;   /* workspace size in frames */
  int32_t reserved;    /* must be 0 */
  double wavelength_m;
  double obstruction;
} pwfs_psf_config_t;

int pwfs_psf_create(const pwfs_psf_config_t* cfg, const float* pupil_amp_host, pwfs_psf_t* out);
/* N, the side of the image. */
int pwfs_psf_info(pwfs_psf_t cam, int32_t* n_image);
/* PSFs of B residual screens d_opd_nm [B][P][P] (device, nm).
 *   accumulate == 0: d_psf [B][N][N] receives each frame's PSF;
 *   accumulate != 0: d_psf [N][N] is read and receives d_psf + sum over the
 *                    B frames (added in frame order: a long-exposure image).
 *   d_strehl [B] (may be NULL): |sum A exp(i phi)|^2 / (sum A)^2 per frame.
 * Either output may be NULL.  Asynchronous on `stream`; a camera may not run
 * on two streams at once (shared workspace). */
int pwfs_psf_compute(pwfs_psf_t cam, const float* d_opd_nm, int32_t B, int32_t accumulate, float* d_psf,
                     float* d_strehl, void* stream);
void pwfs_psf_destroy(pwfs_psf_t cam);

/* Work split ("schedule") that pwfs_measure uses for a slice of B frames
 * (1 <= B <= batch_max; a call with more frames than batch_max runs in
 * slices of batch_max and a last, smaller slice): a_chunk distinct x tilts per
 * row-pass block and k_chunk modulation points per column-pass block.  The
 * modulation sum of the pyramid intensity (mean over the K points, Sec. 4,
 * Tab. 1 "pyramid") is accumulated per chunk and the chunks are added in
 * order, so a schedule changes only the FP32 summation order: results agree
 * to rounding and are bitwise reproducible for a fixed schedule.
 * pwfs_get_schedule returns the schedule in force (the library's default
 * unless one was set or tuned for this B).  pwfs_set_schedule fixes one;
 * a_chunk = k_chunk = 0 restores the default; PWFS_ERR_INVALID_ARG when
 * a_chunk is outside [1, number of distinct x tilts], k_chunk outside
 * [1, n_mod], or the chunk partials would not fit the plan's workspace. */
int pwfs_get_schedule(pwfs_plan_t plan, int32_t B, int32_t* a_chunk, int32_t* k_chunk);
int pwfs_set_schedule(pwfs_plan_t plan, int32_t B, int32_t a_chunk, int32_t k_chunk);

/* Lane form of the line kernels for slices of B frames: 8 (a line on two
 * 4-lane quads, one per half-band projection, P/4 samples per lane) or 32 (a
 * line on two 16-lane rows, P/16 samples per lane, the quad DFT_4 steps done
 * across lanes).  n_pupil 128 and 480 always use 32; 32, 64 use 8; at 160
 * both exist (8 by default; 32 keeps more waves busy for a few frames).  Only
 * the FP32 rounding differs.  PWFS_ERR_UNSUPPORTED for a form the geometry
 * does not have or a field-stop plan, PWFS_ERR_INVALID_ARG for lanes other
 * than 8 or 32. */
int pwfs_get_schedule_lanes(pwfs_plan_t plan, int32_t B, int32_t* lanes);
int pwfs_set_schedule_lanes(pwfs_plan_t plan, int32_t B, int32_t lanes);

/* Autotuner: times the row pass for every distinct number of x-tilt chunks
 * and then the column pass (with the chunk reduction and the slopes) for
 * every distinct number of modulation chunks that fits the workspace, on B
 * flat frames, best of `reps` launches each (1..1000), and keeps the
 * fastest schedule for slices of B frames (a candidate must beat the best
 * so far by 2 %); at n_pupil 160 it does so for both lane forms and keeps
 * the faster.  It allocates and frees a temporary input and output of
 * B frames and waits for `stream`: a set-up call, not for the hot path.
 * ms_default / ms_tuned (may be NULL) receive the measured time of one
 * B-frame call with the default and with the chosen schedule. */
int pwfs_autotune(pwfs_plan_t plan, int32_t B, int32_t reps, void* stream, double* ms_default,
                  double* ms_tuned);

/* Modal reconstruction and integration, m = alpha * R s + beta * m for each
 * of B vectors: the modal reconstructor's product with its matrix (Tab. 1
 * "modalrec", rec.in_slopes -> out_modes in Tab. 2) and the integrator's
 * update (Tab. 1 "control": alpha = gain, beta = 1); also the DM projection
 * opd -= B_KL u (alpha = -1, beta = 1 with R = B_KL).
 *   d_R  device, M * n_s float, row-major [mode][slope].
 *   d_s  device, B * n_s float.
 *   d_m  device, B * M float, read (when beta != 0) and written.
 * FP32 with FP32 accumulation in a fixed order (bitwise reproducible):
 * vector FMAs for B <= 16, FP32 MFMA for larger batches.
 * Asynchronous on `stream`. */
int recon_apply(const float* d_R, int32_t M, int32_t n_s, const float* d_s, int32_t B,
                float alpha, float beta, float* d_m, void* stream);

/* Release every device buffer of the plan (synchronises its device). */
void pwfs_destroy(pwfs_plan_t plan);

/* Static description of a status code. */
const char* pwfs_strerror(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char* pwfs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PWFS_H */
