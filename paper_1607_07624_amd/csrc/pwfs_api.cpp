// pwfs_api.cpp -- C ABI of the modulated pyramid sensor: validation, FP64 table
// generation, workspace management and launch sequencing.
#include "../../include/pwfs.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pwfs_launch.h"

namespace pwfs {
struct alignas(8) cpx {
  float re, im;
};
}  // namespace pwfs

using pwfs::cpx;

struct pwfs_sh_s {
  int device = 0, P = 0, S = 0, s = 0, M = 0, nv = 0, batch_max = 0;
  double kphase = 0.0;
  std::vector<int> valid;
  float* amp = nullptr;
  int* d_valid = nullptr;
  cpx* twm = nullptr;
  float* sref = nullptr;
  cpx* field = nullptr;
  float* zero_opd = nullptr;
  float* tmp = nullptr;
};

struct pwfs_psf_s {
  int device = 0, P = 0, pad = 0, N = 0, batch_max = 0;
  double kphase = 0.0, inv_norm = 0.0;
  float* amp = nullptr;
  cpx* twpad = nullptr;
  cpx* twp = nullptr;
  cpx* field = nullptr;
  cpx* Z = nullptr;
};

namespace {

// Binary circular pupil of diameter P centred at (P-1)/2 (inside iff
// r^2 <= (P/2)^2), minus a central obstruction of diameter eps P.
void circle_pupil(int P, double eps, std::vector<float>& amp) {
  const double c = 0.5 * (P - 1), r2o = 0.25 * P * P;
  const double r2i = 0.25 * eps * eps * P * P;
  for (int y = 0; y < P; ++y)
    for (int x = 0; x < P; ++x) {
      const double r2 = (x - c) * (x - c) + (y - c) * (y - c);
      const bool in = r2 <= r2o && (eps <= 0.0 || r2 >= r2i);
      amp[(size_t)y * P + x] = in ? 1.0f : 0.0f;
    }
}

// P = 128 and 480 use the 32-lane line teams (P / 16 samples per lane).
bool long_lines(int P) { return P == 128 || P == 480; }

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PWFS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace pwfs {
bool inject_alloc_failure();
}

namespace {

int dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) return PWFS_OK;
  if (pwfs::inject_alloc_failure()) return fail(PWFS_ERR_OUT_OF_MEMORY, std::string("injected OOM: ") + what);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(PWFS_ERR_OUT_OF_MEMORY, std::string("hipMalloc(") + what + ", " +
                                            std::to_string(bytes) + " B): " + hipGetErrorString(e));
  }
  return PWFS_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

namespace pwfs {
int set_last_error(int status, const std::string& msg) { return fail(status, msg); }

// Test hook of the device allocators (sensor and network): with the
// environment variable PWFS_FAULT_INJECT = "oom" every allocation fails,
// with "oom:N" the N-th allocation after the variable took that value fails
// (and later ones succeed), so that each partial-allocation clean-up path of
// a create call can be driven.  Unset: no effect.
bool inject_alloc_failure() {
  static std::mutex mu;
  static std::string spec;
  static long count = 0;
  const char* v = std::getenv("PWFS_FAULT_INJECT");
  std::lock_guard<std::mutex> lk(mu);
  const std::string now = v ? v : "";
  if (now != spec) {
    spec = now;
    count = 0;
  }
  if (spec == "oom") return true;
  if (spec.rfind("oom:", 0) == 0) {
    const long n = std::atol(spec.c_str() + 4);
    return ++count == n;
  }
  return false;
}
}  // namespace pwfs

struct pwfs_plan_s {
  pwfs_config_t cfg{};
  int device = 0;
  int N = 0, P = 0, E = 0, S = 0, b = 0, K = 0, n_a = 0, nv = 0, batch_max = 0;
  int Sb = 0;                                   // column-pass images: P / b (S unless det_window)
  int Sd = 0;                                   // det_window (0: integer binning)
  bool fs_on = false;                           // circular field stop: general 2-D path
  int fs_r2max = 0;                             // stop: inside iff u_s^2 + v_s^2 <= fs_r2max
  cpx *fs_rx = nullptr, *fs_ry = nullptr, *fs_tw4n = nullptr, *fs_twp = nullptr, *fs_twi = nullptr,
      *fs_py = nullptr, *fs_Z = nullptr, *fs_W = nullptr;
  double kphase = 0.0;
  std::vector<int> valid;
  // device tables
  float* amp = nullptr;
  cpx* in_a = nullptr;
  cpx* f_a = nullptr;
  cpx* in_b = nullptr;
  cpx* f_b = nullptr;
  cpx* mid = nullptr;
  cpx* tw16 = nullptr;
  cpx* outw = nullptr;
  int* k_order = nullptr;
  int* k_ia = nullptr;
  int* d_valid = nullptr;
  float* sref = nullptr;
  // workspace
  cpx* Rw = nullptr;
  float* partial = nullptr;
  float* pupils = nullptr;
  float* fullres = nullptr;                     // [batch_max][4][P][P] with det_window
  cpx* field = nullptr;
  float* zero_opd = nullptr;
  float* tmp_slopes = nullptr;
  size_t ws_bytes = 0;
  size_t partial_cap = 0;                       // floats in `partial`
  // detector
  bool det_on = false;
  double det_electrons = 0.0, det_ron = 0.0, ref_total = 0.0;  // ref_total: flat-wavefront image sum
  uint64_t det_seed = 0, frame_next = 0;
  float det_gain = 0.f;
  float* pixels = nullptr;                      // [batch_max][4][S][S] detector output scratch
  std::map<int, std::array<int, 2>> sched;      // slice size -> {a_chunk, k_chunk}
  std::map<int, int> teams32;                   // slice size -> 1: 32-lane teams at P = 160
  cpx* mid16 = nullptr;                         // P = 160: mix table of the 32-lane form
  std::vector<float> amp_host;
  // per-kernel timing
  bool timing = false;
  std::vector<std::array<hipEvent_t, 6>> ev_used, ev_free;  // start/stop of row, column, finish
};

namespace {

// Lane form of a slice of B frames: 32-lane teams always for P = 128 and 480,
// at P = 160 when chosen (pwfs_set_schedule_lanes or the autotuner), else
// 8-lane teams (quads).
bool teams32(const pwfs_plan_s* p, int B) {
  if (long_lines(p->P)) return true;
  if (p->P != 160) return false;
  auto it = p->teams32.find(B);
  return it != p->teams32.end() && it->second != 0;
}

// Default work split for a slice of B frames: enough waves per pass to keep
// several in flight on every SIMD of the 256-CU chip.  A wave holds 8 lines
// (8-lane teams) or 2 lines (32-lane teams).
void default_split(const pwfs_plan_s* p, int B, int* a_chunk, int* k_chunk) {
  const long target = 2048;
  const long lines_per_wave = teams32(p, B) ? 2 : 8;
  const long row_waves = (long)p->P / lines_per_wave * p->n_a * B;
  int ac = (int)std::max<long>(1, row_waves / target);
  *a_chunk = std::min(ac, p->n_a);
  const long col_tiles = (long)(2 * p->P) / lines_per_wave * B;   // waves per modulation chunk
  long nc = (target + col_tiles - 1) / col_tiles;
  nc = std::max<long>(1, std::min<long>(nc, p->K));
  *k_chunk = (int)((p->K + nc - 1) / nc);
}

// Split used by pwfs_measure: a schedule set for this slice size, else the default.
void split_work(const pwfs_plan_s* p, int B, int* a_chunk, int* k_chunk, int* n_chunks) {
  auto it = p->sched.find(B);
  if (it != p->sched.end()) {
    *a_chunk = it->second[0];
    *k_chunk = it->second[1];
  } else {
    default_split(p, B, a_chunk, k_chunk);
  }
  *n_chunks = (p->K + *k_chunk - 1) / *k_chunk;
}

// Floats of one (frame, chunk) partial: the chunk's four binned images, or
// per-column row-binned sums when the binning does not divide a long-line
// column block.
size_t partial_per_chunk(const pwfs_plan_s* p) {
  return pwfs::partials_by_column(p->P, p->b) ? (size_t)4 * p->P * p->Sb : (size_t)4 * p->Sb * p->Sb;
}

// A schedule is usable when its chunk partials fit the plan's workspace.
bool schedule_fits(const pwfs_plan_s* p, int B, int a_chunk, int k_chunk) {
  if (B < 1 || B > p->batch_max || a_chunk < 1 || a_chunk > p->n_a || k_chunk < 1 || k_chunk > p->K) return false;
  const size_t nc = (size_t)((p->K + k_chunk - 1) / k_chunk);
  return (size_t)B * nc * partial_per_chunk(p) <= p->partial_cap;
}

int validate(const pwfs_config_t* c) {
  if (!c) return fail(PWFS_ERR_INVALID_ARG, "cfg is NULL");
  if (c->flags & ~3) return fail(PWFS_ERR_INVALID_ARG, "unknown flag bits");
  if (c->n_pupil <= 0 || c->n_fft <= 0 || c->n_bin <= 0 || c->n_mod <= 0 || c->batch_max <= 0)
    return fail(PWFS_ERR_INVALID_ARG, "sizes must be positive");
  if (c->n_pupil % c->n_bin != 0) return fail(PWFS_ERR_INVALID_ARG, "n_pupil must be a multiple of n_bin");
  if (!(c->wavelength_m > 0.0) || !(c->mod_radius_lod >= 0.0) || !(c->obstruction >= 0.0) ||
      !(c->obstruction < 1.0) || !std::isfinite(c->wavelength_m) || !std::isfinite(c->mod_radius_lod))
    return fail(PWFS_ERR_INVALID_ARG, "wavelength, modulation radius or obstruction out of range");
  if (c->norm_mode != 0 && c->norm_mode != 1) return fail(PWFS_ERR_INVALID_ARG, "norm_mode must be 0 or 1");
  if (c->face_shift < 0) return fail(PWFS_ERR_INVALID_ARG, "face_shift must be >= 0");
  if (c->n_mod > 1024) return fail(PWFS_ERR_UNSUPPORTED, "n_mod > 1024");
  if (c->n_fft != 4 * c->n_pupil) return fail(PWFS_ERR_UNSUPPORTED, "n_fft must equal 4 * n_pupil");
  if (c->face_shift != 0 && c->face_shift != c->n_fft / 4)
    return fail(PWFS_ERR_UNSUPPORTED, "face_shift must be n_fft / 4");
  const int P = c->n_pupil;
  if (!(P == 32 || P == 64 || P == 160 || P == 128 || P == 480))
    return fail(PWFS_ERR_UNSUPPORTED, "n_pupil must be 32, 64, 128, 160 or 480");
  const bool b_pow2 = c->n_bin == 1 || c->n_bin == 2 || c->n_bin == 4 || c->n_bin == 8;
  if (!(b_pow2 || (long_lines(P) && c->n_bin == 5 && P % 10 == 0)))
    return fail(PWFS_ERR_UNSUPPORTED, "n_bin must be 1, 2, 4 or 8 (or 5 with n_pupil 480)");
  if (c->batch_max > 65535) return fail(PWFS_ERR_UNSUPPORTED, "batch_max > 65535");
  if (c->reserved != 0) return fail(PWFS_ERR_INVALID_ARG, "reserved must be 0");
  if (!(c->field_stop_lod >= 0.0) || !std::isfinite(c->field_stop_lod))
    return fail(PWFS_ERR_INVALID_ARG, "field_stop_lod must be finite and >= 0");
  if (c->field_stop_lod > 0.0 && !(P == 32 || P == 64 || P == 160))
    return fail(PWFS_ERR_UNSUPPORTED, "a field stop needs n_pupil 32, 64 or 160");
  if (c->det_window != 0) {
    if (c->det_window < 2 || c->det_window > P)
      return fail(PWFS_ERR_INVALID_ARG, "det_window must be 0 or in [2, n_pupil]");
    if (c->n_bin != 1) return fail(PWFS_ERR_INVALID_ARG, "det_window needs n_bin 1");
  }
  return PWFS_OK;
}

void free_plan(pwfs_plan_s* p) {
  if (!p) return;
  DeviceGuard g(p->device);
  void* ptrs[] = {p->amp, p->in_a, p->f_a, p->in_b, p->f_b, p->mid, p->tw16, p->outw, p->k_order, p->k_ia,
                  p->d_valid, p->sref, p->Rw, p->partial, p->pupils, p->pixels, p->field, p->zero_opd,
                  p->tmp_slopes, p->fullres, p->mid16, p->fs_rx, p->fs_ry, p->fs_tw4n, p->fs_twp, p->fs_twi, p->fs_py,
                  p->fs_Z, p->fs_W};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (auto* pool : {&p->ev_used, &p->ev_free})
    for (auto& a : *pool)
      for (hipEvent_t ev : a) (void)hipEventDestroy(ev);
  delete p;
}

// Device memory a slice works in beyond its inputs and outputs: the plan's
// own workspace, or a caller-supplied region (measure_in_workspace).
struct Workspace {
  cpx* Rw;            // row-pass intermediate
  float* partial;     // chunk partials
  float* pupils;      // images when the caller passes none (noiseless images with a detector)
  float* pixels;      // detector output when the caller passes no pupils
  float* fullres;     // full-resolution images (det_window, field stop)
  cpx* field;         // pupil field
  cpx* fs_Z;          // field-stop row transforms
  cpx* fs_W;          // field-stop column transforms
};

Workspace plan_workspace(const pwfs_plan_s* p) {
  return Workspace{p->Rw, p->partial, p->pupils, p->pixels, p->fullres, p->field, p->fs_Z, p->fs_W};
}

pwfs::MeasureArgs slice_args(const pwfs_plan_s* p, const float* opd, int b0, int Bs, float* pupils, float* slopes,
                             const float* sref, const Workspace& ws) {
  pwfs::MeasureArgs a{};
  a.P = p->P;
  a.n_bin = p->b;
  a.K = p->K;
  a.n_a = p->n_a;
  a.nv = p->nv;
  a.norm_mode = p->cfg.norm_mode;
  a.B = Bs;
  split_work(p, Bs, &a.a_chunk, &a.k_chunk, &a.n_chunks);
  a.lines16 = teams32(p, Bs) ? 1 : 0;
  a.kphase = p->kphase;
  a.fp32_phase = (p->cfg.flags & 2) != 0;
  a.opd = opd + (size_t)b0 * p->P * p->P;
  a.pupils = pupils ? pupils + (size_t)b0 * 4 * p->S * p->S : (p->det_on ? ws.pixels : ws.pupils);
  a.det_on = p->det_on ? 1 : 0;
  a.det_gain = p->det_gain;
  a.det_ron = (float)p->det_ron;
  a.det_seed = p->det_seed;
  a.frame0 = p->frame_next + (uint64_t)b0;
  a.intensity = ws.pupils;
  a.slopes = slopes ? slopes + (size_t)b0 * 2 * p->nv : nullptr;
  a.amp = p->amp;
  a.in_a = p->in_a;
  a.f_a = p->f_a;
  a.in_b = p->in_b;
  a.f_b = p->f_b;
  a.mid = (p->P == 160 && a.lines16) ? p->mid16 : p->mid;
  a.tw16 = p->tw16;
  a.outw = p->outw;
  a.k_order = p->k_order;
  a.k_ia = p->k_ia;
  a.valid = p->d_valid;
  a.sref = sref;
  a.Rw = ws.Rw;
  a.field = ws.field;
  a.partial = ws.partial;
  a.fullres = ws.fullres;
  a.rebin_S = (p->Sd > 0 || p->fs_on) ? p->S : 0;
  if (p->fs_on) {
    // Output pass of the field-stop path: modulation chunks for ~2048 blocks.
    const long rows = 2L * p->P / 16 * Bs;
    int nc = (int)std::max<long>(1, std::min<long>(p->K, (2048 + rows - 1) / rows));
    a.k_chunk = (p->K + nc - 1) / nc;
    a.n_chunks = (p->K + a.k_chunk - 1) / a.k_chunk;
    a.fs_on = 1;
    a.fs_r2max = p->fs_r2max;
    a.fs_rx = p->fs_rx;
    a.fs_ry = p->fs_ry;
    a.fs_tw4n = p->fs_tw4n;
    a.fs_twp = p->fs_twp;
    a.fs_twi = p->fs_twi;
    a.fs_py = p->fs_py;
    a.fs_Z = ws.fs_Z;
    a.fs_W = ws.fs_W;
  }
  return a;
}

int run_measure(pwfs_plan_s* p, const float* opd, int B, float* pupils, float* slopes,
                const float* sref, hipStream_t st, const Workspace* ws_in = nullptr) {
  const Workspace ws = ws_in ? *ws_in : plan_workspace(p);
  for (int b0 = 0; b0 < B; b0 += p->batch_max) {
    const int Bs = std::min(p->batch_max, B - b0);
    pwfs::MeasureArgs a = slice_args(p, opd, b0, Bs, pupils, slopes, sref, ws);
    hipEvent_t* ev = nullptr;
    if (p->timing) {
      std::array<hipEvent_t, 6> evs{};
      if (!p->ev_free.empty()) {
        evs = p->ev_free.back();
        p->ev_free.pop_back();
      } else {
        for (auto& x : evs) {
          hipError_t ce = hipEventCreate(&x);
          if (ce != hipSuccess) return hip_fail(ce, "hipEventCreate");
        }
      }
      p->ev_used.push_back(evs);
      ev = p->ev_used.back().data();
    }
    hipError_t e = pwfs::launch_measure(a, st, ev);
    if (e != hipSuccess) return hip_fail(e, "pwfs_measure launch");
  }
  if (p->det_on) p->frame_next += (uint64_t)B;
  return PWFS_OK;
}

}  // namespace

namespace pwfs {

// Carves the regions of one slice of Bs frames out of `base` (256-byte
// aligned regions, in the order of Workspace); returns the bytes used.
// With base == nullptr only the size is computed.
size_t carve_workspace(const pwfs_plan_s* p, int Bs, char* base, Workspace* ws) {
  int ac, kc, nc;
  split_work(p, Bs, &ac, &kc, &nc);
  if (p->fs_on) {
    // the field-stop output pass picks its own modulation chunks
    pwfs::MeasureArgs a = slice_args(p, nullptr, 0, Bs, nullptr, nullptr, nullptr, Workspace{});
    nc = a.n_chunks;
  }
  const size_t P = (size_t)p->P, N = 4 * P, S = (size_t)p->S, K = (size_t)p->K, B = (size_t)Bs;
  const size_t sizes[8] = {
      p->fs_on ? 0 : B * p->n_a * 2 * P * P * sizeof(cpx),
      B * nc * partial_per_chunk(p) * sizeof(float),
      B * 4 * S * S * sizeof(float),
      p->det_on ? B * 4 * S * S * sizeof(float) : 0,
      (p->Sd > 0 || p->fs_on) ? B * 4 * P * P * sizeof(float) : 0,
      B * P * P * sizeof(cpx),
      p->fs_on ? B * K * N * P * sizeof(cpx) : 0,
      p->fs_on ? B * K * 2 * P * N * sizeof(cpx) : 0,
  };
  void** slots[8] = {(void**)&ws->Rw, (void**)&ws->partial, (void**)&ws->pupils, (void**)&ws->pixels,
                     (void**)&ws->fullres, (void**)&ws->field, (void**)&ws->fs_Z, (void**)&ws->fs_W};
  size_t off = 0;
  for (int i = 0; i < 8; ++i) {
    *slots[i] = (base && sizes[i]) ? (void*)(base + off) : nullptr;
    off += (sizes[i] + 255) / 256 * 256;
  }
  return off;
}

// pwfs_measure with every workspace region taken from `ws_base` (ws_bytes
// long, 256-byte aligned) instead of the plan's; the same slices, schedules
// and kernels, so the results are those of pwfs_measure bit for bit.
int measure_in_workspace(pwfs_plan_t p, const float* d_opd_nm, int32_t B, float* d_pupils, float* d_slopes,
                         void* ws_base, size_t ws_bytes, void* stream) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (B < 0) return fail(PWFS_ERR_INVALID_ARG, "B must be >= 0");
  if (B == 0 || (!d_pupils && !d_slopes)) return PWFS_OK;
  if (!d_opd_nm) return fail(PWFS_ERR_INVALID_ARG, "d_opd_nm is NULL");
  if (!ws_base || ((uintptr_t)ws_base & 255) != 0) return fail(PWFS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  const int Bs = std::min<int>(B, p->batch_max);
  Workspace ws{};
  const size_t need = carve_workspace(p, Bs, nullptr, &ws);
  if (need > ws_bytes)
    return fail(PWFS_ERR_UNSUPPORTED, "slice of " + std::to_string(Bs) + " frames needs " + std::to_string(need) +
                                          " bytes of workspace, the static scratch holds " + std::to_string(ws_bytes) +
                                          " (use pwfs_measure, or a plan with a smaller batch_max)");
  carve_workspace(p, Bs, (char*)ws_base, &ws);
  DeviceGuard g(p->device);
  return run_measure(p, d_opd_nm, B, d_pupils, d_slopes, p->sref, (hipStream_t)stream, &ws);
}

int plan_device(pwfs_plan_t p) { return p ? p->device : -1; }

}  // namespace pwfs

extern "C" {

const char* pwfs_strerror(int status) {
  switch (status) {
    case PWFS_OK: return "ok";
    case PWFS_ERR_INVALID_ARG: return "invalid argument";
    case PWFS_ERR_UNSUPPORTED: return "unsupported geometry";
    case PWFS_ERR_NO_DEVICE: return "no HIP device";
    case PWFS_ERR_OUT_OF_MEMORY: return "out of device memory";
    case PWFS_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* pwfs_last_error(void) { return g_last_error.c_str(); }

int pwfs_plan(const pwfs_config_t* cfg, const float* pupil_amp_host, pwfs_plan_t* out) {
  g_last_error.clear();
  if (!out) return fail(PWFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int st = validate(cfg);
  if (st != PWFS_OK) return st;

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(PWFS_ERR_NO_DEVICE, "no HIP device visible");
  }
  auto* p = new pwfs_plan_s();
  p->cfg = *cfg;
  if ((e = hipGetDevice(&p->device)) != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  const int N = cfg->n_fft, P = cfg->n_pupil, K = cfg->n_mod, b = cfg->n_bin;
  p->N = N;
  p->P = P;
  p->E = P / 4;
  p->b = b;
  p->fs_on = cfg->field_stop_lod > 0.0;
  p->Sb = p->fs_on ? P : P / b;
  p->Sd = cfg->det_window;
  p->S = p->Sd > 0 ? p->Sd : P / b;
  p->K = K;
  p->batch_max = cfg->batch_max;
  p->kphase = 2.0 * M_PI * 1e-9 / cfg->wavelength_m;

  // Pupil amplitude.
  std::vector<float> amp((size_t)P * P);
  if (pupil_amp_host) {
    for (size_t i = 0; i < amp.size(); ++i) {
      if (!std::isfinite(pupil_amp_host[i])) {
        delete p;
        return fail(PWFS_ERR_INVALID_ARG, "pupil amplitude has non-finite values");
      }
      amp[i] = pupil_amp_host[i];
    }
  } else {
    circle_pupil(P, cfg->obstruction, amp);
  }
  // Valid subapertures: fill fraction of the b x b block (of the detector
  // pixel's footprint with det_window, overlaps in units of 1 / S) >= 0.5.
  const int S = p->S;
  if (p->Sd > 0) {
    auto ov = [&](int j, int y) {
      return (double)(std::min((y + 1) * S, (j + 1) * P) - std::max(y * S, j * P));
    };
    for (int iy = 0; iy < S; ++iy)
      for (int ix = 0; ix < S; ++ix) {
        double s = 0.0;
        for (int y = (iy * P) / S; y < ((iy + 1) * P + S - 1) / S; ++y)
          for (int x = (ix * P) / S; x < ((ix + 1) * P + S - 1) / S; ++x)
            s += ov(iy, y) * ov(ix, x) * (double)amp[(size_t)y * P + x];
        if (s >= 0.5 * (double)P * P) p->valid.push_back(iy * S + ix);   // area P^2 / S^2 in units 1/S^2
      }
  } else {
    for (int iy = 0; iy < S; ++iy)
      for (int ix = 0; ix < S; ++ix) {
        double s = 0.0;
        for (int dy = 0; dy < b; ++dy)
          for (int dx = 0; dx < b; ++dx) s += amp[(size_t)(iy * b + dy) * P + ix * b + dx];
        if (s >= 0.5 * b * b) p->valid.push_back(iy * S + ix);
      }
  }
  p->nv = (int)p->valid.size();
  p->amp_host = amp;
  if (p->nv == 0) {
    delete p;
    return fail(PWFS_ERR_INVALID_ARG, "pupil has no valid subaperture");
  }

  // Modulation: k and K-k share the x tilt a_k = rho cos(2 pi k / K).
  const double rho = cfg->mod_radius_lod * (double)N / (double)P;
  p->n_a = K / 2 + 1;
  std::vector<int> k_ia(K), k_order;
  for (int k = 0; k < K; ++k) k_ia[k] = std::min(k, K - k);
  // The pairs (k, K-k), which share one x tilt, come first and adjacent, so a
  // chunk of an even number of points stages each of its x tilts once; the
  // unpaired points (k = 0 and, for even K, k = K/2) come last.
  for (int ia = 1; ia < p->n_a; ++ia)
    if (K - ia != ia) {
      k_order.push_back(ia);
      k_order.push_back(K - ia);
    }
  k_order.push_back(0);
  if (K % 2 == 0 && K / 2 != 0) k_order.push_back(K / 2);
  if ((int)k_order.size() != K) {
    delete p;
    return fail(PWFS_ERR_INVALID_ARG, "internal: modulation ordering");
  }
  // Tilt ramps r(x) = exp(i 2 pi t (x - xc) / N) (FP64), negated (the line
  // operator finishes the low face as y_H - f = -y_L, whose intensity is that
  // of y_L) and times the twist w_N^{(2q+1) x} of the two quads.
  const double xc = 0.5 * (P - 1);
  const bool t32 = (cfg->flags & 1) != 0;   // precision study: FP32-generated tables
  std::vector<std::complex<double>> tw(2 * (size_t)P);
  for (int q = 0; q < 2; ++q)
    for (int x = 0; x < P; ++x) {
      const long n = ((long)(2 * q + 1) * x) % N;
      const double ang = -2.0 * M_PI * (double)n / (double)N;
      const float angf = -2.0f * (float)M_PI * (float)n / (float)N;
      tw[(size_t)q * P + x] = t32 ? std::complex<double>(std::cos(angf), std::sin(angf))
                                  : std::complex<double>(std::cos(ang), std::sin(ang));
    }
  auto ramp = [&](double tilt, int x) {
    if (t32) {
      const float turns = (float)tilt * ((float)x - (float)xc) / (float)N;
      const float f = turns - std::floor(turns);
      const float ang = 2.0f * (float)M_PI * f;
      return std::complex<double>(std::cos(ang), std::sin(ang));
    }
    const double turns = tilt * ((double)x - xc) / (double)N;
    const double f = turns - std::floor(turns);
    return std::complex<double>(std::cos(2.0 * M_PI * f), std::sin(2.0 * M_PI * f));
  };
  auto to32 = [](std::complex<double> z) { return cpx{(float)z.real(), (float)z.imag()}; };
  std::vector<cpx> in_a((size_t)p->n_a * 2 * P), f_a((size_t)p->n_a * P), in_b((size_t)K * 2 * P),
      f_b((size_t)K * P);
  for (int ia = 0; ia < p->n_a; ++ia) {
    const double a = rho * std::cos(2.0 * M_PI * (double)ia / (double)K);
    for (int x = 0; x < P; ++x) {
      const std::complex<double> r = ramp(a, x);
      f_a[(size_t)ia * P + x] = to32(-r);
      for (int q = 0; q < 2; ++q) in_a[((size_t)ia * 2 + q) * P + x] = to32(r * tw[(size_t)q * P + x]);
    }
  }
  for (int k = 0; k < K; ++k) {
    const double bk = rho * std::sin(2.0 * M_PI * (double)k / (double)K);
    for (int y = 0; y < P; ++y) {
      const std::complex<double> r = ramp(bk, y);
      f_b[(size_t)k * P + y] = to32(-r);
      for (int q = 0; q < 2; ++q) in_b[((size_t)k * 2 + q) * P + y] = to32(r * tw[(size_t)q * P + y]);
    }
  }
  // Pyramid line-operator tables: output twiddles (4/N) w_N^{-(2q+1) j} and,
  // per quad lane l and in-lane frequency k, the folded mix coefficients
  // A_l / 2 = (1 - i) conj(w_l) w_{l+1} / 2, B_l / 2 = (1 + i) conj(w_l) w_{l-1} / 2
  // with w_l = w_P^{l k} (FP64, lanes mod 4).
  std::vector<cpx> outw(2 * (size_t)P), mid(8 * (size_t)p->E);
  for (int q = 0; q < 2; ++q)
    for (int x = 0; x < P; ++x) {
      const long n = ((long)(2 * q + 1) * x) % N;
      const double ang = t32 ? (double)(2.0f * (float)M_PI * (float)n / (float)N) : 2.0 * M_PI * (double)n / (double)N;
      const double sc = 4.0 / (double)N;
      outw[(size_t)q * P + x] = t32 ? cpx{(float)sc * std::cos((float)ang), (float)sc * std::sin((float)ang)}
                                    : cpx{(float)(sc * std::cos(ang)), (float)(sc * std::sin(ang))};
    }
  auto wlk = [&](int l, int k) {
    const long n = ((long)l * k) % P;
    if (t32) {
      const float angf = -2.0f * (float)M_PI * (float)n / (float)P;
      return std::complex<double>(std::cos(angf), std::sin(angf));
    }
    const double ang = -2.0 * M_PI * (double)n / (double)P;
    return std::complex<double>(std::cos(ang), std::sin(ang));
  };
  auto mix = [&](int l, int k, cpx* dst) {
    dst[0] = to32(std::complex<double>(0.5, -0.5) * std::conj(wlk(l, k)) * wlk((l + 1) & 3, k));
    dst[1] = to32(std::complex<double>(0.5, 0.5) * std::conj(wlk(l, k)) * wlk((l + 3) & 3, k));
  };
  const bool lines32 = long_lines(P);
  const bool have32 = lines32 || P == 160;       // tables of the 32-lane form
  const int E16 = P / 16;
  std::vector<cpx> tw16(have32 ? 4 * (size_t)E16 : 1), mid16(P == 160 ? 8 * (size_t)p->E : 0);
  if (!lines32) {
    for (int l = 0; l < 4; ++l)
      for (int k = 0; k < p->E; ++k) mix(l, k, &mid[((size_t)l * p->E + k) * 2]);
  }
  if (have32) {
    // Lane 4 l1 + l2 of a 16-lane row holds in-lane frequency k1 of outer
    // lane l1 at t' = k1 + E16 rev(l2) after the subgroup DFT_4; its
    // twiddle before that DFT is w_{4 E16}^{l2 k1}.
    std::vector<cpx>& m16 = lines32 ? mid : mid16;
    const int rev2[4] = {0, 2, 1, 3};
    for (int l16 = 0; l16 < 16; ++l16)
      for (int k1 = 0; k1 < E16; ++k1) mix(l16 >> 2, k1 + E16 * rev2[l16 & 3], &m16[((size_t)l16 * E16 + k1) * 2]);
    for (int l2 = 0; l2 < 4; ++l2)
      for (int k1 = 0; k1 < E16; ++k1) {
        const long n = (long)l2 * k1;
        if (t32) {
          const float angf = -2.0f * (float)M_PI * (float)n / (float)(4 * E16);
          tw16[(size_t)l2 * E16 + k1] = cpx{std::cos(angf), std::sin(angf)};
        } else {
          const double ang = -2.0 * M_PI * (double)n / (double)(4 * E16);
          tw16[(size_t)l2 * E16 + k1] = cpx{(float)std::cos(ang), (float)std::sin(ang)};
        }
      }
  }

  // Field-stop path tables (pwfs_fstop.hip): ramps alone (not negated), the
  // residue twists of the zero-padded transforms w_N^{r x}, the inverse ones
  // with the window phase and 1/N, (-i)^r w_N^{-r x} / N, the quad twiddles
  // w_P^{l k1} and the pyramid factor of one axis; the stop is the disc
  // u_s^2 + v_s^2 <= R^2 of radius R = field_stop_lod N / (2P) focal pixels.
  std::vector<cpx> fs_rx, fs_ry, fs_tw4n, fs_twp, fs_twi, fs_py;
  if (p->fs_on) {
    fs_rx.resize((size_t)K * P);
    fs_ry.resize((size_t)K * P);
    for (int k = 0; k < K; ++k) {
      const double ak = rho * std::cos(2.0 * M_PI * (double)k / (double)K);
      const double bk = rho * std::sin(2.0 * M_PI * (double)k / (double)K);
      for (int x = 0; x < P; ++x) {
        fs_rx[(size_t)k * P + x] = to32(ramp(ak, x));
        fs_ry[(size_t)k * P + x] = to32(ramp(bk, x));
      }
    }
    fs_tw4n.resize(4 * (size_t)P);
    fs_twi.resize(4 * (size_t)P);
    for (int r = 0; r < 4; ++r)
      for (int x = 0; x < P; ++x) {
        const long n = ((long)r * x) % N;
        const double ang = -2.0 * M_PI * (double)n / (double)N;
        fs_tw4n[(size_t)r * P + x] = cpx{(float)std::cos(ang), (float)std::sin(ang)};
        const double angi = -0.5 * M_PI * (double)r - ang;
        fs_twi[(size_t)r * P + x] = cpx{(float)(std::cos(angi) / N), (float)(std::sin(angi) / N)};
      }
    fs_twp.resize(4 * (size_t)p->E);
    for (int l = 0; l < 4; ++l)
      for (int k1 = 0; k1 < p->E; ++k1) {
        const double ang = -2.0 * M_PI * (double)(((long)l * k1) % P) / (double)P;
        fs_twp[(size_t)l * p->E + k1] = cpx{(float)std::cos(ang), (float)std::sin(ang)};
      }
    fs_py.resize(N);
    const int delta = N / 4;
    for (int v = 0; v < N; ++v) {
      const long vs = v < N / 2 ? v : v - N;
      const double ang = -2.0 * M_PI * (double)(((long)delta * std::labs(vs)) % N) / (double)N;
      fs_py[v] = cpx{(float)std::cos(ang), (float)std::sin(ang)};
    }
    const double R = 0.5 * cfg->field_stop_lod * (double)N / (double)P;
    const double lim = 2.0 * (N / 2) * (N / 2);
    p->fs_r2max = R * R >= lim ? (int)lim : (int)std::floor(R * R);
  }

  // Device buffers.
  int bm = cfg->batch_max;
  int ac, kc, nc;
  // Chunk partials for any schedule (up to K chunks per frame).
  size_t partial_elems = 0;
  const size_t ppc = partial_per_chunk(p);
  for (int B = 1; B <= bm; ++B) {
    split_work(p, B, &ac, &kc, &nc);
    partial_elems = std::max(partial_elems, (size_t)B * nc * ppc);
  }
  partial_elems = std::max(partial_elems, (size_t)bm * K * ppc);
  p->partial_cap = partial_elems;
  const size_t rw_elems = (size_t)bm * p->n_a * 2 * P * P;
  struct A { void** ptr; size_t bytes; const char* what; } allocs[] = {
      {(void**)&p->amp, amp.size() * sizeof(float), "amp"},
      {(void**)&p->in_a, in_a.size() * sizeof(cpx), "in_a"},
      {(void**)&p->f_a, f_a.size() * sizeof(cpx), "f_a"},
      {(void**)&p->in_b, in_b.size() * sizeof(cpx), "in_b"},
      {(void**)&p->f_b, f_b.size() * sizeof(cpx), "f_b"},
      {(void**)&p->mid, mid.size() * sizeof(cpx), "mid"},
      {(void**)&p->tw16, tw16.size() * sizeof(cpx), "tw16"},
      {(void**)&p->mid16, mid16.size() * sizeof(cpx), "mid16"},
      {(void**)&p->outw, outw.size() * sizeof(cpx), "outw"},
      {(void**)&p->k_order, (size_t)K * sizeof(int), "k_order"},
      {(void**)&p->k_ia, (size_t)K * sizeof(int), "k_ia"},
      {(void**)&p->d_valid, (size_t)p->nv * sizeof(int), "valid"},
      {(void**)&p->sref, (size_t)2 * p->nv * sizeof(float), "sref"},
      {(void**)&p->Rw, p->fs_on ? 0 : rw_elems * sizeof(cpx), "row-pass workspace"},
      {(void**)&p->partial, partial_elems * sizeof(float), "pupil partials"},
      {(void**)&p->pupils, (size_t)bm * 4 * S * S * sizeof(float), "pupil scratch"},
      {(void**)&p->pixels, (size_t)bm * 4 * S * S * sizeof(float), "detector scratch"},
      {(void**)&p->fullres, (p->Sd > 0 || p->fs_on) ? (size_t)bm * 4 * P * P * sizeof(float) : 0,
       "full-resolution images"},
      {(void**)&p->fs_rx, fs_rx.size() * sizeof(cpx), "fs_rx"},
      {(void**)&p->fs_ry, fs_ry.size() * sizeof(cpx), "fs_ry"},
      {(void**)&p->fs_tw4n, fs_tw4n.size() * sizeof(cpx), "fs_tw4n"},
      {(void**)&p->fs_twp, fs_twp.size() * sizeof(cpx), "fs_twp"},
      {(void**)&p->fs_twi, fs_twi.size() * sizeof(cpx), "fs_twi"},
      {(void**)&p->fs_py, fs_py.size() * sizeof(cpx), "fs_py"},
      {(void**)&p->fs_Z, p->fs_on ? (size_t)bm * K * N * P * sizeof(cpx) : 0, "field-stop row transforms"},
      {(void**)&p->fs_W, p->fs_on ? (size_t)bm * K * 2 * P * N * sizeof(cpx) : 0, "field-stop column transforms"},
      {(void**)&p->field, (size_t)bm * P * P * sizeof(cpx), "pupil field"},
      {(void**)&p->zero_opd, (size_t)P * P * sizeof(float), "zero opd"},
      {(void**)&p->tmp_slopes, (size_t)2 * p->nv * sizeof(float), "reference scratch"},
  };
  for (auto& a : allocs) {
    st = dev_alloc(a.ptr, a.bytes, a.what);
    if (st != PWFS_OK) {
      free_plan(p);
      return st;
    }
    p->ws_bytes += a.bytes;
  }
  struct C { void* dst; const void* src; size_t bytes; } copies[] = {
      {p->amp, amp.data(), amp.size() * sizeof(float)},
      {p->in_a, in_a.data(), in_a.size() * sizeof(cpx)},
      {p->f_a, f_a.data(), f_a.size() * sizeof(cpx)},
      {p->in_b, in_b.data(), in_b.size() * sizeof(cpx)},
      {p->f_b, f_b.data(), f_b.size() * sizeof(cpx)},
      {p->mid, mid.data(), mid.size() * sizeof(cpx)},
      {p->tw16, tw16.data(), tw16.size() * sizeof(cpx)},
      {p->mid16, mid16.data(), mid16.size() * sizeof(cpx)},
      {p->outw, outw.data(), outw.size() * sizeof(cpx)},
      {p->k_order, k_order.data(), (size_t)K * sizeof(int)},
      {p->k_ia, k_ia.data(), (size_t)K * sizeof(int)},
      {p->d_valid, p->valid.data(), (size_t)p->nv * sizeof(int)},
      {p->fs_rx, fs_rx.data(), fs_rx.size() * sizeof(cpx)},
      {p->fs_ry, fs_ry.data(), fs_ry.size() * sizeof(cpx)},
      {p->fs_tw4n, fs_tw4n.data(), fs_tw4n.size() * sizeof(cpx)},
      {p->fs_twp, fs_twp.data(), fs_twp.size() * sizeof(cpx)},
      {p->fs_twi, fs_twi.data(), fs_twi.size() * sizeof(cpx)},
      {p->fs_py, fs_py.data(), fs_py.size() * sizeof(cpx)},
  };
  for (auto& c : copies) {
    if (c.bytes == 0) continue;
    if ((e = hipMemcpy(c.dst, c.src, c.bytes, hipMemcpyHostToDevice)) != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "table upload");
    }
  }
  if ((e = hipMemset(p->zero_opd, 0, (size_t)P * P * sizeof(float))) != hipSuccess ||
      (e = hipMemset(p->sref, 0, (size_t)2 * p->nv * sizeof(float))) != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "workspace clear");
  }
  // Reference slopes: a flat wavefront measured with a zero reference.
  st = run_measure(p, p->zero_opd, 1, nullptr, p->tmp_slopes, p->sref, nullptr);
  if (st != PWFS_OK) {
    free_plan(p);
    return st;
  }
  if ((e = hipMemcpy(p->sref, p->tmp_slopes, (size_t)2 * p->nv * sizeof(float), hipMemcpyDeviceToDevice)) !=
          hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "reference slopes");
  }
  // Sum of the flat-wavefront images (the detector's photon budget refers to it).
  {
    std::vector<float> flat((size_t)4 * S * S);
    if ((e = hipMemcpy(flat.data(), p->pupils, flat.size() * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "reference images");
    }
    double tot = 0.0;
    for (float v : flat) tot += (double)v;
    p->ref_total = tot;
  }
  *out = p;
  return PWFS_OK;
}

int pwfs_get_pupil(pwfs_plan_t p, float* amp_host) {
  if (!p || !amp_host) return fail(PWFS_ERR_INVALID_ARG, "plan or amp_host is NULL");
  std::memcpy(amp_host, p->amp_host.data(), p->amp_host.size() * sizeof(float));
  return PWFS_OK;
}

int pwfs_timing_enable(pwfs_plan_t p, int enable) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  DeviceGuard g(p->device);
  for (auto& a : p->ev_used) p->ev_free.push_back(a);
  p->ev_used.clear();
  p->timing = enable != 0;
  return PWFS_OK;
}

int pwfs_timing_read(pwfs_plan_t p, double* ms_row, double* ms_col, double* ms_slopes, int64_t* n_slices) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  DeviceGuard g(p->device);
  double acc[3] = {0.0, 0.0, 0.0};
  for (auto& a : p->ev_used) {
    hipError_t e = hipEventSynchronize(a[5]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    for (int i = 0; i < 3; ++i) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, a[2 * i], a[2 * i + 1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      acc[i] += ms;
    }
  }
  if (ms_row) *ms_row = acc[0];
  if (ms_col) *ms_col = acc[1];
  if (ms_slopes) *ms_slopes = acc[2];
  if (n_slices) *n_slices = (int64_t)p->ev_used.size();
  return PWFS_OK;
}

int pwfs_set_detector(pwfs_plan_t p, const pwfs_detector_t* d) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (!d || d->electrons_per_frame == 0.0) {
    p->det_on = false;
    return PWFS_OK;
  }
  if (!(d->electrons_per_frame > 0.0) || !std::isfinite(d->electrons_per_frame) || !(d->readout_noise_e >= 0.0) ||
      !std::isfinite(d->readout_noise_e))
    return fail(PWFS_ERR_INVALID_ARG, "electrons_per_frame must be > 0 and readout_noise_e >= 0, both finite");
  if (!(p->ref_total > 0.0)) return fail(PWFS_ERR_INVALID_ARG, "flat-wavefront images carry no light");
  p->det_on = true;
  p->det_electrons = d->electrons_per_frame;
  p->det_ron = d->readout_noise_e;
  p->det_seed = d->seed;
  p->det_gain = (float)(d->electrons_per_frame / p->ref_total);
  p->frame_next = 0;
  return PWFS_OK;
}

int pwfs_get_detector(pwfs_plan_t p, float* gain, uint64_t* next_frame) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (gain) *gain = p->det_on ? p->det_gain : 0.f;
  if (next_frame) *next_frame = p->frame_next;
  return PWFS_OK;
}

int pwfs_set_frame_counter(pwfs_plan_t p, uint64_t frame) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  p->frame_next = frame;
  return PWFS_OK;
}

int pwfs_detect(pwfs_plan_t p, const float* d_intensity, int32_t B, uint64_t frame0, float* d_pixels, void* stream) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (!p->det_on) return fail(PWFS_ERR_INVALID_ARG, "no detector set on this plan");
  if (B < 0 || B > 65535) return fail(PWFS_ERR_INVALID_ARG, "B outside [0, 65535]");
  if (B == 0) return PWFS_OK;
  if (!d_intensity || !d_pixels) return fail(PWFS_ERR_INVALID_ARG, "NULL image pointer");
  DeviceGuard g(p->device);
  hipError_t e = pwfs::launch_detector(d_intensity, d_pixels, 4 * p->S * p->S, B, frame0, p->det_gain,
                                       (float)p->det_ron, p->det_seed, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pwfs_detect launch");
  return PWFS_OK;
}

static void free_sh(pwfs_sh_s* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  for (void* q : {(void*)c->amp, (void*)c->d_valid, (void*)c->twm, (void*)c->sref, (void*)c->field,
                  (void*)c->zero_opd, (void*)c->tmp})
    if (q) (void)hipFree(q);
  delete c;
}

static hipError_t run_sh(pwfs_sh_s* c, const float* opd, int B, float* spots, float* slopes, const float* sref,
                         hipStream_t st) {
  for (int b0 = 0; b0 < B; b0 += c->batch_max) {
    const int Bs = std::min(c->batch_max, B - b0);
    pwfs::ShArgs a{};
    a.P = c->P;
    a.S = c->S;
    a.s = c->s;
    a.M = c->M;
    a.nv = c->nv;
    a.B = Bs;
    a.kphase = c->kphase;
    a.opd = opd + (size_t)b0 * c->P * c->P;
    a.amp = c->amp;
    a.valid = c->d_valid;
    a.twm = c->twm;
    a.sref = sref;
    a.field = c->field;
    a.spots = spots ? spots + (size_t)b0 * c->nv * c->M * c->M : nullptr;
    a.slopes = slopes ? slopes + (size_t)b0 * 2 * c->nv : nullptr;
    hipError_t e = pwfs::launch_sh(a, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int pwfs_sh_create(const pwfs_sh_config_t* cfg, const float* pupil_amp_host, pwfs_sh_t* out) {
  g_last_error.clear();
  if (!out) return fail(PWFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(PWFS_ERR_INVALID_ARG, "cfg is NULL");
  const int P = cfg->n_pupil, S = cfg->n_sub, pad = cfg->pad;
  if (P <= 0 || S <= 0 || pad <= 0 || cfg->batch_max <= 0) return fail(PWFS_ERR_INVALID_ARG, "sizes must be positive");
  if (P % S != 0) return fail(PWFS_ERR_INVALID_ARG, "n_pupil must be a multiple of n_sub");
  if (!(cfg->wavelength_m > 0.0) || !std::isfinite(cfg->wavelength_m) || !(cfg->obstruction >= 0.0) ||
      !(cfg->obstruction < 1.0))
    return fail(PWFS_ERR_INVALID_ARG, "wavelength or obstruction out of range");
  const int sp = P / S;
  if (sp > 8 || !(pad == 2 || pad == 4) || pad * sp > 32 || P > 1024 || cfg->batch_max > 65535)
    return fail(PWFS_ERR_UNSUPPORTED, "Shack-Hartmann: subapertures of at most 8 pixels, pad 2 or 4, pad * s <= 32");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(PWFS_ERR_NO_DEVICE, "no HIP device visible");
  }
  auto* c = new pwfs_sh_s();
  if ((e = hipGetDevice(&c->device)) != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDevice");
  }
  c->P = P;
  c->S = S;
  c->s = sp;
  c->M = pad * sp;
  c->batch_max = cfg->batch_max;
  c->kphase = 2.0 * M_PI * 1e-9 / cfg->wavelength_m;
  std::vector<float> amp((size_t)P * P);
  if (pupil_amp_host) {
    for (size_t i = 0; i < amp.size(); ++i) {
      if (!std::isfinite(pupil_amp_host[i])) {
        delete c;
        return fail(PWFS_ERR_INVALID_ARG, "pupil amplitude has non-finite values");
      }
      amp[i] = pupil_amp_host[i];
    }
  } else {
    circle_pupil(P, cfg->obstruction, amp);
  }
  for (int iy = 0; iy < S; ++iy)
    for (int ix = 0; ix < S; ++ix) {
      double f = 0.0;
      for (int dy = 0; dy < sp; ++dy)
        for (int dx = 0; dx < sp; ++dx) f += amp[(size_t)(iy * sp + dy) * P + ix * sp + dx];
      if (f >= 0.5 * sp * sp) c->valid.push_back(iy * S + ix);
    }
  c->nv = (int)c->valid.size();
  if (c->nv == 0) {
    delete c;
    return fail(PWFS_ERR_INVALID_ARG, "no valid subaperture");
  }
  std::vector<cpx> twm((size_t)c->M);
  for (int k = 0; k < c->M; ++k) {
    const double ang = -2.0 * M_PI * (double)k / (double)c->M;
    twm[k] = cpx{(float)std::cos(ang), (float)std::sin(ang)};
  }
  const size_t bm = (size_t)c->batch_max;
  struct A { void** ptr; size_t bytes; const char* what; } allocs[] = {
      {(void**)&c->amp, amp.size() * sizeof(float), "sh amp"},
      {(void**)&c->d_valid, (size_t)c->nv * sizeof(int), "sh valid"},
      {(void**)&c->twm, twm.size() * sizeof(cpx), "sh twiddles"},
      {(void**)&c->sref, (size_t)2 * c->nv * sizeof(float), "sh reference"},
      {(void**)&c->field, bm * P * P * sizeof(cpx), "sh field"},
      {(void**)&c->zero_opd, (size_t)P * P * sizeof(float), "sh zero opd"},
      {(void**)&c->tmp, (size_t)2 * c->nv * sizeof(float), "sh reference scratch"},
  };
  for (auto& a : allocs) {
    int st = dev_alloc(a.ptr, a.bytes, a.what);
    if (st != PWFS_OK) {
      free_sh(c);
      return st;
    }
  }
  if ((e = hipMemcpy(c->amp, amp.data(), amp.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_valid, c->valid.data(), (size_t)c->nv * sizeof(int), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(c->twm, twm.data(), twm.size() * sizeof(cpx), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(c->zero_opd, 0, (size_t)P * P * sizeof(float))) != hipSuccess ||
      (e = hipMemset(c->sref, 0, (size_t)2 * c->nv * sizeof(float))) != hipSuccess ||
      (e = run_sh(c, c->zero_opd, 1, nullptr, c->tmp, c->sref, nullptr)) != hipSuccess ||
      (e = hipMemcpy(c->sref, c->tmp, (size_t)2 * c->nv * sizeof(float), hipMemcpyDeviceToDevice)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    free_sh(c);
    return hip_fail(e, "Shack-Hartmann set-up");
  }
  *out = c;
  return PWFS_OK;
}

int pwfs_sh_info(pwfs_sh_t c, int32_t* n_valid, int32_t* spot_side) {
  if (!c) return fail(PWFS_ERR_INVALID_ARG, "sensor is NULL");
  if (n_valid) *n_valid = c->nv;
  if (spot_side) *spot_side = c->M;
  return PWFS_OK;
}

int pwfs_sh_get_valid(pwfs_sh_t c, int32_t* idx_host) {
  if (!c || !idx_host) return fail(PWFS_ERR_INVALID_ARG, "sensor or idx_host is NULL");
  std::memcpy(idx_host, c->valid.data(), c->valid.size() * sizeof(int32_t));
  return PWFS_OK;
}

int pwfs_sh_get_reference(pwfs_sh_t c, float* sref_host) {
  if (!c || !sref_host) return fail(PWFS_ERR_INVALID_ARG, "sensor or sref_host is NULL");
  DeviceGuard g(c->device);
  hipError_t e = hipMemcpy(sref_host, c->sref, (size_t)2 * c->nv * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "pwfs_sh_get_reference");
  return PWFS_OK;
}

int pwfs_sh_measure(pwfs_sh_t c, const float* d_opd_nm, int32_t B, float* d_spots, float* d_slopes, void* stream) {
  if (!c) return fail(PWFS_ERR_INVALID_ARG, "sensor is NULL");
  if (B < 0) return fail(PWFS_ERR_INVALID_ARG, "B must be >= 0");
  if (B == 0 || (!d_spots && !d_slopes)) return PWFS_OK;
  if (!d_opd_nm) return fail(PWFS_ERR_INVALID_ARG, "d_opd_nm is NULL");
  DeviceGuard g(c->device);
  hipError_t e = run_sh(c, d_opd_nm, B, d_spots, d_slopes, c->sref, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pwfs_sh_measure launch");
  return PWFS_OK;
}

void pwfs_sh_destroy(pwfs_sh_t c) {
  if (!c) return;
  {
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
  }
  free_sh(c);
}

static void free_psf(pwfs_psf_s* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  for (void* q : {(void*)c->amp, (void*)c->twpad, (void*)c->twp, (void*)c->field, (void*)c->Z})
    if (q) (void)hipFree(q);
  delete c;
}

int pwfs_psf_create(const pwfs_psf_config_t* cfg, const float* pupil_amp_host, pwfs_psf_t* out) {
  g_last_error.clear();
  if (!out) return fail(PWFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(PWFS_ERR_INVALID_ARG, "cfg is NULL");
  const int P = cfg->n_pupil, pad = cfg->pad;
  if (P <= 0 || pad <= 0 || cfg->batch_max <= 0 || cfg->reserved != 0)
    return fail(PWFS_ERR_INVALID_ARG, "sizes must be positive and reserved 0");
  if (!(cfg->wavelength_m > 0.0) || !std::isfinite(cfg->wavelength_m) || !(cfg->obstruction >= 0.0) ||
      !(cfg->obstruction < 1.0))
    return fail(PWFS_ERR_INVALID_ARG, "wavelength or obstruction out of range");
  if (!(P == 32 || P == 64 || P == 160)) return fail(PWFS_ERR_UNSUPPORTED, "PSF camera: n_pupil must be 32, 64 or 160");
  if (!(pad == 2 || pad == 4 || pad == 8)) return fail(PWFS_ERR_UNSUPPORTED, "PSF camera: pad must be 2, 4 or 8");
  if (cfg->batch_max > 65535) return fail(PWFS_ERR_UNSUPPORTED, "batch_max > 65535");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(PWFS_ERR_NO_DEVICE, "no HIP device visible");
  }
  auto* c = new pwfs_psf_s();
  if ((e = hipGetDevice(&c->device)) != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDevice");
  }
  c->P = P;
  c->pad = pad;
  c->N = pad * P;
  c->batch_max = cfg->batch_max;
  c->kphase = 2.0 * M_PI * 1e-9 / cfg->wavelength_m;
  std::vector<float> amp((size_t)P * P);
  if (pupil_amp_host) {
    for (size_t i = 0; i < amp.size(); ++i) {
      if (!std::isfinite(pupil_amp_host[i])) {
        delete c;
        return fail(PWFS_ERR_INVALID_ARG, "pupil amplitude has non-finite values");
      }
      amp[i] = pupil_amp_host[i];
    }
  } else {
    circle_pupil(P, cfg->obstruction, amp);
  }
  double sa = 0.0;
  for (float v : amp) sa += (double)v;
  if (!(sa > 0.0)) {
    delete c;
    return fail(PWFS_ERR_INVALID_ARG, "pupil amplitude sums to zero");
  }
  c->inv_norm = 1.0 / (sa * sa);
  const int E = P / 4, N = c->N;
  std::vector<cpx> twpad((size_t)pad * P), twp((size_t)4 * E);
  for (int u1 = 0; u1 < pad; ++u1)
    for (int x = 0; x < P; ++x) {
      const double ang = -2.0 * M_PI * (double)(((long)u1 * x) % N) / (double)N;
      twpad[(size_t)u1 * P + x] = cpx{(float)std::cos(ang), (float)std::sin(ang)};
    }
  for (int l = 0; l < 4; ++l)
    for (int k = 0; k < E; ++k) {
      const double ang = -2.0 * M_PI * (double)(((long)l * k) % P) / (double)P;
      twp[(size_t)l * E + k] = cpx{(float)std::cos(ang), (float)std::sin(ang)};
    }
  const size_t bm = (size_t)cfg->batch_max;
  struct A { void** ptr; size_t bytes; const char* what; } allocs[] = {
      {(void**)&c->amp, amp.size() * sizeof(float), "psf amp"},
      {(void**)&c->twpad, twpad.size() * sizeof(cpx), "psf padding twiddles"},
      {(void**)&c->twp, twp.size() * sizeof(cpx), "psf twiddles"},
      {(void**)&c->field, bm * P * P * sizeof(cpx), "psf field"},
      {(void**)&c->Z, bm * (size_t)N * P * sizeof(cpx), "psf row transforms"},
  };
  for (auto& a : allocs) {
    int st = dev_alloc(a.ptr, a.bytes, a.what);
    if (st != PWFS_OK) {
      free_psf(c);
      return st;
    }
  }
  if ((e = hipMemcpy(c->amp, amp.data(), amp.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->twpad, twpad.data(), twpad.size() * sizeof(cpx), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->twp, twp.data(), twp.size() * sizeof(cpx), hipMemcpyHostToDevice)) != hipSuccess) {
    free_psf(c);
    return hip_fail(e, "psf table upload");
  }
  *out = c;
  return PWFS_OK;
}

int pwfs_psf_info(pwfs_psf_t c, int32_t* n_image) {
  if (!c) return fail(PWFS_ERR_INVALID_ARG, "camera is NULL");
  if (n_image) *n_image = c->N;
  return PWFS_OK;
}

int pwfs_psf_compute(pwfs_psf_t c, const float* d_opd_nm, int32_t B, int32_t accumulate, float* d_psf,
                     float* d_strehl, void* stream) {
  if (!c) return fail(PWFS_ERR_INVALID_ARG, "camera is NULL");
  if (B < 0) return fail(PWFS_ERR_INVALID_ARG, "B must be >= 0");
  if (B == 0 || (!d_psf && !d_strehl)) return PWFS_OK;
  if (!d_opd_nm) return fail(PWFS_ERR_INVALID_ARG, "d_opd_nm is NULL");
  DeviceGuard g(c->device);
  const size_t NN = (size_t)c->N * c->N;
  for (int b0 = 0; b0 < B; b0 += c->batch_max) {
    const int Bs = std::min(c->batch_max, B - b0);
    pwfs::PsfArgs a{};
    a.P = c->P;
    a.pad = c->pad;
    a.B = Bs;
    a.accumulate = accumulate ? 1 : 0;
    a.kphase = c->kphase;
    a.inv_norm = (float)c->inv_norm;
    a.inv_norm_d = c->inv_norm;
    a.opd = d_opd_nm + (size_t)b0 * c->P * c->P;
    a.amp = c->amp;
    a.twpad = c->twpad;
    a.twp = c->twp;
    a.field = c->field;
    a.Z = c->Z;
    a.psf = d_psf ? (accumulate ? d_psf : d_psf + (size_t)b0 * NN) : nullptr;
    a.strehl = d_strehl ? d_strehl + b0 : nullptr;
    hipError_t e = pwfs::launch_psf(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "pwfs_psf_compute launch");
  }
  return PWFS_OK;
}

void pwfs_psf_destroy(pwfs_psf_t c) {
  if (!c) return;
  {
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
  }
  free_psf(c);
}

int pwfs_get_schedule(pwfs_plan_t p, int32_t B, int32_t* a_chunk, int32_t* k_chunk) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (B < 1 || B > p->batch_max) return fail(PWFS_ERR_INVALID_ARG, "B outside [1, batch_max]");
  int a, k, nc;
  split_work(p, B, &a, &k, &nc);
  if (a_chunk) *a_chunk = a;
  if (k_chunk) *k_chunk = k;
  return PWFS_OK;
}

int pwfs_set_schedule(pwfs_plan_t p, int32_t B, int32_t a_chunk, int32_t k_chunk) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (p->fs_on) return fail(PWFS_ERR_UNSUPPORTED, "field-stop plans have a fixed work split");
  if (B < 1 || B > p->batch_max) return fail(PWFS_ERR_INVALID_ARG, "B outside [1, batch_max]");
  if (a_chunk == 0 && k_chunk == 0) {
    p->sched.erase(B);
    return PWFS_OK;
  }
  if (!schedule_fits(p, B, a_chunk, k_chunk))
    return fail(PWFS_ERR_INVALID_ARG, "schedule out of range or its partials exceed the plan workspace");
  p->sched[B] = {a_chunk, k_chunk};
  return PWFS_OK;
}

int pwfs_get_schedule_lanes(pwfs_plan_t p, int32_t B, int32_t* lanes) {
  if (!p || !lanes) return fail(PWFS_ERR_INVALID_ARG, "plan or lanes is NULL");
  if (B < 1 || B > p->batch_max) return fail(PWFS_ERR_INVALID_ARG, "B outside [1, batch_max]");
  *lanes = teams32(p, B) ? 32 : 8;
  return PWFS_OK;
}

int pwfs_set_schedule_lanes(pwfs_plan_t p, int32_t B, int32_t lanes) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (p->fs_on) return fail(PWFS_ERR_UNSUPPORTED, "field-stop plans have a fixed work split");
  if (B < 1 || B > p->batch_max) return fail(PWFS_ERR_INVALID_ARG, "B outside [1, batch_max]");
  if (lanes != 8 && lanes != 32) return fail(PWFS_ERR_INVALID_ARG, "lanes must be 8 or 32");
  if (long_lines(p->P)) {
    if (lanes != 32) return fail(PWFS_ERR_UNSUPPORTED, "n_pupil 128 and 480 run 32-lane teams only");
    return PWFS_OK;
  }
  if (p->P != 160) {
    if (lanes != 8) return fail(PWFS_ERR_UNSUPPORTED, "32-lane teams need n_pupil 128, 160 or 480");
    return PWFS_OK;
  }
  p->teams32[B] = lanes == 32 ? 1 : 0;
  return PWFS_OK;
}

int pwfs_autotune(pwfs_plan_t p, int32_t B, int32_t reps, void* stream, double* ms_default, double* ms_tuned) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (p->fs_on) return fail(PWFS_ERR_UNSUPPORTED, "field-stop plans have a fixed work split");
  if (B < 1 || B > p->batch_max) return fail(PWFS_ERR_INVALID_ARG, "B outside [1, batch_max]");
  if (reps < 1 || reps > 1000) return fail(PWFS_ERR_INVALID_ARG, "reps outside [1, 1000]");
  DeviceGuard g(p->device);
  hipStream_t st = (hipStream_t)stream;
  float* d_opd = nullptr;
  float* d_sl = nullptr;
  std::array<hipEvent_t, 6> ev{};
  int status = PWFS_OK;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (hipEvent_t x : ev)
      if (x) (void)hipEventDestroy(x);
    if (d_opd) (void)hipFree(d_opd);
    if (d_sl) (void)hipFree(d_sl);
  };
  int st_alloc = dev_alloc((void**)&d_opd, (size_t)B * p->P * p->P * sizeof(float), "autotune input");
  if (st_alloc == PWFS_OK) st_alloc = dev_alloc((void**)&d_sl, (size_t)B * 2 * p->nv * sizeof(float), "autotune slopes");
  if (st_alloc != PWFS_OK) {
    cleanup();
    return st_alloc;
  }
  hipError_t e = hipMemsetAsync(d_opd, 0, (size_t)B * p->P * p->P * sizeof(float), st);
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "autotune setup");
  }
  // Best of `reps` timed launches (after one untimed launch) of a schedule:
  // row pass (with the field) and column pass + chunk reduction + slopes.
  auto time_schedule = [&](int a_chunk, int k_chunk, double* row_ms, double* col_ms) -> hipError_t {
    pwfs::MeasureArgs a = slice_args(p, d_opd, 0, B, nullptr, d_sl, p->sref, plan_workspace(p));
    a.a_chunk = a_chunk;
    a.k_chunk = k_chunk;
    a.n_chunks = (p->K + k_chunk - 1) / k_chunk;
    hipError_t le = pwfs::launch_measure(a, st, nullptr);
    *row_ms = *col_ms = 1e30;
    for (int r = 0; r < reps && le == hipSuccess; ++r) {
      le = pwfs::launch_measure(a, st, ev.data());
      if (le == hipSuccess) le = hipEventSynchronize(ev[5]);
      float t0 = 0.f, t1 = 0.f;
      if (le == hipSuccess) le = hipEventElapsedTime(&t0, ev[0], ev[1]);
      if (le == hipSuccess) le = hipEventElapsedTime(&t1, ev[2], ev[5]);
      *row_ms = std::min(*row_ms, (double)t0);
      *col_ms = std::min(*col_ms, (double)t1);
    }
    return le;
  };
  // One search per lane form (both at P = 160): the default split, then the
  // row pass over the distinct numbers of x-tilt chunks, then the column pass
  // over the distinct numbers of modulation chunks.
  const bool had_form = p->teams32.count(B) != 0;
  const int old_form = had_form ? p->teams32[B] : 0;
  auto search = [&](int form, int* ba, int* bk, double* brow, double* bcol, double* dflt) -> hipError_t {
    if (p->P == 160) p->teams32[B] = form;
    int a0, k0;
    default_split(p, B, &a0, &k0);
    double row0, col0;
    hipError_t le = time_schedule(a0, k0, &row0, &col0);
    *ba = a0;
    *bk = k0;
    *brow = row0;
    *bcol = col0;
    *dflt = row0 + col0;
    for (int a = 1; a <= p->n_a && le == hipSuccess; ++a) {
      if (a > 1 && (p->n_a + a - 1) / a == (p->n_a + a - 2) / (a - 1)) continue;
      if (a == a0 || !schedule_fits(p, B, a, k0)) continue;
      double r, c;
      le = time_schedule(a, k0, &r, &c);
      if (le == hipSuccess && r < 0.98 * *brow) {
        *brow = r;
        *ba = a;
      }
    }
    for (int k = 1; k <= p->K && le == hipSuccess; ++k) {
      if (k > 1 && (p->K + k - 1) / k == (p->K + k - 2) / (k - 1)) continue;
      if (k == k0 || !schedule_fits(p, B, *ba, k)) continue;
      double r, c;
      le = time_schedule(*ba, k, &r, &c);
      if (le == hipSuccess && c < 0.98 * *bcol) {
        *bcol = c;
        *bk = k;
      }
    }
    return le;
  };
  int best_a = 0, best_k = 0, best_form = 0;
  double best_row = 0.0, best_col = 0.0, dflt8 = 0.0;
  e = search(0, &best_a, &best_k, &best_row, &best_col, &dflt8);
  if (e == hipSuccess && p->P == 160) {
    int a2, k2;
    double r2, c2, d2;
    e = search(1, &a2, &k2, &r2, &c2, &d2);
    if (e == hipSuccess && r2 + c2 < 0.98 * (best_row + best_col)) {
      best_a = a2;
      best_k = k2;
      best_row = r2;
      best_col = c2;
      best_form = 1;
    }
  }
  if (e != hipSuccess) status = hip_fail(e, "autotune launch");
  cleanup();
  if (status != PWFS_OK) {
    if (p->P == 160) {
      if (had_form)
        p->teams32[B] = old_form;
      else
        p->teams32.erase(B);
    }
    return status;
  }
  p->sched[B] = {best_a, best_k};
  if (p->P == 160) p->teams32[B] = best_form;
  if (ms_default) *ms_default = dflt8;   // 8-lane teams (32-lane at P = 128, 480), default split
  if (ms_tuned) *ms_tuned = best_row + best_col;
  return PWFS_OK;
}

int pwfs_plan_info(pwfs_plan_t p, int32_t* n_valid, int32_t* n_sub, size_t* workspace_bytes) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (n_valid) *n_valid = p->nv;
  if (n_sub) *n_sub = p->S;
  if (workspace_bytes) *workspace_bytes = p->ws_bytes;
  return PWFS_OK;
}

int pwfs_get_valid(pwfs_plan_t p, int32_t* idx_host) {
  if (!p || !idx_host) return fail(PWFS_ERR_INVALID_ARG, "plan or idx_host is NULL");
  std::memcpy(idx_host, p->valid.data(), p->valid.size() * sizeof(int32_t));
  return PWFS_OK;
}

int pwfs_set_valid(pwfs_plan_t p, const int32_t* idx_host, int32_t n) {
  if (!p || !idx_host) return fail(PWFS_ERR_INVALID_ARG, "plan or idx_host is NULL");
  if (n < 1) return fail(PWFS_ERR_INVALID_ARG, "the valid list must not be empty");
  const int S = p->S;
  for (int32_t i = 0; i < n; ++i) {
    if (idx_host[i] < 0 || idx_host[i] >= S * S) return fail(PWFS_ERR_INVALID_ARG, "valid index out of range");
    if (i > 0 && idx_host[i] <= idx_host[i - 1])
      return fail(PWFS_ERR_INVALID_ARG, "valid indices must be strictly ascending");
  }
  DeviceGuard g(p->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "pwfs_set_valid");
  int* dv = nullptr;
  float *sr = nullptr, *ts = nullptr;
  int st = dev_alloc((void**)&dv, (size_t)n * sizeof(int), "valid");
  if (st == PWFS_OK) st = dev_alloc((void**)&sr, (size_t)2 * n * sizeof(float), "sref");
  if (st == PWFS_OK) st = dev_alloc((void**)&ts, (size_t)2 * n * sizeof(float), "reference scratch");
  if (st == PWFS_OK) {
    if ((e = hipMemcpy(dv, idx_host, (size_t)n * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(sr, 0, (size_t)2 * n * sizeof(float))) != hipSuccess)
      st = hip_fail(e, "pwfs_set_valid upload");
  }
  if (st != PWFS_OK) {
    for (void* q : {(void*)dv, (void*)sr, (void*)ts})
      if (q) (void)hipFree(q);
    return st;
  }
  for (void* q : {(void*)p->d_valid, (void*)p->sref, (void*)p->tmp_slopes})
    if (q) (void)hipFree(q);
  p->ws_bytes -= (size_t)p->nv * sizeof(int) + (size_t)4 * p->nv * sizeof(float);
  p->d_valid = dv;
  p->sref = sr;
  p->tmp_slopes = ts;
  p->valid.assign(idx_host, idx_host + n);
  p->nv = n;
  p->ws_bytes += (size_t)n * sizeof(int) + (size_t)4 * n * sizeof(float);
  // Noiseless flat-wavefront reference with the new list (detector bypassed,
  // frame counter untouched).
  const bool det = p->det_on;
  p->det_on = false;
  st = run_measure(p, p->zero_opd, 1, nullptr, p->tmp_slopes, p->sref, nullptr);
  p->det_on = det;
  if (st != PWFS_OK) return st;
  if ((e = hipMemcpy(p->sref, p->tmp_slopes, (size_t)2 * n * sizeof(float), hipMemcpyDeviceToDevice)) !=
          hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return hip_fail(e, "pwfs_set_valid reference");
  return PWFS_OK;
}

int pwfs_get_reference(pwfs_plan_t p, float* sref_host) {
  if (!p || !sref_host) return fail(PWFS_ERR_INVALID_ARG, "plan or sref_host is NULL");
  DeviceGuard g(p->device);
  hipError_t e = hipMemcpy(sref_host, p->sref, (size_t)2 * p->nv * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "pwfs_get_reference");
  return PWFS_OK;
}

int pwfs_set_reference(pwfs_plan_t p, const float* d_sref, void* stream) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  DeviceGuard g(p->device);
  const size_t bytes = (size_t)2 * p->nv * sizeof(float);
  hipError_t e = d_sref ? hipMemcpyAsync(p->sref, d_sref, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream)
                        : pwfs::launch_fill(p->sref, (size_t)2 * p->nv, 0.0f, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pwfs_set_reference");
  return PWFS_OK;
}

int pwfs_measure(pwfs_plan_t p, const float* d_opd_nm, int32_t B, float* d_pupils, float* d_slopes,
                 void* stream) {
  if (!p) return fail(PWFS_ERR_INVALID_ARG, "plan is NULL");
  if (B < 0) return fail(PWFS_ERR_INVALID_ARG, "B must be >= 0");
  if (B == 0 || (!d_pupils && !d_slopes)) return PWFS_OK;
  if (!d_opd_nm) return fail(PWFS_ERR_INVALID_ARG, "d_opd_nm is NULL");
  DeviceGuard g(p->device);
  return run_measure(p, d_opd_nm, B, d_pupils, d_slopes, p->sref, (hipStream_t)stream);
}

int recon_apply(const float* d_R, int32_t M, int32_t n_s, const float* d_s, int32_t B, float alpha,
                float beta, float* d_m, void* stream) {
  if (M <= 0 || n_s <= 0 || B < 0) return fail(PWFS_ERR_INVALID_ARG, "M, n_s must be > 0 and B >= 0");
  if (B == 0) return PWFS_OK;
  if (!d_R || !d_s || !d_m) return fail(PWFS_ERR_INVALID_ARG, "NULL matrix or vector");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(PWFS_ERR_INVALID_ARG, "alpha/beta not finite");
  if (B > 65535 * 8 || M > 65535 * 4) return fail(PWFS_ERR_UNSUPPORTED, "B or M too large");
  hipError_t e = pwfs::launch_recon(d_R, M, n_s, d_s, B, alpha, beta, d_m, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "recon_apply launch");
  return PWFS_OK;
}

void pwfs_destroy(pwfs_plan_t p) {
  if (!p) return;
  {
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
  }
  free_plan(p);
}

}  // extern "C"
