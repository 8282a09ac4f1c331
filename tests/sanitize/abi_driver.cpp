// abi_driver.cpp -- every entry point of the C ABI on its host-side paths:
// NULL handles and pointers, out-of-range configurations and sizes, empty
// batches, status strings, and (with no device visible) the no-device
// status of the create calls.  Built with the host sanitizers
// (AddressSanitizer, UndefinedBehaviorSanitizer) by
// tests/test_abi_sanitize.py; prints one line per check and "done" at the
// end, exits non-zero on the first unexpected status.
#include "pwfs.h"
#include "pwfs_cnn.h"

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

int g_checks = 0;

void expect(const char* what, int got, int want) {
  ++g_checks;
  if (got != want) {
    std::printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want, pwfs_last_error());
    std::exit(1);
  }
}

pwfs_config_t good_config() {
  pwfs_config_t c{};
  c.n_fft = 128;
  c.n_pupil = 32;
  c.n_bin = 2;
  c.n_mod = 16;
  c.batch_max = 2;
  c.diameter_m = 8.0;
  c.wavelength_m = 750e-9;
  c.mod_radius_lod = 3.0;
  return c;
}

}  // namespace

int main(int argc, char** argv) {
  const bool no_device = argc > 1 && std::strcmp(argv[1], "no-device") == 0;
  const int INVALID = PWFS_ERR_INVALID_ARG, UNSUP = PWFS_ERR_UNSUPPORTED;

  // status strings
  for (int s = 0; s >= -6; --s) {
    const char* t = pwfs_strerror(s);
    if (!t || !*t) expect("pwfs_strerror", 1, 0);
  }
  (void)pwfs_strerror(12345);
  (void)pwfs_last_error();

  // plan configuration checks (all before any device call)
  pwfs_plan_t plan = nullptr;
  expect("plan NULL cfg", pwfs_plan(nullptr, nullptr, &plan), INVALID);
  pwfs_config_t c = good_config();
  expect("plan NULL out", pwfs_plan(&c, nullptr, nullptr), INVALID);
  struct Bad { const char* what; void (*edit)(pwfs_config_t&); int status; } bad[] = {
      {"n_pupil 0", [](pwfs_config_t& x) { x.n_pupil = 0; }, INVALID},
      {"n_bin 3", [](pwfs_config_t& x) { x.n_bin = 3; }, INVALID},
      {"batch_max 0", [](pwfs_config_t& x) { x.batch_max = 0; }, INVALID},
      {"wavelength 0", [](pwfs_config_t& x) { x.wavelength_m = 0.0; }, INVALID},
      {"obstruction 1", [](pwfs_config_t& x) { x.obstruction = 1.0; }, INVALID},
      {"norm_mode 2", [](pwfs_config_t& x) { x.norm_mode = 2; }, INVALID},
      {"flags 4", [](pwfs_config_t& x) { x.flags = 4; }, INVALID},
      {"n_fft 100", [](pwfs_config_t& x) { x.n_fft = 100; }, UNSUP},
      {"n_mod 2000", [](pwfs_config_t& x) { x.n_mod = 2000; }, UNSUP},
      {"n_pupil 96", [](pwfs_config_t& x) { x.n_pupil = 96; x.n_fft = 384; }, UNSUP},
      {"det_window 1", [](pwfs_config_t& x) { x.n_bin = 1; x.det_window = 1; }, INVALID},
      {"field stop NaN", [](pwfs_config_t& x) { x.field_stop_lod = 0.0 / 0.0; }, INVALID},
      {"reserved", [](pwfs_config_t& x) { x.reserved = 1; }, INVALID},
  };
  for (auto& b : bad) {
    pwfs_config_t x = good_config();
    b.edit(x);
    expect(b.what, pwfs_plan(&x, nullptr, &plan), b.status);
    if (plan != nullptr) expect("handle cleared on failure", 1, 0);
  }

  // NULL plan handles everywhere
  int32_t i32 = 0, i32b = 0;
  int64_t i64 = 0;
  size_t sz = 0;
  double d0 = 0, d1 = 0, d2 = 0;
  float f = 0;
  uint64_t u64 = 0;
  expect("plan_info", pwfs_plan_info(nullptr, &i32, &i32b, &sz), INVALID);
  expect("get_valid", pwfs_get_valid(nullptr, &i32), INVALID);
  expect("set_valid", pwfs_set_valid(nullptr, &i32, 1), INVALID);
  expect("get_reference", pwfs_get_reference(nullptr, &f), INVALID);
  expect("set_reference", pwfs_set_reference(nullptr, nullptr, nullptr), INVALID);
  expect("measure", pwfs_measure(nullptr, nullptr, 1, nullptr, nullptr, nullptr), INVALID);
  expect("measure_static", pwfs_measure_static(nullptr, nullptr, 1, nullptr, nullptr, nullptr), INVALID);
  expect("get_pupil", pwfs_get_pupil(nullptr, &f), INVALID);
  expect("timing_enable", pwfs_timing_enable(nullptr, 1), INVALID);
  expect("timing_read", pwfs_timing_read(nullptr, &d0, &d1, &d2, &i64), INVALID);
  pwfs_detector_t det{};
  expect("set_detector", pwfs_set_detector(nullptr, &det), INVALID);
  expect("get_detector", pwfs_get_detector(nullptr, &f, &u64), INVALID);
  expect("set_frame_counter", pwfs_set_frame_counter(nullptr, 3), INVALID);
  expect("detect", pwfs_detect(nullptr, nullptr, 1, 0, nullptr, nullptr), INVALID);
  expect("get_schedule", pwfs_get_schedule(nullptr, 1, &i32, &i32b), INVALID);
  expect("set_schedule", pwfs_set_schedule(nullptr, 1, 1, 1), INVALID);
  expect("get_schedule_lanes", pwfs_get_schedule_lanes(nullptr, 1, &i32), INVALID);
  expect("set_schedule_lanes", pwfs_set_schedule_lanes(nullptr, 1, 8), INVALID);
  expect("autotune", pwfs_autotune(nullptr, 1, 1, nullptr, &d0, &d1), INVALID);
  pwfs_destroy(nullptr);

  // reconstructor argument checks
  expect("recon NULL", recon_apply(nullptr, 4, 4, nullptr, 1, 1.f, 0.f, nullptr, nullptr), INVALID);
  expect("recon M 0", recon_apply(nullptr, 0, 4, nullptr, 1, 1.f, 0.f, nullptr, nullptr), INVALID);
  expect("recon B < 0", recon_apply(nullptr, 4, 4, nullptr, -1, 1.f, 0.f, nullptr, nullptr), INVALID);
  expect("recon empty batch", recon_apply(nullptr, 4, 4, nullptr, 0, 1.f, 0.f, nullptr, nullptr), PWFS_OK);

  // Shack-Hartmann and PSF camera
  pwfs_sh_t sh = nullptr;
  pwfs_sh_config_t shc{};
  expect("sh NULL cfg", pwfs_sh_create(nullptr, nullptr, &sh), INVALID);
  expect("sh bad cfg", pwfs_sh_create(&shc, nullptr, &sh), INVALID);
  expect("sh_info", pwfs_sh_info(nullptr, &i32, &i32b), INVALID);
  expect("sh_get_valid", pwfs_sh_get_valid(nullptr, &i32), INVALID);
  expect("sh_get_reference", pwfs_sh_get_reference(nullptr, &f), INVALID);
  expect("sh_measure", pwfs_sh_measure(nullptr, nullptr, 1, nullptr, nullptr, nullptr), INVALID);
  pwfs_sh_destroy(nullptr);
  pwfs_psf_t cam = nullptr;
  pwfs_psf_config_t pc{};
  expect("psf NULL cfg", pwfs_psf_create(nullptr, nullptr, &cam), INVALID);
  expect("psf bad cfg", pwfs_psf_create(&pc, nullptr, &cam), INVALID);
  expect("psf_info", pwfs_psf_info(nullptr, &i32), INVALID);
  expect("psf_compute", pwfs_psf_compute(nullptr, nullptr, 1, 0, nullptr, nullptr, nullptr), INVALID);
  pwfs_psf_destroy(nullptr);

  // learned reconstructor
  pwfs_cnn_t net = nullptr;
  pwfs_cnn_config_t cc{};
  expect("cnn NULL cfg", pwfs_cnn_create(nullptr, &net), INVALID);
  expect("cnn bad cfg", pwfs_cnn_create(&cc, &net), INVALID);
  expect("cnn_num_params", pwfs_cnn_num_params(nullptr, &i64), INVALID);
  expect("cnn_set_params", pwfs_cnn_set_params(nullptr, nullptr, nullptr), INVALID);
  expect("cnn_get_params", pwfs_cnn_get_params(nullptr, nullptr, nullptr), INVALID);
  expect("cnn_get_optimizer", pwfs_cnn_get_optimizer(nullptr, nullptr, nullptr, &i64, nullptr), INVALID);
  expect("cnn_set_optimizer", pwfs_cnn_set_optimizer(nullptr, nullptr, nullptr, 0, nullptr), INVALID);
  expect("cnn_prepare bad", pwfs_cnn_prepare(nullptr, nullptr, nullptr, 0, 1, 40, nullptr, nullptr), INVALID);
  expect("cnn_prepare empty", pwfs_cnn_prepare(nullptr, nullptr, nullptr, 10, 0, 40, nullptr, nullptr), PWFS_OK);
  expect("cnn_forward", pwfs_cnn_forward(nullptr, nullptr, 1, nullptr, nullptr), INVALID);
  expect("cnn_forward_acc", pwfs_cnn_forward_acc(nullptr, nullptr, 1, 1.f, 0.f, nullptr, nullptr), INVALID);
  expect("cnn_gradients", pwfs_cnn_gradients(nullptr, nullptr, nullptr, nullptr, 1, nullptr, nullptr, nullptr),
         INVALID);
  expect("cnn_train_step",
         pwfs_cnn_train_step(nullptr, nullptr, nullptr, nullptr, 1, 1e-3f, 0.9f, 0.999f, 1e-8f, nullptr, nullptr),
         INVALID);
  pwfs_cnn_destroy(nullptr);

  // no device: the create calls fail with PWFS_ERR_NO_DEVICE, nothing leaks
  if (no_device) {
    c = good_config();
    expect("plan no device", pwfs_plan(&c, nullptr, &plan), PWFS_ERR_NO_DEVICE);
    cc.n_sub = 40; cc.c1 = 32; cc.c2 = 64; cc.c3 = 64; cc.hidden = 2048; cc.n_out = 600; cc.batch_max = 4;
    expect("cnn no device", pwfs_cnn_create(&cc, &net), PWFS_ERR_NO_DEVICE);
  }
  std::printf("done: %d checks\n", g_checks);
  return 0;
}
