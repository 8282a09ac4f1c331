// pwfs_static.hip -- pwfs_measure without any allocation: the workspace of a
// measurement (row-pass intermediate, chunk partials, pupil field, internal
// images) comes from one file-scope device array instead of the plan.
//
// The array is device memory the loader creates on each GPU the library
// runs on; host code never passes its name to a kernel or a copy.  The
// device address is looked up once per device with hipGetSymbolAddress (on
// the first call on that device, with that device current) and that address
// is what the kernels receive.
#include "../../include/pwfs.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

namespace pwfs {
int measure_in_workspace(pwfs_plan_t p, const float* d_opd_nm, int32_t B, float* d_pupils, float* d_slopes,
                         void* ws_base, size_t ws_bytes, void* stream);
int plan_device(pwfs_plan_t p);
int set_last_error(int status, const std::string& msg);
}  // namespace pwfs

namespace {

static __device__ __align__(256) unsigned char scratch[PWFS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per device, looked up once

// Device address of `scratch` on `dev` (made current by the caller), or NULL
// with the last error set.
void* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    pwfs::set_last_error(PWFS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return nullptr;
  }
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

}  // namespace

extern "C" int pwfs_measure_static(pwfs_plan_t plan, const float* d_opd_nm, int32_t B, float* d_pupils,
                                   float* d_slopes, void* stream) {
  if (!plan) return pwfs::set_last_error(PWFS_ERR_INVALID_ARG, "plan is NULL");
  const int dev = pwfs::plan_device(plan);
  if (dev < 0 || dev >= kMaxDevices) return pwfs::set_last_error(PWFS_ERR_UNSUPPORTED, "device index out of range");
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) {
    (void)hipGetLastError();
    return pwfs::set_last_error(PWFS_ERR_NO_DEVICE, "hipGetDevice failed");
  }
  if (prev != dev && hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    return pwfs::set_last_error(PWFS_ERR_HIP, "hipSetDevice failed");
  }
  void* base = scratch_on(dev);
  const int st = base ? pwfs::measure_in_workspace(plan, d_opd_nm, B, d_pupils, d_slopes, base,
                                                   PWFS_STATIC_SCRATCH_BYTES, stream)
                      : PWFS_ERR_HIP;
  if (prev != dev) (void)hipSetDevice(prev);
  return st;
}
