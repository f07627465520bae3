// Allocation-free force evaluation: esp_forces on a plan whose device buffers
// are carved out of a fixed, file-scope device array instead of hipMalloc.
//
// The array is one per GPU (each device that loads the library's code objects
// holds its own copy, at its own address, until the process ends).  Host code
// never uses the array's name as a device address: its address on the current
// device is looked up once per device with hipGetSymbolAddress, kept, and
// passed to the plan as the region its buffers live in.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/esp.h"
#include "esp_internal.h"

namespace {

constexpr size_t kScratchBytes = ESP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (looked up on the
// first call made with that device current).
esp_status scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    std::fprintf(stderr, "esp_forces_noalloc: no usable current device (%s)\n",
                 e != hipSuccess ? hipGetErrorString(e) : "device index out of range");
    return ESP_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      std::fprintf(stderr, "esp_forces_noalloc: hipGetSymbolAddress of the scratch array failed on device %d: %s\n",
                   dev, hipGetErrorString(e));
      return ESP_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return ESP_OK;
}

}  // namespace

extern "C" esp_status esp_forces_noalloc(const double h[9], int64_t n, double tol, const esp_opts* o,
                                         const float* xyz, const float* q, float* f, double* out7) {
  if (!h || !xyz || !q || !f) {
    std::fprintf(stderr, "esp_forces_noalloc: null pointer argument\n");
    return ESP_EINVAL;
  }
  esp_opts opt;
  if (o)
    opt = *o;
  else
    esp_opts_default(&opt);
  if (opt.precision != ESP_FP32) {
    std::fprintf(stderr, "esp_forces_noalloc: FP32 only (o->precision must be ESP_FP32)\n");
    return ESP_EINVAL;
  }
  if (opt.params == ESP_LEARNED) {
    // the proposer evaluates its network in device buffers of its own
    std::fprintf(stderr, "esp_forces_noalloc: learned parameters are not served (use ESP_ANALYTIC or ESP_EXPLICIT)\n");
    return ESP_EINVAL;
  }
  if (opt.local_virial) {
    std::fprintf(stderr, "esp_forces_noalloc: local_virial is not served\n");
    return ESP_EINVAL;
  }
  void* base = nullptr;
  esp_status st = scratch_on_current_device(&base);
  if (st != ESP_OK) return st;
  esp_plan_t* p = nullptr;
  size_t used = 0;
  st = espx::plan_in_region(h, n, tol, &opt, base, kScratchBytes, &p, &used);
  if (st < 0) {
    if (st == ESP_ENOMEM)
      std::fprintf(stderr, "esp_forces_noalloc: n = %lld at tol %g needs more than the %zu-byte scratch array\n",
                   static_cast<long long>(n), tol, kScratchBytes);
    return st;
  }
  const esp_status sf = esp_forces(p, xyz, q, f, out7);
  if (sf < 0) std::fprintf(stderr, "esp_forces_noalloc: %s\n", esp_last_error(p));
  espx::plan_release(p);
  return sf < 0 ? sf : st;
}
