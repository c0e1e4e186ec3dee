// bse_apply_noalloc: the pass of bse_apply for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  The partial sums of the pass live in a fixed device
// array of this file instead of the handle's lazily allocated buffers.
//
// The array is a file-scope __device__ object: each GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in symbol); it passes the device address obtained once per device
// with hipGetSymbolAddress while that device is current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bse.h"
#include "bse_internal.h"

namespace {

constexpr size_t kScratchBytes = BSE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];

std::mutex g_mu;
double2* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call
// on the device, with the device current).
hipError_t scratch_ptr(int dev, double2** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (double2*)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// Makes dev current for the scope and restores the previous device.
struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" bse_status bse_apply_noalloc(bse_handle h, bse_op op, bse_precision precision, int64_t nvec,
                                        const void* x, void* y) {
  if (!h) return BSE_ERR_INVALID_ARG;
  const int dev = bse::handle_device(h);
  if (dev < 0 || dev >= kMaxDevices) return BSE_ERR_DEVICE;
  DeviceScope scope(dev);
  if (scope.err != hipSuccess) return BSE_ERR_DEVICE;
  double2* ws = nullptr;
  if (scratch_ptr(dev, &ws) != hipSuccess) return BSE_ERR_DEVICE;
  // every partial the kernels read is written earlier in the same call, so the
  // previous call's contents need no clearing
  return bse::apply_into(h, op, precision, nvec, x, y, ws, kScratchBytes / sizeof(double2));
}
