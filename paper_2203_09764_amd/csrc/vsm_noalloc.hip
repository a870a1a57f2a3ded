// vsm_noalloc.hip -- vsm_smooth on a static device array: the entry point for
// callers that cannot allocate device memory (graph capture, serving loops,
// harnesses that forbid hipMalloc).
#include <mutex>

#include "vsm.h"
#include "vsm_host.h"

using namespace vsm;

namespace {

// The scratch: one array per device, in the library's code object, never
// allocated or freed by a call.  In host code `scratch` names a host-side
// stand-in, not device memory; the device address comes from
// hipGetSymbolAddress, once per device, with that device current, and only that
// address is passed to kernels.
constexpr size_t kScratchBytes = (size_t)VSM_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, or null with *status
// set (the HIP error recorded for vsm_last_hip_error).
void* device_scratch(int* status) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *status = note_hip_error(e);
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *status = VSM_E_PARAM;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *status = note_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *status = VSM_OK;
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

size_t vsm_noalloc_scratch_bytes(void) { return kScratchBytes; }

int vsm_smooth_noalloc(const int32_t dims[4], int32_t precision, void* links_dev, const int8_t* z3_dev,
                       const double* gauge_dev, int32_t n_sweeps, double rho, double eps,
                       const vsm_schedule* sched, int32_t measure_every, vsm_stats* stats_dev, void* stream) {
  // the size check comes first, so that an oversized call fails before any HIP call
  int rc = check_sched(sched);
  if (rc) return rc;
  rc = check_dims_impl(dims, sched->order, precision);
  if (rc) return rc;
  if (ws_layout(dims, precision, sched->order).total > kScratchBytes) return VSM_E_WORKSPACE;
  void* ws = device_scratch(&rc);
  if (!ws) return rc;
  // smooth_impl clears the rejection counter and rewrites the charges, the
  // reduction slots and the smearing buffer before it reads them
  return smooth_impl(dims, precision, links_dev, z3_dev, gauge_dev, (char*)ws, kScratchBytes, n_sweeps, rho, eps,
                     sched, measure_every, stats_dev, (hipStream_t)stream);
}

}  // extern "C"
