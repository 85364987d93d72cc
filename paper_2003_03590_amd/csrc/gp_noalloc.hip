// gp_energies_static: gp_energies with its diagnostics workspace in a static
// device array, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ object of GP_STATIC_WORK_BYTES, held by
// every GPU the library runs on until the process ends.  Host code never passes
// the array's name to a kernel (in host code it is only a stand-in for the
// symbol): on the first call on a device, with that device current, its device
// address is looked up with hipGetSymbolAddress and kept per device; kernels get
// that address as their workspace argument, exactly as gp_energies passes the
// caller's workspace.  Nothing in this path calls hipMalloc or hipFree.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gp.h"

struct gp_plan_s;

namespace gpk {
gp_status energies_static_args(gp_plan_s* p, const void* psi, const gp_energy* out, size_t max_bytes);
gp_status energies_on(gp_plan_s* p, const void* psi, void* work, gp_energy* out);
gp_status report_error(gp_status st, const char* msg);
}  // namespace gpk

// 4 states of the largest grid served: 96^3 complex128 or 128^3 complex64
static __device__ __align__(256) unsigned char scratch[GP_STATIC_WORK_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of the array (looked up once per device)
gp_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return gpk::report_error(GP_ERR_HIP, "hipGetDevice failed or device index out of range");
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return gpk::report_error(GP_ERR_HIP, "hipGetSymbolAddress of the static workspace failed");
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GP_OK;
}
}  // namespace

extern "C" gp_status gp_energies_static(gp_plan_t* p, const void* psi, gp_energy* out) {
  gp_status st = gpk::energies_static_args(p, psi, out, GP_STATIC_WORK_BYTES);
  if (st != GP_OK) return st;
  void* work = nullptr;
  if ((st = scratch_address(&work)) != GP_OK) return st;
  return gpk::energies_on(p, psi, work, out);
}
