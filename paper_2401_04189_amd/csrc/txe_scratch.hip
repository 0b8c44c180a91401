// Workspace of the allocation-free apply: one file-scope device array per
// GPU, held from the load of this code object until the process ends.  Host
// code never uses the array's name as an address: at set-up (context
// creation, once per device, with that device current) hipGetSymbolAddress
// returns the device address of that GPU's copy, kept per device and passed
// to the kernels like any workspace pointer.  This translation unit holds no
// kernel, so the array's code object is separate from the kernels'.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/txe.h"
#include "txe_internal.h"

namespace txe {

static __device__ __align__(256) unsigned char scratch[TXE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};
bool g_done[MAX_DEVICES] = {};
}  // namespace

// The device address of the scratch array on `device` (the current device
// must be `device`); the symbol lookup runs once per device and its result
// (or error) is kept.
hipError_t scratch_address(int device, void **ptr) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    void *p = nullptr;
    g_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[device] = g_err[device] == hipSuccess ? p : nullptr;
    g_done[device] = true;
  }
  *ptr = g_ptr[device];
  return g_err[device];
}

}  // namespace txe
