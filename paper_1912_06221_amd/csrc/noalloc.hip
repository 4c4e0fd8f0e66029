// Device-resident scratch memory for the entry points that allocate nothing
// (ardg_rhs_eval_noalloc).
//
// The edge fluxes of one right-hand side evaluation live in a file-scope
// device array instead of memory the library allocates on first use.  The
// array's name is a host-side stand-in in host code: its device address is
// taken once per device with hipGetSymbolAddress, with that device current,
// and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>

#include "noalloc.hpp"

namespace ardg {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace ardg
