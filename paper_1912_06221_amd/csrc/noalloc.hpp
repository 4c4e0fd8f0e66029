// Scratch memory of the entry points that allocate nothing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace ardg {

// Capacity of the per-device scratch array (64 MiB): the edge fluxes of
// one right-hand side, F * (E_int + E_bdy) * Nfp values of the compute type.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;

// Device address of `device`'s scratch array, looked up with
// hipGetSymbolAddress on the first call for that device (which must be the
// current device then) and cached.  Allocates nothing.
hipError_t noalloc_scratch(int device, void** ptr);

}  // namespace ardg
