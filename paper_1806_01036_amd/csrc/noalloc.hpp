// Device scratch of the allocation-free entry point (host interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace borth {

// A file-scope device array of this many doubles (32 MiB) per device, whose
// device address noalloc_setup takes once per device (hipGetSymbolAddress,
// that device current) and noalloc_scratch returns afterwards (null before
// setup).
constexpr int64_t kNoallocScratchDoubles = int64_t(1) << 22;
hipError_t noalloc_setup(int device);
double* noalloc_scratch(int device);

}  // namespace borth
