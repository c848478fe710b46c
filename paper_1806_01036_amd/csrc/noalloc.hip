// Device scratch of the allocation-free entry point
// (borth_orthonormalize_noalloc): one file-scope array per device that holds
// the status words, the k x k workspace and the per-workgroup Gram partials
// of a call, so that the call itself allocates nothing.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy is taken once per device with
// hipGetSymbolAddress (at context creation, that device current) and only
// that address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.hpp"

namespace borth {

static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) {
    e = hipSetDevice(device);
    if (e != hipSuccess) return e;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) hipSetDevice(cur);
  if (e != hipSuccess) return e;
  g_ptr[device] = (double*)p;
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace borth
