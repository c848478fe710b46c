// Streaming probes: the HBM rates a plain kernel reaches on this device, the
// yardstick the sweeps of the path are compared against (a read of n bytes,
// and a copy of n bytes to another buffer).  Each thread moves 16-byte
// vectors in a grid-stride loop with U vectors in flight; the read folds its
// data into one word per workgroup so that nothing is elided.  The launch
// shapes tried are a few multiples of the compute-unit count; the fastest
// counts.
#include <hip/hip_runtime.h>

#include <vector>

#include "ctx.hpp"

namespace borth {
namespace {

typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

template <int U>
__global__ void __launch_bounds__(256) probe_read_kernel(const u4_t* __restrict__ src, int64_t n,
                                                         unsigned* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  u4_t acc = {0u, 0u, 0u, 0u};
  for (; i + (U - 1) * stride < n; i += U * stride) {
    u4_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u];
  }
  for (; i < n; i += stride) acc ^= src[i];
  const unsigned x = acc.x ^ acc.y ^ acc.z ^ acc.w;
  __shared__ unsigned red[256];
  red[threadIdx.x] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned r = 0u;
    for (int t = 0; t < 256; ++t) r ^= red[t];
    sink[blockIdx.x] = r;
  }
}

template <int U, bool NT>
__global__ void __launch_bounds__(256) probe_copy_kernel(const u4_t* __restrict__ src,
                                                         u4_t* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    u4_t v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (NT)
        __builtin_nontemporal_store(v[u], dst + i + u * stride);
      else
        dst[i + u * stride] = v[u];
    }
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace
}  // namespace borth

using namespace borth;

extern "C" borth_status borth_stream_probe(borth_ctx c, int kind, const void* src, void* dst,
                                           int64_t nbytes, int reps, double* best_ms,
                                           int* best_grid) {
  if (!c) return BORTH_ERR_ARG;
  if (!src || !dst || !best_ms || nbytes < 16 || (nbytes & 15) || reps < 1 || kind < 0 ||
      kind > 2 || (((uintptr_t)src | (uintptr_t)dst) & 15))
    return fail_arg(c, "stream probe arguments");
  hipSetDevice(c->device);
  int cus = 0;
  HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device), "attr");
  const int64_t n = nbytes / 16;
  // a read writes one word per workgroup to dst (at most 16 x CUs words)
  std::vector<int> grids = {2 * cus, 4 * cus, 8 * cus, 16 * cus};
  unsigned* sink = kind == 0 ? (unsigned*)dst : nullptr;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0), "hipEventCreate");
  HIPCHK(c, hipEventCreate(&e1), "hipEventCreate");
  double best = 1e30;
  int bg = 0;
  const u4_t* s = (const u4_t*)src;
  u4_t* d = (u4_t*)dst;
  for (int g : grids) {
    auto launch = [&]() {
      if (kind == 0)
        hipLaunchKernelGGL((probe_read_kernel<4>), dim3(g), dim3(256), 0, c->stream, s, n, sink);
      else if (kind == 1)
        hipLaunchKernelGGL((probe_copy_kernel<4, false>), dim3(g), dim3(256), 0, c->stream, s, d, n);
      else
        hipLaunchKernelGGL((probe_copy_kernel<4, true>), dim3(g), dim3(256), 0, c->stream, s, d, n);
    };
    launch();  // warm-up
    HIPCHK(c, hipEventRecord(e0, c->stream), "hipEventRecord");
    for (int r = 0; r < reps; ++r) launch();
    HIPCHK(c, hipEventRecord(e1, c->stream), "hipEventRecord");
    HIPCHK(c, hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    const double per = ms / reps;
    if (per < best) {
      best = per;
      bg = g;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *best_ms = best;
  if (best_grid) *best_grid = bg;
  return BORTH_OK;
}
