// Measurement probes, the yardsticks the sweeps of the path are compared
// against.  Streaming: the HBM rates a plain kernel reaches on this device
// (a read of n bytes, and a copy of n bytes to another buffer); each thread
// moves 16-byte vectors in a grid-stride loop with U vectors in flight, the
// read folds its data into one word per workgroup so that nothing is
// elided, and the launch shapes tried are a few multiples of the
// compute-unit count.  FP64 vector ALU: the rate of register-only chains of
// binary64 operations (plain FMAs, or the biased DD step of the Gram sweep)
// at 1 to 8 waves per SIMD.  The fastest shape counts.
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

// Register-only FP64 chains over 16 independent sums per thread, two rows
// of operands per trip (128 FP64 instructions): KIND 0 plain FMAs, KIND 1 the
// biased DD step of the Gram sweep (s' = fma(a, b, s); d = s' - s;
// e = fma(a, b, -d); acc += e).  The sums are written to out.
template <int KIND>
__global__ void __launch_bounds__(256) probe_valu_kernel(double* __restrict__ out, int iters,
                                                         double x0) {
  double acs[16], acc[16], a0[4], b0[4], a1[4], b1[4];
  const double t = threadIdx.x * 1e-3 + x0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a0[i] = 1.0 + t * (i + 1);
    b0[i] = 1.0 - t * (i + 2) * 1e-3;
    a1[i] = 1.0 - t * (i + 3) * 1e-2;
    b1[i] = 1.0 + t * (i + 4) * 1e-4;
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    acs[e] = 1024.0 + e;
    acc[e] = 0.0;
  }
  auto step = [&](const double* a, const double* b) {
#pragma unroll
    for (int g8 = 0; g8 < 16; g8 += 8) {
      if (KIND == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            acs[g8 + e] = __builtin_fma(a[(g8 + e) / 4], b[(e + r) % 4], acs[g8 + e]);
      } else {
        double sn[8], d[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) sn[e] = __builtin_fma(a[(g8 + e) / 4], b[e % 4], acs[g8 + e]);
#pragma unroll
        for (int e = 0; e < 8; ++e) d[e] = sn[e] - acs[g8 + e];
#pragma unroll
        for (int e = 0; e < 8; ++e) d[e] = __builtin_fma(a[(g8 + e) / 4], b[e % 4], -d[e]);
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[g8 + e] = acc[g8 + e] + d[e];
#pragma unroll
        for (int e = 0; e < 8; ++e) acs[g8 + e] = sn[e];
      }
    }
  };
  for (int it = 0; it < iters; ++it) {
    step(a0, b0);
    step(a1, b1);
  }
  double r = 0.0;
#pragma unroll
  for (int e = 0; e < 16; ++e) r += acs[e] + acc[e];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = r;
}

}  // namespace
}  // namespace borth

using namespace borth;

extern "C" borth_status borth_valu_probe(borth_ctx c, int kind, void* sink, int64_t nbytes,
                                         double* lane_ops_per_s, int* waves) {
  if (!c) return BORTH_ERR_ARG;
  if (!sink || !lane_ops_per_s || kind < 0 || kind > 1 || nbytes < 0 || ((uintptr_t)sink & 7))
    return fail_arg(c, "valu probe arguments");
  hipSetDevice(c->device);
  int cus = 0;
  HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device), "attr");
  // the largest launch: 8 waves per SIMD = 8 workgroups of 256 threads per CU
  if (nbytes < (int64_t)8 * cus * 256 * (int64_t)sizeof(double))
    return fail_arg(c, "valu probe: sink smaller than 8 x 256 doubles per compute unit");
  const int iters = 2000;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0), "hipEventCreate");
  HIPCHK(c, hipEventCreate(&e1), "hipEventCreate");
  double best = 0.0;
  int bw = 0;
  for (int per : {1, 2, 4, 8}) {
    const int grid = per * cus;
    auto launch = [&]() {
      if (kind == 0)
        hipLaunchKernelGGL(probe_valu_kernel<0>, dim3(grid), dim3(256), 0, c->stream, (double*)sink, iters, 0.5);
      else
        hipLaunchKernelGGL(probe_valu_kernel<1>, dim3(grid), dim3(256), 0, c->stream, (double*)sink, iters, 0.5);
    };
    launch();  // warm-up
    HIPCHK(c, hipEventRecord(e0, c->stream), "hipEventRecord");
    for (int r = 0; r < 3; ++r) launch();
    HIPCHK(c, hipEventRecord(e1, c->stream), "hipEventRecord");
    HIPCHK(c, hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    // 128 FP64 instructions per trip and thread
    const double ops = 128.0 * iters * grid * 256.0 * 3.0;
    const double rate = ops / (ms * 1e-3);
    if (rate > best) {
      best = rate;
      bw = per;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *lane_ops_per_s = best;
  if (waves) *waves = bw;
  return BORTH_OK;
}

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
