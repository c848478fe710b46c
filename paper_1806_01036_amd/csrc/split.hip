// Split-precision Gram sweep for an fp32 block X on the matrix cores.
//
// Each fp32 element is split into two bfloat16 words, h = bf16(x) and
// l = bf16(x - h) (round to nearest even; x - h is exact in fp32), so that
// h + l carries 16 significant bits of x.  The Gram matrix is approximated by
//     G ~ H^T H + H^T L + L^T H
// with v_mfma_f32_16x16x32_bf16 (fp32 accumulation); the dropped L^T L term
// and the unsplit remainder are ~2^-16 of |x_i||x_j|.  fp32 accumulators are
// flushed into binary64 every `flush` 32-row groups so that the fp32
// accumulation error stays below the split error.  The resulting Gram
// matrix is accurate to ~2^-15 relative; the factorization that follows uses
// a diagonal shift to stay positive definite and later binary64 passes win
// the accuracy back.
//
// Operand layout: lane l supplies, for column block I, the 8 values of
// column 16 I + l % 16 in rows 32 g + 8 (l / 16) + e, e = 0..7; the same
// register serves as the A operand (tile row I) and the B operand (tile
// column I), so the contraction over the 32 rows pairs matching rows.
#include "dd.hpp"
#include "internal.hpp"

namespace borth {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4s_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int tile_index_s(int ti, int tj, int T4) {
  return ti * T4 - (ti * (ti - 1)) / 2 + (tj - ti);
}

template <int T>
__global__ void __launch_bounds__(256) gram_split_kernel(Src s, GramLayout L, int64_t ngroups,
                                                         int flush, double* __restrict__ part) {
  constexpr int NTL = T * (T + 1) / 2;
  __shared__ double red[NTL * 4 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int c = lane & 15, kg = lane >> 4;
  const float* __restrict__ X = (const float*)s.X;
  f4_t a32[NTL];
  d4s_t a64[NTL];
#pragma unroll
  for (int i = 0; i < NTL; ++i) {
    a32[i] = f4_t{0.f, 0.f, 0.f, 0.f};
    a64[i] = d4s_t{0.0, 0.0, 0.0, 0.0};
  }
  int since = 0;
  const int64_t gstride = (int64_t)gridDim.x * nw;
  for (int64_t g = (int64_t)blockIdx.x * nw + wave; g < ngroups; g += gstride) {
    const int64_t rbase = g * 32 + kg * 8;
    bf16x8_t h[T], l[T];
    // unconditional loads (row clamped to m - 1, column to 0), zero selected after
    float xv[T][8];
#pragma unroll
    for (int I = 0; I < T; ++I) {
      const int col = 16 * I + c;
      const int cc = col < L.k ? col : 0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t row = rbase + e;
        xv[I][e] = X[(row < s.m ? row : s.m - 1) * s.ldx + cc];
      }
    }
#pragma unroll
    for (int I = 0; I < T; ++I) {
      const int col = 16 * I + c;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t row = rbase + e;
        const float x = (row < s.m && col < L.k) ? xv[I][e] : 0.f;
        const __bf16 hb = (__bf16)x;
        h[I][e] = hb;
        l[I][e] = (__bf16)(x - (float)hb);
      }
    }
    int idx = 0;
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
      for (int J = I; J < T; ++J) {
        a32[idx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h[I], h[J], a32[idx], 0, 0, 0);
        a32[idx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h[I], l[J], a32[idx], 0, 0, 0);
        a32[idx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l[I], h[J], a32[idx], 0, 0, 0);
        ++idx;
      }
    if (++since == flush) {
#pragma unroll
      for (int i = 0; i < NTL; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) a64[i][v] += (double)a32[i][v];
        a32[i] = f4_t{0.f, 0.f, 0.f, 0.f};
      }
      since = 0;
    }
  }
#pragma unroll
  for (int i = 0; i < NTL; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) a64[i][v] += (double)a32[i][v];

  for (int w = 1; w < nw; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(i * 4 + v) * 64 + lane] = a64[i][v];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) a64[i][v] += red[(i * 4 + v) * 64 + lane];
    }
  }
  if (wave != 0) return;
  double* out = part + (int64_t)blockIdx.x * L.E;
  int idx = 0;
#pragma unroll
  for (int I = 0; I < T; ++I)
#pragma unroll
    for (int J = I; J < T; ++J) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = 16 * I + 4 * kg + v, gj = 16 * J + c;
        if (gi < L.Wp && gj < L.Wp && (gi >> 2) <= (gj >> 2)) {
          const int e = tile_index_s(gi >> 2, gj >> 2, L.T4) * 16 + (gi & 3) * 4 + (gj & 3);
          out[e] = a64[idx][v];
        }
      }
      ++idx;
    }
}

}  // namespace

hipError_t launch_gram_split(const Src& s, const GramLayout& L, double* partials, int64_t cap,
                             int* nwg_out, const TuneGram& tune, hipStream_t st) {
  if (!s.x_f32 || L.kyp != 0 || L.k > 64) return hipErrorInvalidValue;
  const int T = (L.Wp + 15) / 16;
  const int64_t ngroups = (s.m + 31) / 32;
  int nwg = tune.nwg > 0 ? tune.nwg : 1024;
  const int64_t need = (ngroups + 3) / 4;
  if (nwg > need) nwg = (int)(need > 0 ? need : 1);
  if ((int64_t)nwg * L.E > cap) return hipErrorInvalidValue;
  const int flush = tune.rows > 0 ? (tune.rows + 31) / 32 : 8;
  switch (T) {
    case 1: hipLaunchKernelGGL(gram_split_kernel<1>, dim3(nwg), dim3(256), 0, st, s, L, ngroups, flush, partials); break;
    case 2: hipLaunchKernelGGL(gram_split_kernel<2>, dim3(nwg), dim3(256), 0, st, s, L, ngroups, flush, partials); break;
    case 3: hipLaunchKernelGGL(gram_split_kernel<3>, dim3(nwg), dim3(256), 0, st, s, L, ngroups, flush, partials); break;
    default: hipLaunchKernelGGL(gram_split_kernel<4>, dim3(nwg), dim3(256), 0, st, s, L, ngroups, flush, partials); break;
  }
  *nwg_out = nwg;
  return hipGetLastError();
}

}  // namespace borth
