// Basis update sweep (TSMM), "Y = Xt Z" of Sec. 4.2 with the phase-I
// projection folded in:  T = (S - Y C) Z  per row, S = X (first pass) or
// Q_1 (later passes).  Optionally a second stage T = (T - Y C2) Z2 follows in
// registers (CholQR2 with Q_1 recomputed instead of stored), and the Gram
// matrix of [Y | T] needed by the next pass is accumulated from the values
// just computed ("kernel fusion ... to further reduce memory accesses",
// Sec. 4.2).
//
// Layout: a workgroup has NW waves; each wave owns a 64-row panel of [Y | S]
// in LDS (row stride Wp + 2 doubles: conflict-free 16-byte row reads).
//   1. coalesced global -> LDS load of the panel (zero-filled outside m, k, ky);
//   2. lane r computes row r: xt = s - y C (FMAs, C and Z are wave-uniform
//      and come through scalar loads), then t_j = sum_{i<=j} xt_i Z_ij (all i
//      for a dense Z), written back into the row;
//   3. coalesced LDS -> global store of T (if Q is given);
//   4. the Gram of [Y | T] over the panel on the matrix cores
//      (v_mfma_f64_16x16x4, operands read from LDS), accumulated per wave.
// The waves' Gram accumulators are summed in wave order at the end and
// written as one partial per workgroup (same tile layout as the Gram sweep).
#pragma once
#include "dd.hpp"
#include "internal.hpp"

namespace borth {

namespace upd {

typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int tile_index_u(int ti, int tj, int T4) {
  return ti * T4 - (ti * (ti - 1)) / 2 + (tj - ti);
}


// GR: 0 = no Gram, 1 = Gram of T (no Y), 2 = Gram of [Y | T] with ky <= 16.
template <int K, bool TWO, int GR, typename ST>
__global__ void __launch_bounds__(256) update_kernel(UpdDev a,
                                                         const double* __restrict__ C1,
                                                         const double* __restrict__ Z1,
                                                         const double* __restrict__ C2,
                                                         const double* __restrict__ Z2) {
  extern __shared__ double lds[];
  constexpr bool GRAM = GR != 0;
  constexpr int T16max = GR == 2 ? (K + 31) / 16 : (K + 15) / 16;
  constexpr int NTLc = T16max * (T16max + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  const int stride = a.Wp + 2;
  double* pan = lds + wave * 64 * stride;
  const int kyp = a.kyp, ky = a.ky;
  const int T16 = (a.gWp + 15) >> 4;  // <= T16max (host checks)
  const ST* __restrict__ X = (const ST*)a.X;

  d4_t acc[NTLc];
  if (GRAM) {
#pragma unroll
    for (int i = 0; i < NTLc; ++i) acc[i] = d4_t{0.0, 0.0, 0.0, 0.0};
  }

  const int64_t pstride = (int64_t)gridDim.x * NW;
  const int64_t niter = (a.npanels - (int64_t)blockIdx.x * NW + pstride - 1) / pstride;
  for (int64_t it = 0; it < niter; ++it) {
    const int64_t pnl = (int64_t)blockIdx.x * NW + wave + it * pstride;
    const bool live = pnl < a.npanels;
    const int64_t row0 = pnl * 64;
    // 1. load [Y | S] panel
    if (live) {
      for (int idx = lane; idx < 64 * kyp; idx += 64) {
        const int r = idx / kyp, c = idx - r * kyp;
        const int64_t row = row0 + r;
        pan[r * stride + c] = (row < a.m && c < ky) ? a.Y[row * a.ldy + c] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int idx = lane + 64 * q;
        const int r = idx / K, c = idx % K;
        const int64_t row = row0 + r;
        pan[r * stride + kyp + c] = (row < a.m && c < a.k) ? (double)X[row * a.ldx + c] : 0.0;
      }
    }
    __syncthreads();
    // 2. per-row transform (lane = row)
    if (live) {
      double* rowp = pan + lane * stride;
#pragma unroll 1
      for (int stage = 0; stage < (TWO ? 2 : 1); ++stage) {
        const double* __restrict__ C = stage ? C2 : C1;
        const double* __restrict__ Z = stage ? Z2 : Z1;
        double xt[K];
#pragma unroll
        for (int j = 0; j < K; j += 2) {
          const double2 v = *(const double2*)(rowp + kyp + j);
          xt[j] = v.x;
          xt[j + 1] = v.y;
        }
        for (int l = 0; l < ky; ++l) {
          const double yl = rowp[l];
#pragma unroll
          for (int j = 0; j < K; ++j) xt[j] = __builtin_fma(-yl, C[l * K + j], xt[j]);
        }
        if (a.dense) {
#pragma unroll 1
          for (int j = 0; j < K; ++j) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < K; ++i) s = __builtin_fma(xt[i], Z[i * K + j], s);
            rowp[kyp + j] = s;
          }
        } else {
#pragma unroll
          for (int j = 0; j < K; ++j) {
            double s = xt[0] * Z[j];
#pragma unroll
            for (int i = 1; i <= j; ++i) s = __builtin_fma(xt[i], Z[i * K + j], s);
            rowp[kyp + j] = s;
          }
        }
      }
    }
    __syncthreads();
    // 3. store
    if (live && a.Q) {
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int idx = lane + 64 * q;
        const int r = idx / K, c = idx % K;
        const int64_t row = row0 + r;
        if (row < a.m && c < a.k) a.Q[row * a.ldq + c] = pan[r * stride + kyp + c];
      }
    }
    // 4. Gram of [Y | T] on the matrix cores
    if (GRAM && live) {
      const int c = lane & 15, rs = lane >> 4;
      for (int g = 0; g < 16; ++g) {
        const double* rp = pan + (4 * g + rs) * stride + a.gbase;
        double v[T16max];
#pragma unroll
        for (int I = 0; I < T16max; ++I) {
          const int col = 16 * I + c;
          v[I] = (I < T16 && col < a.gWp) ? rp[col] : 0.0;
        }
        int idx = 0;
#pragma unroll
        for (int I = 0; I < T16max; ++I)
#pragma unroll
          for (int J = I; J < T16max; ++J) {
            if (J < T16)
              acc[idx] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[I], v[J], acc[idx], 0, 0, 0);
            ++idx;
          }
      }
    }
    __syncthreads();
  }

  if (!GRAM) return;
  // Sum the waves' accumulators in wave order into wave 0, write the partial.
  double* red = lds;
  for (int w = 1; w < NW; ++w) {
    __syncthreads();
    if (wave == w) {
      int idx = 0;
#pragma unroll
      for (int I = 0; I < T16max; ++I)
#pragma unroll
        for (int J = I; J < T16max; ++J) {
          if (J < T16)
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) red[(idx * 4 + vv) * 64 + lane] = acc[idx][vv];
          ++idx;
        }
    }
    __syncthreads();
    if (wave == 0) {
      int idx = 0;
#pragma unroll
      for (int I = 0; I < T16max; ++I)
#pragma unroll
        for (int J = I; J < T16max; ++J) {
          if (J < T16)
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) acc[idx][vv] += red[(idx * 4 + vv) * 64 + lane];
          ++idx;
        }
    }
  }
  if (wave != 0) return;
  double* out = a.part + (int64_t)blockIdx.x * a.gE;
  const int c = lane & 15, rs = lane >> 4;
  int idx = 0;
#pragma unroll
  for (int I = 0; I < T16max; ++I)
#pragma unroll
    for (int J = I; J < T16max; ++J) {
      if (J < T16) {
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          // v_mfma_f64_16x16x4 D layout: lane l, register vv -> D[l/16 + 4 vv][l%16]
          const int gi = 16 * I + rs + 4 * vv, gj = 16 * J + c;
          if (gi < a.gWp && gj < a.gWp && (gi >> 2) <= (gj >> 2)) {
            const int e = tile_index_u(gi >> 2, gj >> 2, a.gT4) * 16 + (gi & 3) * 4 + (gj & 3);
            out[e] = acc[idx][vv];
          }
        }
      }
      ++idx;
    }
}

template <int K, bool TWO, int GR, typename ST>
hipError_t launch_upd_t(const UpdDev& d, const UpdateArgs& a, int nwg, hipStream_t st) {
  const int NW = (d.Wp <= 48) ? 4 : 2;
  const size_t panel = (size_t)NW * 64 * (d.Wp + 2);
  constexpr int T16max = GR == 2 ? (K + 31) / 16 : (K + 15) / 16;
  const size_t red = GR ? T16max * (T16max + 1) / 2 * 4 * 64 : 0;
  const size_t shmem = sizeof(double) * (panel > red ? panel : red);
  hipLaunchKernelGGL((update_kernel<K, TWO, GR, ST>), dim3(nwg), dim3(64 * NW), shmem, st, d,
                     a.C1, a.Z1, a.C2, a.Z2);
  return hipGetLastError();
}

template <int K, bool TWO, typename ST>
hipError_t launch_upd_g(const UpdDev& d, const UpdateArgs& a, int nwg, hipStream_t st) {
  if (!d.part) return launch_upd_t<K, TWO, 0, ST>(d, a, nwg, st);
  if (!a.gram_with_y || d.kyp == 0) return launch_upd_t<K, TWO, 1, ST>(d, a, nwg, st);
  if (d.kyp <= 16) return launch_upd_t<K, TWO, 2, ST>(d, a, nwg, st);
  return hipErrorInvalidValue;
}

template <int K>
hipError_t launch_upd_k(const UpdDev& d, const UpdateArgs& a, int nwg, hipStream_t st) {
  if (a.src.x_f32) {
    if (a.two_stage || d.kyp || (d.part && a.gram_with_y)) return hipErrorInvalidValue;
    return d.part ? launch_upd_t<K, false, 1, float>(d, a, nwg, st)
                  : launch_upd_t<K, false, 0, float>(d, a, nwg, st);
  }
  if (a.two_stage) return launch_upd_g<K, true, double>(d, a, nwg, st);
  return launch_upd_g<K, false, double>(d, a, nwg, st);
}

}  // namespace upd
}  // namespace borth
