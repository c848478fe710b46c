// Basis update sweep for narrow blocks: T = (S - Y C) Z per row (Sec. 4.2,
// the projection against the locked vectors followed by the product with the
// factor), for k <= 8 new columns and 0 <= ky <= 64 locked ones, on the
// vector ALUs; optionally with the next pass's Gram columns [Y | T]^T T
// accumulated from the values just computed (the fusion of operations that
// Sec. 4.2 uses to save a sweep over the block; Y^T Y does not change between
// passes and is not recomputed).
//
// With a handful of columns the product is a stream over [Y | S] with a few
// multiply-adds per value: the 16-column tiles of the matrix cores would be
// mostly padding, and the stream is bound by HBM.  The kernel is laid out
// for the stream:
//  * one wave per workgroup (so LDS is granted per wave and many waves fit a
//    CU), one row per lane, 64-row panels taken in a grid-stride loop;
//  * a panel of Y (64 ky values, one contiguous range when ldy == ky) is read
//    with flat loads -- lane l takes values l, l + 64, l + 128, ... -- so that
//    each load instruction covers consecutive bytes, then scattered into LDS
//    rows of odd stride, where each lane reads its own row without bank
//    conflicts;
//  * the next panel's loads are issued before the current panel is computed,
//    so every wave keeps a panel in flight while it works;
//  * C and Z are the same for every lane and are read through the scalar
//    cache; given their low words (the DD variant of Sec. 4.2, extended
//    precision throughout the orthogonalization), the projection and the
//    product with Z run with the Dot2 step and the result is rounded once;
//  * the fused Gram switches to one column per lane: T goes next to Y in the
//    panel's LDS rows and lane c accumulates column c of [Y | T] times each
//    column of T over the panel's rows (in several row phases when the block
//    has fewer than 32 columns), in binary64 or with the Dot2 step.
// The subtraction comes first, in the paper's order: when S lies close to
// span(Y), S Z and Y C Z are much larger than T and would cancel.
#pragma once
#include <map>
#include <mutex>
#include <tuple>

#include "dd.hpp"
#include "internal.hpp"

namespace borth {
namespace nrw {

__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef double d2_t __attribute__((ext_vector_type(2)));

// Fused Gram kinds: 0 none, 1 binary64, 2 DD; 3 and 4 the same weighted by
// the diagonal of B (B-inner products).
__host__ __device__ constexpr int gr_prec(int gr) { return gr > 2 ? gr - 2 : gr; }
__host__ __device__ constexpr bool gr_weighted(int gr) { return gr > 2; }

// LDS row stride of a panel: Y, then (fused Gram) the KN columns of T and
// (weighted) the row's weight; odd.
__host__ __device__ inline int row_stride(int ky, int kn, int gr) {
  return (ky + (gr ? kn : 0) + (gr_weighted(gr) ? 1 : 0)) | 1;
}

// LDS doubles of one wave: the panel, or the phase sums of the fused Gram.
inline size_t lds_doubles(int ky, int kn, int gr) {
  const size_t pan = 64 * (size_t)row_stride(ky, kn, gr);
  const size_t red = gr ? 2 * 64 * (size_t)kn : 0;
  return pan > red ? pan : red;
}

// KN: k rounded up to 1, 2, 4 or 8.  KYB: bound on ky (0, 16, 32 or 64), the
// size of the register buffer that holds a lane's share of a Y panel.  C is
// ky x kp and Z kp x kp, row-major, zero beyond k.
// FAST: Y stored densely (ldy == ky), ky even and Y 16-byte aligned: a full
// panel is one contiguous range of 32 ky pairs, read as 16-byte loads, pair
// q of lane l being pair 64 q + l; LDS positions of the pairs are computed
// once.  Otherwise (and for a ragged last panel) value q of lane l is value
// 64 q + l of the panel, addressed through its row and column.
// GR: 0 no Gram; 1 binary64, 2 DD partials of [Y | T]^T T in the layout G
// (make_layout_xcols), one per workgroup (ky + k <= 64); 3, 4: the same of
// [Y | T]^T B T with B = diag(a.bw).
template <int KN, int KYB, bool FAST, int GR>
__global__ void __launch_bounds__(64) narrow_kernel(UpdDev a, int kp, GramLayout G) {
  extern __shared__ double pan[];
  if (stopped(a.stop, a.pass)) return;
  const int lane = threadIdx.x;
  const int ky = a.ky, k = a.k;
  const int SP = row_stride(ky, KN, GR);
  const int64_t m = a.m;
  const int64_t nfull = FAST ? m / 64 : (m + 63) / 64;  // panels of the main loop
  const double BORTH_GLOBAL* __restrict__ Yg = gmem(a.Y);
  const double BORTH_GLOBAL* __restrict__ Xg = gmem((const double*)a.X);
  // constant address space: uniform reads go through the scalar cache
  typedef const double __attribute__((address_space(4)))* cptr;
  const cptr Cg = (cptr)a.C1;
  const cptr Zg = (cptr)a.Z1;
  const cptr Clg = (cptr)a.C1lo;  // DD arithmetic when the low words are given
  const cptr Zlg = (cptr)a.Z1lo;
  const bool pdd = a.C1lo != nullptr && a.Z1lo != nullptr;
  double BORTH_GLOBAL* __restrict__ Qg = gmem(a.Q);
  const int dense = a.dense;
  constexpr int NY = KYB > 0 ? KYB : 1;
  constexpr int NP = FAST ? (NY + 1) / 2 : 1;
  double yv[NY];
  d2_t yp[NP];
  int loff[NP];
  double xv[KN];
  constexpr bool WB = gr_weighted(GR);
  constexpr int GP = gr_prec(GR);  // 1 binary64, 2 DD
  double wv = 1.0;                 // WB: weight of this lane's row of the loaded panel

  // Fused Gram: lane -> column c of [Y | T], row phase h of H.
  const int W = ky + k;
  const int H = GR ? 64 / (W > 0 ? W : 1) : 1;
  const int gc = GR ? lane % W : 0, gh = GR ? lane / W : 0;
  const bool gact = GR && gh < H;
  double gs[KN], gcmp[KN];
#pragma unroll
  for (int j = 0; j < KN; ++j) gs[j] = gcmp[j] = 0.0;

  // The loads below are straight-line code with no branch on ky: a branch
  // per load would make the compiler wait for every load in flight at each
  // join.  Values past the last one re-read the last value (a cache hit) and
  // are stored to its LDS slot again.
  //
  // Generic addressing: flat position f = 64 q + lane -> row f / ky,
  // column f % ky, advanced by (64 / ky, 64 % ky) per q while q < ky.  Every
  // row is below 64 (f < 64 ky), so LDS stays in bounds.
  const int ky1 = ky > 0 ? ky : 1;
  const int dr = 64 / ky1, dc = 64 % ky1;
  const int r0l = lane / ky1, c0l = lane % ky1;
  const int nq = ky >> 1;  // FAST: pairs per lane
  if (FAST) {
    // pair q covers flat positions 2 (64 q + lane) + {0, 1}, one row (ky even)
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int f = 2 * (64 * (q < nq ? q : nq - 1) + lane);
      loff[q] = (f / ky1) * SP + f % ky1;
    }
  }
  auto step = [&](int q, int& r, int& c) {
    const bool go = q + 1 < ky;
    const int c2 = c + dc;
    const bool wrap = c2 >= ky;
    r = go ? r + dr + (wrap ? 1 : 0) : r;
    c = go ? (wrap ? c2 - ky : c2) : c;
  };

  // Generic loads of panel p (rows past m clamped to the last row: in
  // bounds, results never stored).
  auto load_generic = [&](int64_t p) {
    const int64_t row0 = p * 64;
    const int nrows = (int)(m - row0 < 64 ? m - row0 : 64);
    if (KYB > 0) {
      int r = r0l, c = c0l;
#pragma unroll
      for (int q = 0; q < NY; ++q) {
        const int rr = r < nrows ? r : nrows - 1;
        yv[q] = Yg[(row0 + rr) * a.ldy + c];
        step(q, r, c);
      }
    }
    const int rx = lane < nrows ? lane : nrows - 1;
#pragma unroll
    for (int j = 0; j < KN; ++j) {
      const double v = Xg[(row0 + rx) * a.ldx + (j < k ? j : k - 1)];
      xv[j] = j < k ? v : 0.0;
    }
    if (WB) wv = gmem(a.bw)[row0 + rx];
  };
  auto store_generic = [&]() {
    if (KYB > 0) {
      int r = r0l, c = c0l;
#pragma unroll
      for (int q = 0; q < NY; ++q) {
        pan[r * SP + c] = yv[q];
        step(q, r, c);
      }
    }
  };
  // Full panel p, contiguous: 16-byte loads.
  auto load_fast = [&](int64_t p) {
    const int64_t row0 = p * 64;
    if (KYB > 0) {
      const d2_t BORTH_GLOBAL* yb = (const d2_t BORTH_GLOBAL*)(Yg + row0 * ky) + lane;
#pragma unroll
      for (int q = 0; q < NP; ++q) yp[q] = yb[64 * (q < nq ? q : nq - 1)];
    }
#pragma unroll
    for (int j = 0; j < KN; ++j) {
      const double v = Xg[(row0 + lane) * a.ldx + (j < k ? j : k - 1)];
      xv[j] = j < k ? v : 0.0;
    }
    if (WB) wv = gmem(a.bw)[row0 + lane];
  };
  auto store_fast = [&]() {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      pan[loff[q]] = yp[q].x;
      pan[loff[q] + 1] = yp[q].y;
    }
  };
  // T = S - Y C (one fused multiply-add per product term, S first), Q = T Z;
  // with the fused Gram, T joins the panel and is accumulated column-wise.
  auto compute_store = [&](const double* xs, double ws, int64_t row0, int nrows) {
    double qv[KN], qlo[KN];
    if (!pdd) {
      double t[KN];
#pragma unroll
      for (int j = 0; j < KN; ++j) t[j] = xs[j];
      if (KYB > 0) {
        const double* yrow = pan + lane * SP;
#pragma unroll 4
        for (int c = 0; c < ky; ++c) {
          const double y = yrow[c];
#pragma unroll
          for (int j = 0; j < KN; ++j) t[j] = __builtin_fma(y, -Cg[c * kp + j], t[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < KN; ++j) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < KN; ++l)
          if (l <= j || dense) s = __builtin_fma(t[l], Zg[l * kp + j], s);  // Z upper triangular unless dense
        qv[j] = s;
      }
    } else {
      // DD: T = S - Y (C_hi + C_lo) with the Dot2 step (T kept as a pair),
      // then Q = T (Z_hi + Z_lo) likewise, rounded once at the end
      double ts[KN], te[KN];
#pragma unroll
      for (int j = 0; j < KN; ++j) {
        ts[j] = xs[j];
        // a DD input X: its low word starts the error term
        te[j] = (a.Xlo && lane < nrows && j < k) ? a.Xlo[(row0 + lane) * a.ldx + j] : 0.0;
      }
      if (KYB > 0) {
        const double* yrow = pan + lane * SP;
#pragma unroll 2
        for (int c = 0; c < ky; ++c) {
          const double y = yrow[c];
#pragma unroll
          for (int j = 0; j < KN; ++j) {
            dot2_step(ts[j], te[j], y, -Cg[c * kp + j]);
            te[j] = __builtin_fma(y, -Clg[c * kp + j], te[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < KN; ++j) {
        double s = 0.0, e = 0.0;
#pragma unroll
        for (int l = 0; l < KN; ++l)
          if (l <= j || dense) {
            const double zh = Zg[l * kp + j];
            dot2_step(s, e, ts[l], zh);
            e = __builtin_fma(ts[l], Zlg[l * kp + j], __builtin_fma(te[l], zh, e));
          }
        const dd_t q = two_sum(s, e);
        qv[j] = q.hi;
        qlo[j] = q.lo;
      }
    }
    if (lane < nrows) {
#pragma unroll
      for (int j = 0; j < KN; ++j)
        if (j < k) Qg[(row0 + lane) * a.ldq + j] = qv[j];
      // DD result requested: its low words (qv holds the rounded sum)
      if (pdd && a.Qlo)
#pragma unroll
        for (int j = 0; j < KN; ++j)
          if (j < k) a.Qlo[(row0 + lane) * a.ldq + j] = qlo[j];
    }
    if (GR) {
      // rows past m contribute nothing: their T is zero (their Y is finite)
#pragma unroll
      for (int j = 0; j < KN; ++j) pan[lane * SP + ky + j] = lane < nrows ? qv[j] : 0.0;
      if (WB) pan[lane * SP + ky + KN] = ws;
      lds_sync();
      if (gact) {
        for (int r = gh; r < 64; r += H) {
          const double* row = pan + r * SP;
          const double v = row[gc];
          const double w = WB ? row[ky + KN] : 1.0;
#pragma unroll
          for (int j = 0; j < KN; ++j) {
            // weighted: w t_j = th + tl exactly (TwoProduct), then v (th + tl)
            const double t = row[ky + j];
            const double th = WB ? t * w : t;
            if (GP == 2) {
              dot2_step(gs[j], gcmp[j], v, th);
              if (WB) gcmp[j] = __builtin_fma(v, __builtin_fma(t, w, -th), gcmp[j]);
            } else {
              gs[j] = __builtin_fma(v, th, gs[j]);
            }
          }
        }
      }
    }
  };

  const int64_t stride = gridDim.x;
  int64_t p = blockIdx.x;
  if (p < nfull) {
    if (FAST) load_fast(p); else load_generic(p);
    for (;;) {
      const int64_t row0 = p * 64;
      const int nrows = (int)(m - row0 < 64 ? m - row0 : 64);
      lds_sync();  // this wave's reads of the previous panel are done
      if (FAST) store_fast(); else store_generic();
      double xs[KN];
#pragma unroll
      for (int j = 0; j < KN; ++j) xs[j] = xv[j];
      const double ws = wv;
      const int64_t nx = p + stride;
      if (nx < nfull) {  // in flight while this panel is computed
        if (FAST) load_fast(nx); else load_generic(nx);
      }
      lds_sync();
      compute_store(xs, ws, row0, nrows);
      if (nx >= nfull) break;
      p = nx;
    }
  }
  // FAST: the ragged last panel, by the wave whose grid-stride sequence
  // reaches it
  if (FAST && m % 64 != 0 && (int64_t)blockIdx.x == nfull % stride) {
    lds_sync();
    load_generic(nfull);
    store_generic();
    lds_sync();
    compute_store(xv, wv, nfull * 64, (int)(m - nfull * 64));
  }
  if (!GR) return;

  // Partial of this workgroup: row phases summed in phase order, then
  // written in the tile layout G (zero for padding entries).
  lds_sync();
  double* ph = pan;  // [phase h][column c][j] hi, then lo
  const int PW = 64 * KN;
  if (gact) {
#pragma unroll
    for (int j = 0; j < KN; ++j) {
      const dd_t v = GP == 2 ? dot2_finish(gs[j], gcmp[j]) : dd_from(gs[j]);
      ph[(gh * W + gc) * KN + j] = v.hi;
      ph[PW + (gh * W + gc) * KN + j] = v.lo;
    }
  }
  lds_sync();
  if (gact && gh == 0) {
#pragma unroll
    for (int j = 0; j < KN; ++j) {
      dd_t v = dd_make(ph[gc * KN + j], ph[PW + gc * KN + j]);
      for (int h = 1; h < H; ++h) {
        const int x = (h * W + gc) * KN + j;
        v = GP == 2 ? dd_add(v, dd_make(ph[x], ph[PW + x])) : dd_from(v.hi + ph[x]);
      }
      gs[j] = v.hi;
      gcmp[j] = v.lo;
    }
  }
  lds_sync();
  if (gact && gh == 0) {
#pragma unroll
    for (int j = 0; j < KN; ++j) {
      ph[gc * KN + j] = gs[j];
      ph[PW + gc * KN + j] = gcmp[j];
    }
  }
  lds_sync();
  double BORTH_GLOBAL* out = gmem(a.part) + (int64_t)blockIdx.x * G.E * (GP == 2 ? 2 : 1);
  for (int e = lane; e < G.E; e += 64) {
    // tile t of the layout: row ti holds tiles tj = max(ti, ty) .. T4 - 1
    int t = e >> 4, ti = 0;
    for (;;) {
      const int cnt = G.T4 - (ti > G.ty ? ti : G.ty);
      if (t < cnt) break;
      t -= cnt;
      ++ti;
    }
    const int tj = (ti > G.ty ? ti : G.ty) + t;
    const int pi = 4 * ti + ((e >> 2) & 3), pj = 4 * tj + (e & 3);
    const int li = pi < G.kyp ? (pi < ky ? pi : -1) : (pi - G.kyp < k ? ky + pi - G.kyp : -1);
    const int j = pj - G.kyp;
    const bool ok = li >= 0 && j >= 0 && j < k;
    const double hi = ok ? ph[li * KN + (ok ? j : 0)] : 0.0;
    const double lo = ok ? ph[PW + li * KN + (ok ? j : 0)] : 0.0;
    if (GP == 2) {
      out[2 * e] = hi;
      out[2 * e + 1] = lo;
    } else {
      out[e] = hi;
    }
  }
}

// Resident waves of a kernel instance (cached per device and LDS size).
template <int KN, int KYB, bool FAST, int GR>
int resident_waves(size_t shmem) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  static std::mutex mu;
  static std::map<std::tuple<int, size_t>, int> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(std::make_tuple(dev, shmem));
    if (it != cache.end()) return it->second;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, narrow_kernel<KN, KYB, FAST, GR>, 64, shmem) !=
          hipSuccess ||
      per < 1)
    return 0;
  std::lock_guard<std::mutex> lk(mu);
  cache[std::make_tuple(dev, shmem)] = per * cus;
  return per * cus;
}

// Launch with at most max_wg workgroups (the fused Gram's partial slots);
// *grid_out = workgroups launched (= partials written).
template <int KN, int KYB, bool FAST, int GR>
hipError_t launch_t(const UpdDev& d, int kp, const GramLayout& G, int64_t max_wg, int* grid_out,
                    hipStream_t st) {
  const size_t shmem = sizeof(double) * lds_doubles(d.ky, KN, GR);
  const int resident = resident_waves<KN, KYB, FAST, GR>(shmem);
  if (resident < 1) return hipErrorInvalidConfiguration;
  int64_t grid = (d.m + 63) / 64;
  if (grid > resident) grid = resident;
  if (grid > max_wg) grid = max_wg;
  if (grid < 1) return hipErrorInvalidValue;
  *grid_out = (int)grid;
  hipLaunchKernelGGL((narrow_kernel<KN, KYB, FAST, GR>), dim3((unsigned)grid), dim3(64), shmem, st, d,
                     kp, G);
  return hipGetLastError();
}

inline bool fast_y(const UpdDev& d) {
  return d.ky > 0 && d.ky % 2 == 0 && d.ldy == d.ky && ((uintptr_t)d.Y & 15) == 0;
}

inline int kn_of(int k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : 8; }

}  // namespace nrw
}  // namespace borth
