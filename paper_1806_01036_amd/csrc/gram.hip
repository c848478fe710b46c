// Gram sweeps (TSMTTSM): G = V^T V for the tall-skinny V = [Y | X].
//
// The Gram matrix is where most of the orthogonalization's work lies
// (Sec. 4.2); for a few columns it is bound by the HBM stream.  Four
// kernels, all writing per-workgroup partials in one shared layout (4x4
// tiles of the upper triangle, see GramLayout) that a fixed-order reduction
// turns into G:
//
//  gram_mfma_kernel    binary64 on the matrix cores, v_mfma_f64_16x16x4:
//                      each wave streams 4-row groups straight from HBM into
//                      registers; lane l holds V[r0 + l/16][16 I + l%16],
//                      which is both the A operand of tile row I and the B
//                      operand of tile column I, so a 16x16 tile of G costs
//                      one MFMA per 4 rows and no LDS traffic.
//  gram_tiles_kernel   binary64 or double-double on the vector ALUs: row
//                      panels are staged in LDS with coalesced loads, each
//                      thread owns a 4x4 tile of G (and a row phase) and
//                      accumulates it.  DD runs the 4-instruction biased
//                      error-free sum (each panel summed on a power-of-two
//                      bias and folded into a DD total), or on request the
//                      8-instruction Dot2 step (dd.hpp).
//  gram_dd_dma_kernel  the biased DD sum with its row panels copied from HBM
//                      straight into LDS (gfx950 global_load_lds_dwordx4);
//                      the default DD sweep for 16-byte aligned binary64 rows,
//                      and with Dot2 sums the Dot2 sweep of a single block.
//  reduce_kernel       sums the partials in workgroup order (DD additions in
//                      DD mode) -- no floating-point atomics, so every result
//                      is bitwise reproducible.
#include <map>
#include <mutex>
#include <tuple>

#include "dd.hpp"
#include "gram_impl.hpp"
#include "internal.hpp"

namespace borth {

GramLayout make_layout(int ky, int k, int kp_min) {
  GramLayout L;
  L.ky = ky;
  L.kyp = (ky + 3) & ~3;
  L.k = k;
  int kp = (k + 3) & ~3;
  L.kp = kp < kp_min ? kp_min : kp;
  L.Wp = L.kyp + L.kp;
  L.T4 = L.Wp / 4;
  L.ntiles = L.T4 * (L.T4 + 1) / 2;
  L.E = 16 * L.ntiles;
  L.ty = 0;
  return L;
}

GramLayout make_layout_xcols(int ky, int k, int kp_min) {
  GramLayout L = make_layout(ky, k, kp_min);
  L.ty = L.kyp / 4;
  int n = 0;
  for (int ti = 0; ti < L.T4; ++ti) n += L.T4 - (ti > L.ty ? ti : L.ty);
  L.ntiles = n;
  L.E = 16 * n;
  return L;
}

// Kernel wrappers of the bodies in gram_impl.hpp.
template <bool DD, int NTB, bool BATCH, bool WB>
__global__ void __launch_bounds__(NTB) gram_tiles_kernel(GramSeg one,
                                                         const GramSeg* __restrict__ tab,
                                                         const int* __restrict__ wg2seg) {
  extern __shared__ double lds[];
  gram_tiles_body<DD, NTB, BATCH, WB>(one, tab, wg2seg, (int)blockIdx.x, lds);
}

template <bool BATCH, bool HASY, int WPC, bool D2 = false>
__global__ void __launch_bounds__(256, 2) gram_dd_dma_kernel(GramSeg one,
                                                             const GramSeg* __restrict__ tab,
                                                             const int* __restrict__ wg2seg) {
  extern __shared__ double lds_all[];
  gram_dd_dma_body<BATCH, HASY, WPC, D2>(one, tab, wg2seg, (int)blockIdx.x, lds_all);
}

// ---------------------------------------------------------------------------
// binary64 Gram of a narrow block (padded width WP <= 8, no weights): one row
// per lane and step, UR rows in flight per lane, all WP (WP + 1) / 2 products
// of a row in registers.  The tile kernel would give each thread a 4x4 tile
// and two rows per panel here, and the MFMA kernel would leave most lanes of
// a 16-column operand empty; both stay far from the HBM stream.  The
// workgroup's sums are combined in a fixed order (shuffle tree in each wave,
// then the waves in order) into one partial in the tile layout.
template <int WP, int KYP>
__global__ void __launch_bounds__(256) gram_rows_kernel(GramSeg g) {
  const Src& s = g.s;
  if (stopped(s.stop, s.pass)) return;
  const GramLayout& L = g.L;
  constexpr int NPR = WP * (WP + 1) / 2, UR = WP <= 4 ? 8 : 4;
  double acc[NPR];
#pragma unroll
  for (int x = 0; x < NPR; ++x) acc[x] = 0.0;
  const int64_t nthr = (int64_t)g.nwg * 256;
  const int ky = L.ky, k = L.k;
  const double BORTH_GLOBAL* Yg = gmem(s.Y);
  const double BORTH_GLOBAL* Xg = gmem((const double*)s.X);
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < s.m; r += UR * nthr) {
    // unconditional loads: row clamped to m - 1, column to the last valid
    // one; the zeros (past m, padding columns) are selected afterwards
    double v[UR][WP];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int64_t row = r + u * nthr;
      const int64_t rc = row < s.m ? row : s.m - 1;
#pragma unroll
      for (int c = 0; c < WP; ++c) {
        const bool isy = c < KYP;
        const int j = isy ? c : c - KYP;
        const int lim = isy ? ky : k;
        const double x = isy ? Yg[rc * s.ldy + (j < ky ? j : ky - 1)]
                             : Xg[rc * s.ldx + (j < k ? j : k - 1)];
        v[u][c] = (row < s.m && j < lim) ? x : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      int x = 0;
#pragma unroll
      for (int i = 0; i < WP; ++i)
#pragma unroll
        for (int j = i; j < WP; ++j, ++x) acc[x] = __builtin_fma(v[u][i], v[u][j], acc[x]);
    }
  }
  __shared__ double red[4][NPR];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int x = 0; x < NPR; ++x) {
    double a = acc[x];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (lane == 0) red[w][x] = a;
  }
  __syncthreads();
  // the partial: tiles (ti <= tj) of 16 entries; the lower half of a diagonal
  // tile holds the mirror entry
  double BORTH_GLOBAL* out = gmem(g.part) + (int64_t)blockIdx.x * L.E;
  for (int e = threadIdx.x; e < L.E; e += 256) {
    int ti, tj;
    decode_tile(e / 16, L, ti, tj);
    int i = 4 * ti + (e % 16) / 4, j = 4 * tj + e % 4;
    if (i > j) {
      const int t = i;
      i = j;
      j = t;
    }
    const int x = i * WP - i * (i - 1) / 2 + (j - i);
    out[e] = ((red[0][x] + red[1][x]) + red[2][x]) + red[3][x];
  }
}

// ---------------------------------------------------------------------------
// binary64 MFMA kernel: T = padded width / 16 column blocks.
typedef double d4_t __attribute__((ext_vector_type(4)));

template <int T, int U, bool BATCH>
__global__ void __launch_bounds__(256) gram_mfma_kernel(GramSeg one,
                                                        const GramSeg* __restrict__ tab,
                                                        const int* __restrict__ wg2seg) {
  constexpr int NTL = T * (T + 1) / 2;
  __shared__ double red[NTL * 4 * 64];
  const GramSeg gs = BATCH ? tab[wg2seg[blockIdx.x]] : one;
  const Src& s = gs.s;
  if (stopped(s.stop, s.pass)) return;
  const GramLayout& L = gs.L;
  const int64_t ngroups = gs.nunits;
  const int wg = (int)blockIdx.x - gs.wg0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int c = lane & 15, rsub = lane >> 4;
  d4_t acc[NTL];
#pragma unroll
  for (int i = 0; i < NTL; ++i) acc[i] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int64_t gstride = (int64_t)gs.nwg * nw;
  int64_t g = (int64_t)wg * nw + wave;
  for (; g < ngroups; g += U * gstride) {
    double v[U][T];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t gg = g + u * gstride;
      const int64_t row = (gg < ngroups) ? gg * 4 + rsub : s.m;
#pragma unroll
      for (int I = 0; I < T; ++I) v[u][I] = fetch(s, L, row, 16 * I + c);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int idx = 0;
#pragma unroll
      for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = I; J < T; ++J) {
          acc[idx] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][I], v[u][J], acc[idx], 0, 0, 0);
          ++idx;
        }
    }
  }

  // Fixed-order cross-wave sum into wave 0.
  for (int w = 1; w < nw; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) red[(i * 4 + vv) * 64 + lane] = acc[i][vv];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) acc[i][vv] += red[(i * 4 + vv) * 64 + lane];
    }
  }
  if (wave != 0) return;
  double BORTH_GLOBAL* out = gmem(gs.part) + (int64_t)wg * L.E;
  int idx = 0;
#pragma unroll
  for (int I = 0; I < T; ++I)
#pragma unroll
    for (int J = I; J < T; ++J) {
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        // D layout of v_mfma_f64_16x16x4: lane l, register vv holds
        // D[l / 16 + 4 vv][l % 16].
        const int gi = 16 * I + rsub + 4 * vv;
        const int gj = 16 * J + c;
        if (gi < L.Wp && gj < L.Wp && (gi >> 2) <= (gj >> 2)) {
          const int e = tile_index(gi >> 2, gj >> 2, L.T4) * 16 + (gi & 3) * 4 + (gj & 3);
          out[e] = acc[idx][vv];
        }
      }
      ++idx;
    }
}

// ---------------------------------------------------------------------------
// Blocks of a reduction launch: G threads per Gram entry (reduce_groups), the
// 1024-thread block covering 1024 / G entries.  G depends on the segment's
// own size and precision only, so a segment's summation order does not
// depend on the others in a batched launch.

int reduce_blocks(int E, bool dd) {
  const int epb = 1024 / reduce_groups(E, dd);
  return (E + epb - 1) / epb;
}

template <bool DD>
__global__ void __launch_bounds__(1024) reduce_kernel(ReduceSeg one,
                                                      const ReduceSeg* __restrict__ tab) {
  __shared__ double sh[1024], sl[1024];
  const ReduceSeg rs = tab ? tab[blockIdx.y] : one;
  if (stopped(rs.stop, rs.pass)) return;
  const GramLayout& L = rs.L;
  const double BORTH_GLOBAL* __restrict__ part = gmem(rs.part);
  const int nwg = rs.nwg;
  double BORTH_GLOBAL* __restrict__ Ghi = gmem(rs.Ghi);
  double BORTH_GLOBAL* __restrict__ Glo = rs.Glo ? gmem(rs.Glo) : nullptr;
  const int E = L.E;
  const int G = reduce_groups(E, DD), EPB = 1024 / G;
  if ((int)blockIdx.x * EPB >= E) return;  // batched launch: a smaller segment
  const int el = threadIdx.x % EPB, g = threadIdx.x / EPB;
  const int e = blockIdx.x * EPB + el;
  double h = 0.0, l = 0.0;
  if (e < E) {
    // partials g, g + G, ...: loaded 16 (DD) or 32 at a time so that their
    // latencies overlap (the chain is latency-bound), added in index order
    constexpr int B = DD ? 16 : 32;
    for (int w0 = g; w0 < nwg; w0 += G * B) {
      double vh[B], vl[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int w = w0 + G * u;
        const int64_t off = (int64_t)(w < nwg ? w : 0) * E + e;
        vh[u] = DD ? part[2 * off] : part[off];
        vl[u] = DD ? part[2 * off + 1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (w0 + G * u >= nwg) break;
        if (DD) {
          const dd_t v = dd_add(dd_make(h, l), dd_make(vh[u], vl[u]));
          h = v.hi;
          l = v.lo;
        } else {
          h += vh[u];
        }
      }
    }
  }
  sh[threadIdx.x] = h;
  sl[threadIdx.x] = l;
  __syncthreads();
  if (g != 0 || e >= E) return;
  for (int q = 1; q < G; ++q) {
    if (DD) {
      const dd_t v = dd_add(dd_make(h, l), dd_make(sh[q * EPB + el], sl[q * EPB + el]));
      h = v.hi;
      l = v.lo;
    } else {
      h += sh[q * EPB + el];
    }
  }
  const int t = e >> 4, a = (e >> 2) & 3, b = e & 3;
  int ti, tj;
  decode_tile(t, L, ti, tj);
  const int pi = 4 * ti + a, pj = 4 * tj + b;
  if (pi > pj) return;  // lower half of a diagonal tile: written by its mirror
  auto logical = [&](int p) -> int {
    if (p < L.kyp) return p < L.ky ? p : -1;
    const int j = p - L.kyp;
    return j < L.k ? L.ky + j : -1;
  };
  const int li = logical(pi), lj = logical(pj);
  if (li < 0 || lj < 0) return;
  const int W = L.ky + L.k;
  Ghi[li * W + lj] = h;
  Ghi[lj * W + li] = h;
  if (Glo) {
    Glo[li * W + lj] = DD ? l : 0.0;
    Glo[lj * W + li] = DD ? l : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Host side.  A sweep's shape: the MFMA kernel (binary64, 16 <= Wp <= 80) or
// the VALU tile kernel (DD, or binary64 outside that range).

int gram_kind(const GramLayout& L, int mode, bool weighted) {
  const int W16 = (L.Wp + 15) / 16;
  return (mode == 0 && !weighted && L.ty == 0 && L.Wp >= 16 && W16 <= 5) ? 0 : 1;
}

// 256 threads (one 4x4 tile each; row phases when there are fewer than 128
// tiles) up to 256 tiles (Wp <= 88); wider blocks take 1024 threads.
int gram_tiles_threads(const GramLayout& L) { return L.ntiles <= 256 ? 256 : 1024; }

// The DD tile kernel at 256 threads accumulates on biased sums (see
// gram_tiles_kernel).
static bool gram_biased(int mode, const Src& s, int NT) {
  (void)s;
  return mode == 1 && NT == 256;
}

// Rows per panel of the tile kernel: nq load steps of NT / Wp rows, nq in
// 5..8 (biased DD: 9..16, at most 2 NT rows) chosen so that the S = NT /
// ntiles row phases get equal shares (the fewest idle rows per panel row).
static int gram_tiles_rows(const GramLayout& L, int NT, bool biased) {
  const int RS = NT / L.Wp, S = NT / L.ntiles;
  // biased: at most 2 NT rows (each thread stages the weights of two rows)
  const int q2 = RS > 0 ? 2 * NT / RS : 16;
  const int qmax = biased ? (q2 < 16 ? q2 : 16) : 8;
  const int qmin = qmax < 5 ? qmax : 5;
  if (RS < 1 || S < 1) return qmax * (RS > 0 ? RS : 1);
  auto cbits = [](int per) {
    int c = 0;
    while ((1 << c) < 2 * per + 1) ++c;
    return c;
  };
  // biased: the smallest bias exponent reachable with at least 8 rows per
  // thread (24 with a single row phase, whose panels are short), then the
  // estimated time: idle rows and one fold per panel (about 3 rows' work)
  const int pmin = S == 1 ? 24 : 8;
  int cmin = 99;
  if (biased)
    for (int nq = qmax; nq >= qmin; --nq) {
      const int per = (nq * RS + S - 1) / S;
      if (per >= pmin || nq == qmax) cmin = cbits(per) < cmin ? cbits(per) : cmin;
    }
  int best = qmax;
  double best_w = 1e9;
  for (int nq = qmax; nq >= (biased ? qmin : 5); --nq) {
    const int P = nq * RS;
    const int per = (P + S - 1) / S;
    if (biased && (cbits(per) > cmin || (per < pmin && nq != qmax))) continue;
    const double idle = (double)(per * S - P) / P;
    const double w = biased ? (1.0 + idle) * (1.0 + 3.0 / per) : idle;
    if (w < best_w - 1e-12) {
      best_w = w;
      best = nq;
    }
  }
  return best * RS;
}

// LDS of one DMA-sweep workgroup (two are resident per compute unit, which
// has 160 KiB).
constexpr size_t kDmaLdsBytes = 80 * 1024;

// LDS of a DMA-sweep workgroup with panels of P rows: the panel (rows of
// stride Wp + 2, then 1 KiB of slack) and the column maxima.
static size_t gram_dma_lds(const GramLayout& L, int P) {
  return (size_t)P * (L.Wp + 2) * sizeof(double) + 1024 + (size_t)L.Wp * sizeof(double);
}

// The DMA-staged DD sweep (gram_dd_dma_kernel): biased DD on 256 threads
// over 16-byte aligned rows of binary64 data without weights, or Dot2 sums
// (allow_dot2, a single block).
bool gram_dma_ok(const Src& s, const GramLayout& L, int mode, int NT, bool allow_dot2) {
  if (mode != 1 || NT != 256 || s.bw || (s.dot2 && !allow_dot2) || s.x_f32) return false;
  if (L.ntiles > 256) return false;
  // the shortest panel (4 rows per phase) must fit
  if (gram_dma_lds(L, 4 * (NT / L.ntiles)) > kDmaLdsBytes) return false;
  if ((reinterpret_cast<uintptr_t>(s.X) & 15) || (s.ldx & 1) || (L.k & 1)) return false;
  if (L.ky > 0 && ((reinterpret_cast<uintptr_t>(s.Y) & 15) || (s.ldy & 1) || (L.ky & 1)))
    return false;
  return true;
}

// Rows per panel of the DMA sweep: S phases of np rows each, np at most 40
// (the bias exponent cb then stays at most 7) and a multiple of 4, the
// tallest panel whose rows (stride Wp + 2, 1 KiB of slack) and column maxima
// fit the workgroup's LDS.  A panel's
// rounding error grows about as np 2^cb ~ 2 np^2 per thread and is averaged
// over the panels summed, so a short block (fewer than 16 panels' worth of
// rows at the full height) takes shorter panels.  Dot2 sums have no bias:
// up to 128 rows per phase.
static int gram_dma_rows(const GramLayout& L, int S, int64_t m, bool dot2 = false) {
  int np = dot2 ? 128 : 40;
  while (np > 4 && gram_dma_lds(L, S * np) > kDmaLdsBytes) np -= 4;
  const int64_t short_np = m / (16 * (int64_t)S);
  if (short_np < np) np = short_np < 4 ? 4 : (int)(short_np & ~(int64_t)3);
  return S * np;
}

int64_t gram_units(const Src& s, const GramLayout& L, int mode, int NT, bool allow_dot2) {
  if (gram_kind(L, mode, s.bw != nullptr) == 0) return (s.m + 3) / 4;
  const int P = gram_dma_ok(s, L, mode, NT, allow_dot2)
                    ? gram_dma_rows(L, NT / L.ntiles, s.m, s.dot2 != 0)
                    : gram_tiles_rows(L, NT, gram_biased(mode, s, NT));
  return (s.m + P - 1) / P;
}

int gram_max_wg(const Src& s, const GramLayout& L, int mode, int NT, bool allow_dot2) {
  const int64_t u = gram_units(s, L, mode, NT, allow_dot2);
  const int64_t need = gram_kind(L, mode, s.bw != nullptr) == 0 ? (u + 3) / 4 : u;
  return (int)(need < 1 ? 1 : (need > (1 << 20) ? (1 << 20) : need));
}

bool gram_seg(const Src& s, const GramLayout& L, int mode, int NT, double* part, int wg0,
              int nwg, GramSeg* out, size_t* shmem, bool allow_dot2) {
  GramSeg g;
  g.s = s;
  g.L = L;
  g.part = part;
  g.wg0 = wg0;
  g.nwg = nwg;
  g.nunits = gram_units(s, L, mode, NT, allow_dot2);
  g.P = 0;
  g.S = 0;
  *shmem = 0;
  if (gram_kind(L, mode, s.bw != nullptr) == 1 && gram_dma_ok(s, L, mode, NT, allow_dot2)) {
    g.S = NT / L.ntiles;
    if (g.S < 1) return false;
    g.P = gram_dma_rows(L, g.S, s.m, s.dot2 != 0);
    g.nunits = (s.m + g.P - 1) / g.P;
    // panel rows, column maxima, and slack for the spare lanes of the last
    // transfer instruction (a wave writes 64 chunks of 16 bytes)
    const size_t panel = gram_dma_lds(L, g.P);
    const size_t redn = g.S > 1 ? (size_t)L.E * 2 * sizeof(double) : 0;
    *shmem = panel > redn ? panel : redn;
    if (*shmem > kDmaLdsBytes) return false;
  } else if (gram_kind(L, mode, s.bw != nullptr) == 1) {
    g.S = NT / L.ntiles;
    if (g.S < 1 || NT / L.Wp < 1) return false;
    g.P = gram_tiles_rows(L, NT, gram_biased(mode, s, NT));
    g.nunits = (s.m + g.P - 1) / g.P;
    // biased DD (256 threads): two column-maxima buffers after the panel
    const int panel = g.P * (L.Wp + 2) + (gram_biased(mode, s, NT) ? 2 * (L.Wp + 1) : 0);
    const int redn = g.S > 1 ? L.E * (mode ? 2 : 1) : 0;  // one phase: no LDS reduction
    *shmem = sizeof(double) * (size_t)(panel > redn ? panel : redn);
  }
  *out = g;
  return true;
}

hipError_t launch_gram_segs(int kind, int mode, int NT_or_T, size_t shmem, int grid,
                            const GramSeg& one, const GramSeg* tab, const int* wg2seg,
                            hipStream_t st) {
  if (grid < 1) return hipSuccess;
  const bool b = tab != nullptr;
#define BORTH_MFMA(T, U)                                                                       \
  do {                                                                                         \
    if (b)                                                                                     \
      hipLaunchKernelGGL((gram_mfma_kernel<T, U, true>), dim3(grid), dim3(256), 0, st, one, tab, wg2seg); \
    else                                                                                       \
      hipLaunchKernelGGL((gram_mfma_kernel<T, U, false>), dim3(grid), dim3(256), 0, st, one, tab, wg2seg); \
  } while (0)
#define BORTH_TILES(D, N)                                                                      \
  do {                                                                                         \
    if (b)                                                                                     \
      hipLaunchKernelGGL((gram_tiles_kernel<D, N, true, false>), dim3(grid), dim3(N), shmem, st, one, tab, wg2seg); \
    else if (one.s.bw)                                                                         \
      hipLaunchKernelGGL((gram_tiles_kernel<D, N, false, true>), dim3(grid), dim3(N), shmem, st, one, tab, wg2seg); \
    else                                                                                       \
      hipLaunchKernelGGL((gram_tiles_kernel<D, N, false, false>), dim3(grid), dim3(N), shmem, st, one, tab, wg2seg); \
  } while (0)
  if (kind == 0) {
    switch (NT_or_T) {
      case 1: BORTH_MFMA(1, 16); break;
      case 2: BORTH_MFMA(2, 8); break;
      case 3: BORTH_MFMA(3, 2); break;
      case 4: BORTH_MFMA(4, 4); break;
      case 5: BORTH_MFMA(5, 2); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (NT_or_T == kGramDmaArg) {
    if (mode != 1) return hipErrorInvalidValue;
    static std::once_flag attr;
    std::call_once(attr, [] {
      const void* fns[5] = {(const void*)gram_dd_dma_kernel<false, false, 0>,
                            (const void*)gram_dd_dma_kernel<false, false, 32>,
                            (const void*)gram_dd_dma_kernel<false, true, 0>,
                            (const void*)gram_dd_dma_kernel<true, true, 0>,
                            (const void*)gram_dd_dma_kernel<false, true, 0, true>};
      for (const void* f : fns)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDmaLdsBytes);
    });
    // a batched launch takes the Y-capable kernel (its segments may differ;
    // their sums are biased); a single block with Dot2 sums the Dot2
    // instance; 32 columns without Y: the instance with the row layout
    // built in
    if (b)
      hipLaunchKernelGGL((gram_dd_dma_kernel<true, true, 0>), dim3(grid), dim3(256), shmem, st, one, tab, wg2seg);
    else if (one.s.dot2)
      hipLaunchKernelGGL((gram_dd_dma_kernel<false, true, 0, true>), dim3(grid), dim3(256), shmem, st, one, tab, wg2seg);
    else if (one.L.ky > 0)
      hipLaunchKernelGGL((gram_dd_dma_kernel<false, true, 0>), dim3(grid), dim3(256), shmem, st, one, tab, wg2seg);
    else if (one.L.Wp == 32 && one.L.ntiles == 36 && one.S == 256 / 36)
      hipLaunchKernelGGL((gram_dd_dma_kernel<false, false, 32>), dim3(grid), dim3(256), shmem, st, one, tab, wg2seg);
    else
      hipLaunchKernelGGL((gram_dd_dma_kernel<false, false, 0>), dim3(grid), dim3(256), shmem, st, one, tab, wg2seg);
  } else if (NT_or_T == 256) {
    if (mode == 1) BORTH_TILES(true, 256); else BORTH_TILES(false, 256);
  } else if (NT_or_T == 1024) {
    if (mode == 1) BORTH_TILES(true, 1024); else BORTH_TILES(false, 1024);
  } else {
    return hipErrorInvalidValue;
  }
#undef BORTH_MFMA
#undef BORTH_TILES
  return hipGetLastError();
}

// Workgroups of the tile kernel resident on the device at once, from the
// occupancy of the kernel instance (cached per device and shape).
int gram_tiles_resident(int mode, int NT, size_t shmem) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, size_t>, int> cache;
  const auto key = std::make_tuple(dev, mode, NT, shmem);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e;
  if (NT == kGramDmaArg)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gram_dd_dma_kernel<false, false, 32>, 256, shmem);
  else if (NT == 256)
    e = mode ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gram_tiles_kernel<true, 256, false, false>, 256, shmem)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gram_tiles_kernel<false, 256, false, false>, 256, shmem);
  else
    e = mode ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gram_tiles_kernel<true, 1024, false, false>, 1024, shmem)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gram_tiles_kernel<false, 1024, false, false>, 1024, shmem);
  if (e != hipSuccess || per < 1) return 0;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = per * cus;
  return per * cus;
}

hipError_t launch_gram(const Src& s, const GramLayout& L, int mode, double* partials,
                       int64_t cap, int* nwg_out, const TuneGram& tune, hipStream_t st) {
  if (s.bw && s.x_f32) return hipErrorInvalidValue;
  if (mode == 0 && !s.bw && !s.x_f32 && L.ty == 0 && L.Wp <= 8) {
    // narrow binary64 block: the row kernel, a few rows per lane in flight
    const int64_t want = (s.m + 256 * 4 * 4 - 1) / (256 * 4 * 4);  // >= 4 trips per lane
    int nwg = tune.nwg > 0 ? tune.nwg : 1024;
    if (nwg > want) nwg = (int)(want > 0 ? want : 1);
    if ((int64_t)nwg * L.E > cap) return hipErrorInvalidValue;
    GramSeg g;
    g.s = s;
    g.L = L;
    g.part = partials;
    g.nunits = s.m;
    g.P = g.S = 0;
    g.wg0 = 0;
    g.nwg = nwg;
    *nwg_out = nwg;
    if (L.Wp == 4)
      hipLaunchKernelGGL((gram_rows_kernel<4, 0>), dim3(nwg), dim3(256), 0, st, g);
    else if (L.kyp == 0)
      hipLaunchKernelGGL((gram_rows_kernel<8, 0>), dim3(nwg), dim3(256), 0, st, g);
    else
      hipLaunchKernelGGL((gram_rows_kernel<8, 4>), dim3(nwg), dim3(256), 0, st, g);
    return hipGetLastError();
  }
  const int kind = gram_kind(L, mode, s.bw != nullptr);
  const int NT = kind == 0 ? 256 : gram_tiles_threads(L);
  const bool dma = kind == 1 && gram_dma_ok(s, L, mode, NT, true);
  int nwg = tune.nwg > 0 ? tune.nwg : 1024;
  if (tune.nwg <= 0 && kind == 1) {
    // ALU-bound tile kernel: two full rounds of resident workgroups (measured
    // best on the 4M x 32 DD Gram: 1536 against 1024 or 2048)
    GramSeg g0;
    size_t sh0 = 0;
    if (gram_seg(s, L, mode, NT, partials, 0, 1, &g0, &sh0, true)) {
      const int r = gram_tiles_resident(mode, dma ? kGramDmaArg : NT, sh0);
      if (r > 0) nwg = 2 * r;
    }
    const int64_t fit = cap / ((int64_t)L.E * (mode ? 2 : 1));  // partial slots available
    if (nwg > fit) nwg = (int)(fit > 0 ? fit : 1);
  }
  const int mx = gram_max_wg(s, L, mode, NT, true);
  if (nwg > mx) nwg = mx;
  if ((int64_t)nwg * L.E * (mode ? 2 : 1) > cap) return hipErrorInvalidValue;
  GramSeg g;
  size_t shmem = 0;
  if (!gram_seg(s, L, mode, NT, partials, 0, nwg, &g, &shmem, true)) return hipErrorInvalidValue;
  const int arg = kind == 0 ? (L.Wp + 15) / 16 : (dma ? kGramDmaArg : NT);
  *nwg_out = nwg;
  return launch_gram_segs(kind, mode, arg, shmem, nwg, g, nullptr, nullptr, st);
}

hipError_t launch_reduce_segs(int mode, int nb, int nseg, const ReduceSeg& one,
                              const ReduceSeg* tab, hipStream_t st) {
  if (nb < 1 || nseg < 1) return hipSuccess;
  if (mode == 1)
    hipLaunchKernelGGL(reduce_kernel<true>, dim3(nb, nseg), dim3(1024), 0, st, one, tab);
  else
    hipLaunchKernelGGL(reduce_kernel<false>, dim3(nb, nseg), dim3(1024), 0, st, one, tab);
  return hipGetLastError();
}

hipError_t launch_reduce(const GramLayout& L, int mode, const double* partials, int nwg,
                         double* G_hi, double* G_lo, hipStream_t st, const int* stop, int pass) {
  ReduceSeg r{L, partials, nwg, G_hi, G_lo, stop, pass};
  return launch_reduce_segs(mode, reduce_blocks(L.E, mode == 1), 1, r, nullptr, st);
}

// DD Gram of [Y | X] for X = X_hi + X_lo (both binary64 words given), from
// the DD Grams A of [Y | X_hi], B of [X_hi | X_lo] and C of [Y | X_lo]
// (unpadded, row stride = width): G_YY = A_YY, G_YX = A_YX + C_YX and
// G_XX = B_hh + B_hl + B_lh + B_ll, DD additions, written over A.
__global__ void gram_dd_combine_kernel(int ky, int k, double* Ahi, double* Alo,
                                       const double* Bhi, const double* Blo, const double* Chi,
                                       const double* Clo) {
  const int W = ky + k, e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= W * W) return;
  const int i = e / W, j = e % W;
  if (i < ky && j < ky) return;
  dd_t v;
  if (i >= ky && j >= ky) {
    const int a = i - ky, b = j - ky, WB = 2 * k;
    auto g = [&](int r, int c) { return dd_make(Bhi[r * WB + c], Blo[r * WB + c]); };
    v = dd_add(dd_add(g(a, b), g(a, k + b)), dd_add(g(k + a, b), g(k + a, k + b)));
  } else {
    v = dd_add(dd_make(Ahi[e], Alo[e]), dd_make(Chi[e], Clo[e]));
  }
  Ahi[e] = v.hi;
  Alo[e] = v.lo;
}

hipError_t launch_gram_dd_combine(int ky, int k, double* Ahi, double* Alo, const double* Bhi,
                                  const double* Blo, const double* Chi, const double* Clo,
                                  hipStream_t st) {
  const int n = (ky + k) * (ky + k);
  hipLaunchKernelGGL(gram_dd_combine_kernel, dim3((n + 255) / 256), dim3(256), 0, st, ky, k, Ahi,
                     Alo, Bhi, Blo, Chi, Clo);
  return hipGetLastError();
}

__global__ void fill_int_kernel(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace borth
