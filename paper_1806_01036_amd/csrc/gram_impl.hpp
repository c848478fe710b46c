// Device code of the Gram sweeps shared by their kernels (gram.hip) and the
// persistent batched kernel (batch_persistent.hip): the tile-layout helpers
// and the bodies of the VALU tile sweep and of the DMA-staged DD sweep.  A
// body runs as workgroup bid of a launch (or as a persistent workgroup's
// task) over the dynamic LDS at the pointer it is given.
#pragma once
#include "dd.hpp"
#include "internal.hpp"

namespace borth {

// Tile t of the layout's enumeration -> (ti, tj): row ti holds the tiles
// tj = max(ti, ty) .. T4 - 1.
__device__ __forceinline__ void decode_tile(int t, const GramLayout& L, int& ti, int& tj) {
  int r = 0, base = 0;
  auto cnt = [&](int row) { return L.T4 - (row > L.ty ? row : L.ty); };
  while (t >= base + cnt(r)) {
    base += cnt(r);
    ++r;
  }
  ti = r;
  tj = (r > L.ty ? r : L.ty) + (t - base);
}

__device__ __forceinline__ int tile_index(int ti, int tj, int T4) {
  return ti * T4 - (ti * (ti - 1)) / 2 + (tj - ti);
}

// Element (row, c) of the padded [Y | X] block (zero outside; X binary64).
// The load is unconditional -- row clamped to m - 1, column to 0 -- so that
// consecutive fetches issue back to back; the zero is selected afterwards.
__device__ __forceinline__ double fetch(const Src& s, const GramLayout& L, int64_t row, int c) {
  const bool isy = c < L.kyp;
  const int j = c - L.kyp;
  const bool ok = row < s.m && (isy ? c < L.ky : j < L.k);
  const int64_t rc = row < s.m ? row : s.m - 1;
  const double BORTH_GLOBAL* p = isy ? gmem(s.Y) + rc * s.ldy + (c < L.ky ? c : 0)
                                     : gmem((const double*)s.X) + rc * s.ldx + (j < L.k ? j : 0);
  const double v = *p;
  return ok ? v : 0.0;
}

// ---------------------------------------------------------------------------
// VALU tile kernel (binary64 or DD).

// WB: rows weighted by the diagonal of B (s.bw): each product a_i (w b_j),
// with w b_j split exactly (TwoProduct) in DD mode.
template <bool DD, int NTB, bool BATCH, bool WB>
__device__ __forceinline__ void gram_tiles_body(const GramSeg& one, const GramSeg* __restrict__ tab,
                                                const int* __restrict__ wg2seg, int bid,
                                                double* lds) {
  const GramSeg g = BATCH ? tab[wg2seg[bid]] : one;
  const Src& s = g.s;
  if (stopped(s.stop, s.pass)) return;
  const GramLayout& L = g.L;
  const int P = g.P, S = g.S;
  const int64_t npanels = g.nunits;
  const int wg = bid - g.wg0, nwg = g.nwg;
  const int stride = L.Wp + 2;
  const int tid = threadIdx.x, NT = blockDim.x;
  const int nt = L.ntiles;
  const bool active = tid < nt * S;
  const int t = active ? tid % nt : 0;
  const int phase = active ? tid / nt : 0;
  int ti, tj;
  decode_tile(t, L, ti, tj);

  // BIAS (DD, 256 threads): each panel's sums are accumulated on top of a
  // power-of-two bias sigma > 2x the largest sum B the thread's rows of the
  // panel can reach (plus one product), so that the running value stays in
  // [sigma - B, sigma + B] and consecutive values are within a factor 1.5:
  // the rounded sum s' = fma(a, b, s) then gives the exact increment s' - s
  // (Sterbenz) and the exact rounding error a b - (s' - s) up to one final
  // rounding of at most u ulp(sigma) -- 4 instructions per product instead
  // of Dot2's 8.  sigma comes from the panel's column maxima (M_c < 2^E_c:
  // sigma = 2^(E_i + E_j + cb), 2^cb >= 2 x rows per thread + 1); at the end
  // of the panel the exact sum acs - sigma is added into the running total th
  // with TwoSum, its error and the panel's rounding errors go to acc, and
  // (th, acc) is renormalized so that acc stays below ulp(th).  The panel
  // height is chosen on the host for a small 2^cb (the rounding error per
  // product scales with sigma) and few idle rows.
  constexpr bool BIAS = DD && NTB == 256;
  // the caller may ask for Dot2 instead (uniform per launch); the weighted
  // sweep always runs biased (both loops in one kernel would not fit two
  // waves per SIMD)
  const bool biased = BIAS && (WB || !s.dot2);
  double acs[16], acc[16], th[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    acs[e] = 0.0;
    acc[e] = 0.0;
    th[e] = 0.0;
  }

  // Panel loads: thread t owns column lc = t % Wp and rows lr + q RS
  // (RS = NT / Wp rows per step, P = nq RS rows per panel, nq <= 8 chosen
  // on the host so that the S row phases split P evenly), so one pointer and
  // one stride per thread address all its loads.  The next panel's loads are
  // issued into registers before the current panel is processed, so HBM
  // latency overlaps the arithmetic.
  constexpr int NQ = BIAS ? 16 : 8;
  const int nq = P / (NT / L.Wp);
  const int RS = NT / L.Wp;
  const int lc = tid % L.Wp, lr = tid / L.Wp;
  const bool isy = lc < L.kyp;
  const bool ldr = lr < RS && (isy ? lc < L.ky : lc - L.kyp < L.k);
  const int64_t ld = isy ? s.ldy : s.ldx;
  // column clamped to a valid one; loads below are unconditional
  const double BORTH_GLOBAL* bd = isy ? gmem(s.Y) + (lc < L.ky ? lc : 0)
                                      : gmem((const double*)s.X) + (lc - L.kyp < L.k ? lc - L.kyp : 0);
  // The raw loaded values stay in pf until the panel is stored to LDS (the
  // zero for rows beyond m and padding columns is selected there), so the
  // wait for the loads falls after the arithmetic of the current panel.
  double pf[NQ];
  // WB: weights of panel rows tid and tid + NT (P <= 2 NT)
  double pfw[2] = {0.0, 0.0};
  const int64_t step = (int64_t)RS * ld;
  auto fetch_panel = [&](int64_t pnl) {
    if (WB) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = tid + h * NT;
        const int64_t rw = pnl * P + (t < P ? t : 0);
        pfw[h] = gmem(s.bw)[rw < s.m ? rw : s.m - 1];
      }
    }
    const int64_t row0 = pnl * P + lr;
    if ((pnl + 1) * P <= s.m) {
      // full panel (uniform branch): rows in range, pointer steps of RS rows
      const double BORTH_GLOBAL* p = bd + row0 * ld;
#pragma unroll
      for (int q = 0; q < NQ; ++q) pf[q] = p[(q < nq ? q : 0) * step];
    } else {
      const int64_t mlast = s.m - 1;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        // load steps beyond nq re-read the first row (a cache hit) and are dropped
        const int64_t row = row0 + (q < nq ? q : 0) * RS;
        pf[q] = bd[(row < s.m ? row : mlast) * ld];
      }
    }
  };
  // BIAS: per-column maxima of |V| over the panel (and, WB, of the weights
  // in slot Wp), as the bit patterns of non-negative doubles (ordered like
  // unsigned integers), two buffers of CW entries alternating between
  // panels; cb from the rows a thread takes per panel.
  unsigned long long* cmx = (unsigned long long*)(lds + P * stride);
  const int CW = L.Wp + 1;
  int cb = 0;
  if (BIAS) {
    const int np = (P + S - 1) / S;
    while ((1 << cb) < 2 * np + 1) ++cb;
    for (int x = tid; x < 2 * CW; x += NT) cmx[x] = 0ull;
  }
  int par = 0;
  fetch_panel(wg);
  for (int64_t pnl = wg; pnl < npanels; pnl += nwg, par ^= 1) {
    __syncthreads();
    if (lr < RS) {
      const int64_t row0 = pnl * P + lr;
      double mx = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (q < nq) {
          const double v = (ldr && row0 + q * RS < s.m) ? pf[q] : 0.0;
          lds[(lr + q * RS) * stride + lc] = v;
          if (BIAS) mx = fmax(mx, fabs(v));
        }
      if (BIAS) atomicMax(&cmx[par * CW + lc], (unsigned long long)__double_as_longlong(mx));
    }
    // the other buffer is free (its panel's readers passed the barrier above)
    if (BIAS)
      for (int x = tid; x < CW; x += NT) cmx[(par ^ 1) * CW + x] = 0ull;
    // the weight of each row sits in the spare column Wp of its LDS row
    if (WB) {
      double mw = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = tid + h * NT;
        if (t < P) {
          const double w = pnl * P + t < s.m ? pfw[h] : 0.0;
          lds[t * stride + L.Wp] = w;
          mw = fmax(mw, fabs(w));
        }
      }
      if (BIAS && tid < P) atomicMax(&cmx[par * CW + L.Wp], (unsigned long long)__double_as_longlong(mw));
    }
    __syncthreads();
    fetch_panel(pnl + nwg);
    if (biased && active) {
      // WB: |w b_j| <= M_w M_j with M_w <= 2^ew (ew = ceil(log2 M_w): 0 for
      // unit weights, which then take exactly the unweighted path's sigma)
      int ew = 0;
      if (WB) {
        const double mw = __longlong_as_double((long long)cmx[par * CW + L.Wp]);
        ew = __builtin_amdgcn_frexp_exp(mw);
        if (__builtin_amdgcn_frexp_mant(mw) == 0.5) --ew;
      }
      int ea[4], eb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ea[i] = __builtin_amdgcn_frexp_exp(__longlong_as_double((long long)cmx[par * CW + 4 * ti + i]));
        eb[i] = __builtin_amdgcn_frexp_exp(__longlong_as_double((long long)cmx[par * CW + 4 * tj + i])) + cb + ew;
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) acs[e] = __builtin_amdgcn_ldexp(1.0, ea[e / 4] + eb[e % 4]);
      // two rows per trip (the new sums alternate register sets, no copies);
      // one with weights, whose split products need the registers
      constexpr int UNR = WB ? 1 : 2;
#pragma unroll UNR
      for (int r = phase; r < P; r += S) {
        const double* row = lds + r * stride;
        double a[4], b[4], bl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = row[4 * ti + i];
          b[i] = row[4 * tj + i];
        }
        if (WB) {
          const double w = row[L.Wp];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double h = b[j] * w;
            bl[j] = __builtin_fma(b[j], w, -h);  // w b_j = h + bl exactly
            b[j] = h;
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int e = 4 * i + j;
            const double sn = __builtin_fma(a[i], b[j], acs[e]);
            const double d = sn - acs[e];  // exact
            acc[e] = acc[e] + __builtin_fma(a[i], b[j], -d);
            if (WB) acc[e] = __builtin_fma(a[i], bl[j], acc[e]);
            acs[e] = sn;
          }
      }
      // fold: th += acs - sigma (exact difference) with TwoSum.  sigma is
      // recomputed from the exponents (the empty asm keeps the compiler from
      // holding 16 sigmas in registers across the row loop instead).
#pragma unroll
      for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(ea[i]), "+v"(eb[i]));
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const double h = acs[e] - __builtin_amdgcn_ldexp(1.0, ea[e / 4] + eb[e % 4]);
        const dd_t t = two_sum(th[e], h);
        const dd_t n = fast_two_sum(t.hi, acc[e] + t.lo);
        th[e] = n.hi;
        acc[e] = n.lo;
      }
    } else if (active) {
#pragma unroll 2
      for (int r = phase; r < P; r += S) {
        const double* row = lds + r * stride;
        double a[4], b[4], bl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = row[4 * ti + i];
          b[i] = row[4 * tj + i];
          bl[i] = 0.0;
        }
        if (WB) {
          const double w = row[L.Wp];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double h = b[j] * w;
            bl[j] = DD ? __builtin_fma(b[j], w, -h) : 0.0;  // w b_j = h + bl exactly
            b[j] = h;
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (DD) {
              dot2_step(acs[4 * i + j], acc[4 * i + j], a[i], b[j]);
              if (WB) acc[4 * i + j] = __builtin_fma(a[i], bl[j], acc[4 * i + j]);
            } else {
              acs[4 * i + j] = __builtin_fma(a[i], b[j], acs[4 * i + j]);
            }
          }
      }
    }
  }

  const int E = L.E;
  if (S == 1) {
    // one row phase: each thread's tile is its part of the partial
    if (!active) return;
    double BORTH_GLOBAL* out = gmem(g.part) + (int64_t)wg * E * (DD ? 2 : 1);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      if (DD) {
        const dd_t v = dot2_finish(biased ? th[e] : acs[e], acc[e]);
        out[2 * (t * 16 + e)] = v.hi;
        out[2 * (t * 16 + e) + 1] = v.lo;
      } else {
        out[t * 16 + e] = acs[e];
      }
    }
    return;
  }
  // Combine the row phases in phase order in LDS (the threads of phase ph add
  // their tiles to the running sum, one phase per barrier), then write this
  // WG's partial.
  __syncthreads();
  double* red = lds;
  for (int ph = 0; ph < S; ++ph) {
    if (active && phase == ph) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int x = t * 16 + e;
        if (DD) {
          dd_t v = dot2_finish(biased ? th[e] : acs[e], acc[e]);
          if (ph > 0) v = dd_add(dd_make(red[2 * x], red[2 * x + 1]), v);
          red[2 * x] = v.hi;
          red[2 * x + 1] = v.lo;
        } else {
          red[x] = ph > 0 ? red[x] + acs[e] : acs[e];
        }
      }
    }
    __syncthreads();
  }
  double BORTH_GLOBAL* out = gmem(g.part) + (int64_t)wg * E * (DD ? 2 : 1);
  for (int x = tid; x < E * (DD ? 2 : 1); x += NT) out[x] = red[x];
}

// ---------------------------------------------------------------------------
// DD Gram with biased accumulation, row panels staged by direct
// global-to-LDS transfers (gfx950 global_load_lds_dwordx4).
//
// The same arithmetic as the biased path of gram_tiles_kernel (each thread
// owns a 4x4 tile and a row phase; each panel's sums run on a power-of-two
// bias from the panel's column maxima and are folded into a DD total at the
// panel's end), with the panel brought in differently: every 16-byte chunk
// of the panel's rows is copied from HBM straight into LDS by the memory
// unit, so no registers hold the panel on its way and no instructions store
// it.  That frees the registers the register-staged kernel spent on its
// prefetch and lets a panel be two to three times taller, so the fold, the
// bias set-up and the barriers are paid over more rows.  The panel's load
// latency is covered by the other workgroup resident on the compute unit
// (a second buffer per workgroup would halve the panel height within the
// same LDS, and the extra folds cost more than the overlap gains).
//
// Per panel: transfer (each wave issues its share of the chunks) while the
// previous panel's sums are folded -> wait, barrier -> rows past m zeroed,
// column maxima into LDS -> barrier -> tile sums on the bias -> barrier.
// The LDS row stride is Wp + 2 doubles (Wp / 2 + 1 chunks); the chunk after
// a row's Wp columns, and the chunks of the padding columns between Y and X
// or after X, are filled with a copy of a valid chunk of that row: they are
// read only into products that land in padded Gram entries, which the
// reduction drops.
//
// Needs 16-byte aligned rows: X and Y 16-byte aligned, even ldx, ldy, ky and
// k, binary64, no weights (host check gram_dma_ok).  HASY: the sweep has Y
// columns (ky > 0), so a chunk's source may be either matrix.  WPC > 0: the
// padded width is WPC and the row phases 256 / ntiles (checked on the host),
// so that the LDS offsets of a loop trip are immediates.  D2: Dot2 sums
// (the 8-instruction step of dd.hpp, as the tile kernel's Dot2 mode) in
// place of the biased ones -- no column maxima, no bias and no folds; the
// panel height is then set by the LDS alone.
template <bool BATCH, bool HASY, int WPC, bool D2 = false>
__device__ __forceinline__ void gram_dd_dma_body(const GramSeg& one, const GramSeg* __restrict__ tab,
                                                 const int* __restrict__ wg2seg, int bid,
                                                 double* lds_all) {
  // LDS: column maxima (Wp words of 8 bytes), then the panel (P rows of
  // Wp + 2 doubles), then 1 KiB of slack
  const GramSeg g = BATCH ? tab[wg2seg[bid]] : one;
  const Src& s = g.s;
  if (stopped(s.stop, s.pass)) return;
  const GramLayout& L = g.L;
  const int Wp = WPC > 0 ? WPC : L.Wp;
  const int T4 = Wp / 4;
  const int nt = WPC > 0 ? T4 * (T4 + 1) / 2 : L.ntiles;
  const int S = WPC > 0 ? 256 / nt : g.S;
  const int P = g.P;
  const int np = P / S;  // rows per thread and panel (P = S np, np a multiple of 4)
  const int64_t npanels = g.nunits;
  const int wg = bid - g.wg0, nwg = g.nwg;
  const int stride = Wp + 2, cpr = stride / 2;
  const int nchunks = P * cpr;
  const int tid = threadIdx.x, wave = tid >> 6;
  const bool active = tid < nt * S;
  const int t = active ? tid % nt : 0;
  const int phase = active ? tid / nt : 0;
  int ti, tj;
  decode_tile(t, L, ti, tj);
  int cb = 0;
  while ((1 << cb) < 2 * np + 1) ++cb;
  // column maxima of the panel as the high words of |x| (sign bit shifted
  // out): their maximum has the exponent field of the column maximum
  unsigned* cmx = (unsigned*)lds_all;
  double* lds = lds_all + Wp;

  double acs[16], acc[16], th[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    acs[e] = 0.0;
    acc[e] = 0.0;
    th[e] = 0.0;
  }
  const double BORTH_GLOBAL* Xg = gmem((const double*)s.X);
  const double BORTH_GLOBAL* Yg = gmem(s.Y);
  // maxima pass: thread -> (pair of data columns, row group), 16-byte reads
  const int mcp = Wp / 2;  // column pairs of a row
  const int mcol = tid % mcp, mgrp = tid / mcp, ngrp = 256 / mcp;
  // Transfer plan: chunk q = 256 i + tid of a panel lands at byte 16 q of
  // the panel in LDS (the LDS base of one instruction is uniform per wave).
  // Its source, relative to the panel's first row, is the same for every
  // full panel: off[i] doubles into X, or into Y where bit i of ymask is set.
  // Instructions i < nfull cover 256 chunks; one more covers the rest.
  constexpr int kMaxChunks = 20;  // P cpr <= 5120 (80 KiB of LDS)
  const int nfull = nchunks / 256, nci = (nchunks + 255) / 256;
  unsigned off[kMaxChunks];  // bytes
  unsigned ymask = 0u;
  // Within a row the chunks are permuted: slot h T4 + c (h = 0, 1) holds
  // columns 4 c + 2 h, 4 c + 2 h + 1 -- the first halves of the 4-column
  // groups, then the second halves -- so that the lanes of one LDS read,
  // which take the same half of up to eight different groups, fall into
  // different banks; slot 2 T4 is the padding chunk.
  auto slot_col = [&](int p) { return p < 2 * T4 ? 4 * (p % T4) + 2 * (p / T4) : Wp; };
  auto chunk_src = [&](int q, int& r, int& o) -> bool {
    r = q / cpr;
    const int col = slot_col(q - r * cpr);
    if (HASY && col + 1 < L.ky) {
      o = col;
      return true;
    }
    o = (col >= L.kyp && col - L.kyp + 1 < L.k) ? col - L.kyp : 0;
    return false;
  };
#pragma unroll
  for (int i = 0; i < kMaxChunks; ++i) {
    off[i] = 0u;
    const int q = 256 * i + tid;
    if (i < nci && q < nchunks) {
      int r, o;
      const bool y = chunk_src(q, r, o);
      off[i] = (unsigned)(((y ? (int64_t)r * s.ldy : (int64_t)r * s.ldx) + o) * 8);
      if (y) ymask |= 1u << i;
    }
  }
  // issues the transfers of panel pnl (rows past m: the last row again)
  auto transfer = [&](int64_t pnl) {
    const int64_t row0 = pnl * P;
    const int64_t rem = s.m - row0;
    const int rows = rem < P ? (int)rem : P;
    if (rows == P) {
      // uniform base + per-lane 32-bit byte offset (the saddr form)
      const char BORTH_GLOBAL* xb = (const char BORTH_GLOBAL*)(Xg + row0 * s.ldx);
      const char BORTH_GLOBAL* yb = HASY ? (const char BORTH_GLOBAL*)(Yg + row0 * s.ldy) : xb;
#pragma unroll
      for (int i = 0; i < kMaxChunks; ++i) {
        if (i < nfull || (i == nfull && i < nci && 256 * i + tid < nchunks)) {
          const char BORTH_GLOBAL* src = (HASY && ((ymask >> i) & 1u)) ? yb + off[i] : xb + off[i];
          __builtin_amdgcn_global_load_lds((const void BORTH_GLOBAL*)src,
                                           (void __attribute__((address_space(3)))*)(lds + 2 * (256 * i + 64 * wave)),
                                           16, 0, 0);
        }
      }
    } else {
      for (int q0 = 0; q0 < nchunks; q0 += 256) {
        const int q = q0 + tid;
        if (q < nchunks) {
          int r, o;
          const bool y = chunk_src(q, r, o);
          const int64_t row = row0 + (r < rows ? r : rows - 1);
          const double BORTH_GLOBAL* src = y ? Yg + row * s.ldy + o : Xg + row * s.ldx + o;
          __builtin_amdgcn_global_load_lds((const void BORTH_GLOBAL*)src,
                                           (void __attribute__((address_space(3)))*)(lds + 2 * (q0 + 64 * wave)),
                                           16, 0, 0);
        }
      }
    }
  };
  // sigma exponent of column c: E_c with M_c < 2^E_c (frexp exponent of a
  // normal maximum; a zero or subnormal maximum takes E_c = -1022)
  auto col_exp = [&](int c) {
    const unsigned h = cmx[c] >> 21;  // exponent field (the shift removed the sign)
    return (h > 0 ? (int)h : 1) - 1022;
  };

  // fold of the finished panel: its exact biased sums (acs - sigma) into
  // the DD totals (th, acc)
  int ea[4], eb[4];
  auto fold = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(ea[i]), "+v"(eb[i]));
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const double h = acs[e] - __builtin_amdgcn_ldexp(1.0, ea[e / 4] + eb[e % 4]);
      const dd_t tt = two_sum(th[e], h);
      const dd_t n = fast_two_sum(tt.hi, acc[e] + tt.lo);
      th[e] = n.hi;
      acc[e] = n.lo;
    }
  };

  bool folded = true;  // no panel's sums pending
  for (int64_t pnl = wg; pnl < npanels; pnl += nwg) {
    const int64_t rem = s.m - pnl * P;
    const int rows = rem < P ? (int)rem : P;
    // every thread has finished the previous panel (its sums and its reads
    // of the column maxima): this panel's transfers fly while that panel's
    // sums are folded
    __syncthreads();
    transfer(pnl);
    if constexpr (!D2) {
      if (!folded && active) fold();
      for (int x = tid; x < Wp; x += 256) cmx[x] = 0u;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (rows < P) {
      // last panel: rows past m (copies of the last row) become zeros
      for (int x = tid; x < (P - rows) * stride; x += 256) lds[rows * stride + x] = 0.0;
    }
    if (!D2 && mgrp < ngrp) {
      unsigned m0 = 0u, m1 = 0u;
#pragma unroll 4
      for (int r = mgrp; r < rows; r += ngrp) {
        const uint4 v = *(const uint4*)(lds + r * stride + 2 * mcol);
        m0 = max(m0, v.y << 1);
        m1 = max(m1, v.w << 1);
      }
      const int c0 = slot_col(mcol);
      atomicMax(&cmx[c0], m0);
      atomicMax(&cmx[c0 + 1], m1);
    }
    __syncthreads();
    if (active) {
      if constexpr (!D2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ea[i] = col_exp(4 * ti + i);
          eb[i] = col_exp(4 * tj + i) + cb;
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) acs[e] = __builtin_amdgcn_ldexp(1.0, ea[e / 4] + eb[e % 4]);
      }
      // One row at a time, the next row's operands read from LDS while this
      // row's products are summed (two register sets, A and B, alternate;
      // np is even).  Column 4 c + x of a row sits at double 2 c + x (x < 2)
      // or 2 T4 + 2 c + x - 2 (x >= 2) of its slots.
      const int rstep = S * stride;
      const double* pa = lds + phase * stride + 2 * ti;
      const double* pb = lds + phase * stride + 2 * tj;
      auto load_row = [&](double* a, double* b, int row) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int xo = x < 2 ? x : 2 * T4 + x - 2;
          a[x] = pa[row * rstep + xo];
          b[x] = pb[row * rstep + xo];
        }
      };
      // each of the four steps runs over eight sums before the next step,
      // so that neighbouring instructions are independent
      auto sum_row = [&](const double* a, const double* b) {
        if constexpr (D2) {
#pragma unroll
          for (int e = 0; e < 16; ++e) dot2_step(acs[e], acc[e], a[e / 4], b[e % 4]);
          return;
        }
#pragma unroll
        for (int g8 = 0; g8 < 16; g8 += 8) {
          double sn[8], d[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) sn[e] = __builtin_fma(a[(g8 + e) / 4], b[e % 4], acs[g8 + e]);
#pragma unroll
          for (int e = 0; e < 8; ++e) d[e] = sn[e] - acs[g8 + e];  // exact
#pragma unroll
          for (int e = 0; e < 8; ++e) d[e] = __builtin_fma(a[(g8 + e) / 4], b[e % 4], -d[e]);
#pragma unroll
          for (int e = 0; e < 8; ++e) acc[g8 + e] = acc[g8 + e] + d[e];
#pragma unroll
          for (int e = 0; e < 8; ++e) acs[g8 + e] = sn[e];
        }
      };
      // (the last step reads its own row again instead of a row past the
      // panel, which keeps the loop body free of branches)
      double ra[4], rb[4], qa[4], qb[4];
      load_row(ra, rb, 0);
      for (int i = 0; i < np; i += 2) {
        load_row(qa, qb, i + 1);
        sum_row(ra, rb);
        load_row(ra, rb, i + 2 < np ? i + 2 : i + 1);
        sum_row(qa, qb);
      }
    }
    folded = false;
  }
  if constexpr (!D2) {
    if (!folded && active) fold();
  }
  __syncthreads();

  const int E = L.E;
  if (S == 1) {
    if (!active) return;
    double BORTH_GLOBAL* out = gmem(g.part) + (int64_t)wg * E * 2;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const dd_t v = dot2_finish(D2 ? acs[e] : th[e], acc[e]);
      out[2 * (t * 16 + e)] = v.hi;
      out[2 * (t * 16 + e) + 1] = v.lo;
    }
    return;
  }
  // row phases combined in phase order in LDS, then this workgroup's partial
  double* red = lds_all;
  for (int ph = 0; ph < S; ++ph) {
    if (active && phase == ph) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int x = t * 16 + e;
        dd_t v = dot2_finish(D2 ? acs[e] : th[e], acc[e]);
        if (ph > 0) v = dd_add(dd_make(red[2 * x], red[2 * x + 1]), v);
        red[2 * x] = v.hi;
        red[2 * x + 1] = v.lo;
      }
    }
    __syncthreads();
  }
  double BORTH_GLOBAL* out = gmem(g.part) + (int64_t)wg * E * 2;
  for (int x = tid; x < E * 2; x += 256) out[x] = red[x];
}
// Partial sums per entry of the reduction: the reduction kernel's thread
// groups (G of them, G a function of E) each sum the partials g, g + G, ...
// in index order, and group 0 then adds groups 1 .. G - 1 in order.
// Threads per Gram entry of the reduction (a function of the segment's size
// and precision only): more of them spread the partials over more compute
// units; the groups' sums are then added one after another, which for DD
// sums costs more per group.
__host__ __device__ inline int reduce_groups(int E, bool dd) {
  return E <= 256 ? 64 : (E <= 1024 ? (dd ? 64 : 128) : 32);
}

// The whole reduction of one segment by one workgroup (any size), entry by
// entry in the same order of operations as reduce_kernel, so the two give
// the same bits; writes G (both triangles) like reduce_kernel.
template <bool DD>
__device__ __forceinline__ void reduce_segment_body(const ReduceSeg& rs) {
  const GramLayout& L = rs.L;
  const double BORTH_GLOBAL* __restrict__ part = gmem(rs.part);
  const int nwg = rs.nwg, E = L.E, G = reduce_groups(E, DD);
  double BORTH_GLOBAL* __restrict__ Ghi = gmem(rs.Ghi);
  double BORTH_GLOBAL* __restrict__ Glo = rs.Glo ? gmem(rs.Glo) : nullptr;
  const int W = L.ky + L.k;
  for (int e = (int)threadIdx.x; e < E; e += (int)blockDim.x) {
    double h = 0.0, l = 0.0;
    for (int g = 0; g < G; ++g) {
      double gh = 0.0, gl = 0.0;
      for (int w = g; w < nwg; w += G) {
        const int64_t off = (int64_t)w * E + e;
        if (DD) {
          const dd_t v = dd_add(dd_make(gh, gl), dd_make(part[2 * off], part[2 * off + 1]));
          gh = v.hi;
          gl = v.lo;
        } else {
          gh += part[off];
        }
      }
      if (g == 0) {
        h = gh;
        l = gl;
      } else if (DD) {
        const dd_t v = dd_add(dd_make(h, l), dd_make(gh, gl));
        h = v.hi;
        l = v.lo;
      } else {
        h += gh;
      }
    }
    const int t = e >> 4, a = (e >> 2) & 3, b = e & 3;
    int ti, tj;
    decode_tile(t, L, ti, tj);
    const int pi = 4 * ti + a, pj = 4 * tj + b;
    if (pi > pj) continue;  // lower half of a diagonal tile: written by its mirror
    auto logical = [&](int p) -> int {
      if (p < L.kyp) return p < L.ky ? p : -1;
      const int j = p - L.kyp;
      return j < L.k ? L.ky + j : -1;
    };
    const int li = logical(pi), lj = logical(pj);
    if (li < 0 || lj < 0) continue;
    Ghi[li * W + lj] = h;
    Ghi[lj * W + li] = h;
    if (Glo) {
      Glo[li * W + lj] = DD ? l : 0.0;
      Glo[lj * W + li] = DD ? l : 0.0;
    }
  }
}

}  // namespace borth
