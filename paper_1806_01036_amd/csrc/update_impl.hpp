// Basis update sweep (TSMM), the product of the projected block with Z
// (Sec. 4.2), with the phase-I projection folded in:  T = (S - Y C) Z per
// row, S = X (first pass) or Q_1 (later passes), the subtraction first (as
// the paper orders it: when S lies close to span(Y), S Z and Y C Z are much
// larger than T and would cancel).  Optionally a second stage
// T = (T - Y C_2) Z_2 follows (CholQR2 with Q_1 recomputed instead of stored),
// and the Gram matrix of [Y | T] (or of T) needed by the next pass is
// accumulated from the values just computed (the fusion of operations that
// Sec. 4.2 uses to save memory traffic).
//
// The product is a dense contraction with a tiny right factor, so it runs
// on the matrix cores (v_mfma_f64_16x16x4):
//  * each wave streams its own panels of [Y | S] (64 rows; 16 for K = 64),
//    with no workgroup barrier in the loop: coalesced global loads -> LDS
//    (row stride KYP + K + 2 doubles, compile-time, so all offsets are
//    immediates);
//  * Z and -C are the B operands (lane l holds Z[4 s + l / 16][16 J + l % 16]):
//    in registers for the whole kernel for K <= 32, in LDS shared by the
//    workgroup for K = 64; the A operands (lane l: S[row l % 16][col 4 s +
//    l / 16]) are read from LDS;
//  * a workgroup streams the rows of one block; a batched launch covers many
//    blocks, each owning a range of the grid's workgroups (UpdDev table);
//  * the result tile (lane l, register v: T[row l / 16 + 4 v][col 16 J +
//    l % 16]) is stored straight to global memory, and the same registers
//    are the operands of the fused Gram MFMA (4-row groups v), so T never
//    goes back through LDS unless a second stage needs it as an A operand.
// Each wave's Gram accumulators are summed in wave order at the end and
// written as one partial per workgroup (same tile layout as the Gram sweep).
#pragma once
#include "dd.hpp"
#include "internal.hpp"

namespace borth {

namespace upd {

typedef double d4_t __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int tile_index_u(int ti, int tj, int T4) {
  return ti * T4 - (ti * (ti - 1)) / 2 + (tj - ti);
}

// Orders this wave's LDS accesses across its lanes (LDS instructions of one
// wave execute in order; the fences keep the compiler from reordering them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Widths K >= 64 keep the B operands (Z, W) in LDS, shared by the
// workgroup's waves, and stream 16-row panels: their operands would not fit
// the register file next to the fused Gram accumulators, and 64-row panels
// of [Y | X] would leave fewer than one wave per SIMD under the LDS budget.
__host__ __device__ constexpr bool upd_zl(int K) { return K >= 64; }
// Rows per wave panel: 16 at K >= 64, and at K = 32 with Y columns (two
// 32-row buffers of [Y | S] per wave would leave 1.5 waves per SIMD under
// the LDS budget; 16-row ones allow 2); 32 otherwise.
__host__ __device__ constexpr int upd_rows(int K, int KYP) {
  return (upd_zl(K) || (K == 32 && KYP > 0)) ? 16 : 32;
}
__host__ __device__ constexpr int upd_zs(int K) { return K + 2; }  // LDS row stride of Z / W
// Panels brought in by direct global-to-LDS transfers, so that the next
// panel's rows are in flight while the current one is computed (16-byte
// aligned rows):
//  * K = 16, 32 with at most 16 Y columns (binary64): two panel buffers per
//    wave, the next panel lands in the other one;
//  * K = 64 with at most 16 Y columns, single stage (binary64 rows; fp32
//    rows without Y): one buffer per wave; the panel's projection is done
//    and its A operands are read into registers first, then the next
//    panel's transfer overwrites the buffer during the product.
__host__ __device__ constexpr bool upd_dma_class(int K, int KYP) {
  return (K >= 16 && K <= 32 && KYP <= 16) || (K == 64 && KYP <= 16);
}
__host__ __device__ constexpr int upd_pbufs(int K, bool dma) { return dma ? (upd_zl(K) ? 1 : 2) : 1; }
// Row stride (elements) of a panel in LDS: [Y | S] converted to binary64
// with two padding columns; fp32 rows taken by the transfers stay fp32 (four
// padding columns keep rows 16-byte aligned).
__host__ __device__ constexpr int upd_prow(int K, int KYP, bool dma, bool f32) {
  return (dma && f32) ? K + 4 : KYP + K + 2;
}
// LDS doubles of one panel buffer.
__host__ __device__ constexpr int upd_panel_doubles(int K, int KYP, bool dma, bool f32) {
  return (dma && f32) ? upd_rows(K, KYP) * upd_prow(K, KYP, dma, f32) / 2
                      : upd_rows(K, KYP) * upd_prow(K, KYP, dma, f32);
}

// LDS bytes of a workgroup with nw waves (its panel buffers plus the shared
// Z / W operands of each stage when they live in LDS).
inline long upd_lds_bytes(int K, int KYP, int nw, int nst = 1, bool dma = false, bool f32 = false) {
  const long zreg = upd_zl(K) ? (long)nst * (K + KYP) * upd_zs(K) : 0;
  return 8L * (zreg + (long)nw * upd_pbufs(K, dma) * upd_panel_doubles(K, KYP, dma, f32));
}

// Waves per workgroup (1..8): the most resident waves per CU under the 160 KB
// of LDS, at most 8 (2 per SIMD); larger workgroups preferred, except that
// at K = 32 and 64 two workgroups of four waves are taken over one of eight
// when both fit (measured 3 % faster on the K = 32 sweeps and 2-4 % on the
// K = 64 ones: a workgroup's start and its partial-sum epilogue then
// overlap the other's stream).
inline int upd_waves(int K, int KYP, int nst = 1, bool dma = false, bool f32 = false) {
  int best = 1, best_waves = 0;
  for (int nw = 1; nw <= 8; nw <<= 1) {
    const long b = upd_lds_bytes(K, KYP, nw, nst, dma, f32);
    const int wgs = (int)((160L * 1024) / b);
    int waves = wgs * nw;
    if (waves > 8) waves = 8;
    if (wgs >= 1 && (waves > best_waves || (waves == best_waves && !(K >= 32 && best == 4)))) {
      best = nw;
      best_waves = waves;
    }
  }
  return best;
}

// GR: 0 = no Gram, 1 = Gram of T, 2 = Gram of [Y | T] (KYP = 16).
// DMA: the panels come in by direct transfers into two LDS buffers per wave
// (upd_dma_class; binary64 rows with X, Y 16-byte aligned, even ldx, ldy,
// k and ky).
//
// The body runs as workgroup bid of a launch (or a persistent workgroup's
// task) with NW streaming waves over the LDS at lds; further waves of the
// workgroup take part in its barriers only.
template <int K, int KYP, bool TWO, int GR, typename ST, bool BATCH, bool DMA>
__device__ __forceinline__ void update_body(const UpdDev& one, const UpdDev* __restrict__ tab,
                                            const int* __restrict__ wg2seg, int bid, int NW,
                                            double* lds) {
  const UpdDev a = BATCH ? tab[wg2seg[bid]] : one;
  if (stopped(a.stop, a.pass)) return;
  const int wg = bid - a.wg0;
  constexpr int S = KYP + K + 2;     // LDS row stride (doubles)
  constexpr int KC = (K + 15) / 16;  // 16-column blocks of T
  constexpr int KV = K < 16 ? K : 16;  // valid columns per T block
  constexpr int KS = K / 4;          // k-steps over S
  constexpr int YS = KYP / 4;        // k-steps over Y
  constexpr int NST = TWO ? 2 : 1;
  constexpr int YB = GR == 2 ? 1 : 0;  // Gram blocks taken by Y
  constexpr int GW = GR == 2 ? KYP + K : K;  // padded Gram width
  constexpr int T16 = YB + KC;       // Gram column blocks
  constexpr int NTL = T16 * (T16 + 1) / 2;
  constexpr int GT4 = GW / 4;
  constexpr int RPQ = 64 / K;        // panel rows per load step
  constexpr bool ZL = upd_zl(K);     // B operands in LDS
  constexpr int PR = upd_rows(K, KYP);  // rows per wave panel
  constexpr int NLQ = PR * K / 64;   // X load steps per panel
  constexpr int NLY = PR * KYP / 64; // Y load steps per panel
  constexpr int ZS = upd_zs(K);
  constexpr int ZST = (K + KYP) * ZS;  // LDS doubles of one stage's Z / W
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ky = a.ky;
  const int dense = a.dense;
  const int c16 = lane & 15, r4 = lane >> 4;
  // SB: K = 64 with transfers, one panel buffer per wave (upd_dma_class)
  constexpr bool SB = DMA && ZL;
  static_assert(!SB || (KYP <= 16 && !TWO && (KYP == 0 || sizeof(ST) == 8)),
                "single-buffer transfers: K = 64, one stage, binary64 rows with Y");
  static_assert(!DMA || SB || sizeof(ST) == 8, "double-buffer transfers: binary64 rows");
  constexpr int PD = upd_panel_doubles(K, KYP, DMA, sizeof(ST) == 4);
  double* zl = lds;
  double* pan0 = lds + (ZL ? NST * ZST : 0) + wave * upd_pbufs(K, DMA) * PD;
  double* pan = pan0;

  // B operands: in registers (lane l holds Z[4 s + l / 16][16 J + l % 16] and
  // -C[4 s + l / 16][16 J + l % 16]), or for ZL rows of Z then rows of -C in
  // LDS, read at the same positions.
  double zb[ZL ? 1 : NST][ZL ? 1 : KS][ZL ? 1 : KC];
  double wb[ZL ? 1 : NST][(ZL || YS == 0) ? 1 : YS][ZL ? 1 : KC];
  if (ZL) {
    for (int e = threadIdx.x; e < NST * (K + KYP) * K; e += blockDim.x) {
      const int st = e / ((K + KYP) * K);
      const int r = (e / K) % (K + KYP), c = e % K;
      const double BORTH_GLOBAL* __restrict__ Zg = gmem(st ? a.Z2 : a.Z1);
      const double BORTH_GLOBAL* __restrict__ Cg = gmem(st ? a.C2 : a.C1);
      zl[st * ZST + r * ZS + c] = r < K ? Zg[r * K + c] : ((r - K) < ky ? -Cg[(r - K) * K + c] : 0.0);
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const double BORTH_GLOBAL* __restrict__ Zg = gmem(st ? a.Z2 : a.Z1);
      const double BORTH_GLOBAL* __restrict__ Cg = gmem(st ? a.C2 : a.C1);
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int J = 0; J < KC; ++J) {
          const int col = 16 * J + c16;
          zb[ZL ? 0 : st][ZL ? 0 : s][ZL ? 0 : J] = col < K ? Zg[(4 * s + r4) * K + col] : 0.0;
        }
#pragma unroll
      for (int s = 0; s < YS; ++s)
#pragma unroll
        for (int J = 0; J < KC; ++J) {
          const int row = 4 * s + r4, col = 16 * J + c16;
          wb[ZL ? 0 : st][ZL ? 0 : s][ZL ? 0 : J] = (row < ky && col < K) ? -Cg[row * K + col] : 0.0;
        }
    }
  }
  auto bz = [&](int st, int s, int J) -> double {
    return ZL ? zl[st * ZST + (4 * s + r4) * ZS + 16 * J + c16] : zb[ZL ? 0 : st][ZL ? 0 : s][ZL ? 0 : J];
  };
  auto bw = [&](int st, int s, int J) -> double {
    return ZL ? zl[st * ZST + (K + 4 * s + r4) * ZS + 16 * J + c16] : wb[ZL ? 0 : st][ZL ? 0 : s][ZL ? 0 : J];
  };

  d4_t gacc[NTL];
#pragma unroll
  for (int i = 0; i < NTL; ++i) gacc[i] = d4_t{0.0, 0.0, 0.0, 0.0};

  const int64_t wstride = (int64_t)a.nwg * NW;
  const int64_t npanels = (a.m + PR - 1) / PR;
  int64_t pnl = wave < NW ? (int64_t)wg * NW + wave : npanels;
  constexpr int KY1 = KYP > 0 ? KYP : 1;
  constexpr int RY = 64 / KY1;
  const int ry0 = lane / KY1, cy = lane % KY1;
  const int rx0 = lane / K, cx = lane % K;
  const bool cyin = cy < ky, cxin = cx < a.k;
  const int aoff = c16 * S + r4;  // A operand: row l % 16, column l / 16
  const int doff = r4 * S + c16;  // result layout: row l / 16, column l % 16
  // Direct transfers: chunk q = 64 i + lane (16 bytes) of a panel lands at
  // byte 16 q of the wave's buffer (row q / (S / 2), columns 2 (q % (S / 2))
  // and the next).  Chunks of padding columns and rows past m copy a valid
  // chunk of the row (or of the last row): padding columns meet zero rows of
  // Z and W and land in padded Gram entries; rows past m are zeroed before
  // use.
  constexpr int CPR = S / 2, NCH = PR * CPR, NDI = (NCH + 63) / 64;
  auto transfer = [&](int64_t p, double* buf) {
    const int64_t r0 = p * PR;
    const int64_t last = a.m - 1;
#pragma unroll
    for (int i = 0; i < NDI; ++i) {
      const int q = 64 * i + lane;
      if (i + 1 < NDI || q < NCH) {
        const int r = q / CPR, col = 2 * (q % CPR);
        int64_t row = r0 + r;
        row = row < last ? row : last;
        const double BORTH_GLOBAL* src;
        if (KYP > 0 && col < KYP)
          src = gmem(a.Y) + row * a.ldy + (col + 1 < ky ? col : 0);
        else
          src = gmem((const double*)a.X) + row * a.ldx + (col - KYP + 1 < a.k ? col - KYP : 0);
        __builtin_amdgcn_global_load_lds((const void BORTH_GLOBAL*)src,
                                         (void __attribute__((address_space(3)))*)(buf + 128 * i), 16, 0, 0);
      }
    }
  };
  if constexpr (SB) {
    // Chunk q (16 bytes) of a panel lands at byte 16 q of the wave's buffer:
    // row q / CPR, elements EPC (q % CPR) and on; padding chunks and rows past
    // m copy a valid chunk (as above).
    constexpr int EPC = 16 / (int)sizeof(ST);
    constexpr int RS = upd_prow(K, KYP, true, sizeof(ST) == 4);
    constexpr int CPR = RS / EPC, NCH1 = PR * CPR, NDI1 = (NCH1 + 63) / 64;
    // with Y and a fused Gram: the next transfer starts after the product
    constexpr bool LATE = YS > 0 && GR > 0;
    ST* pst = (ST*)pan0;
    auto chunk = [&](int64_t r0, int i) {
      const int64_t last = a.m - 1;
      const int q = 64 * i + lane;
      if (i + 1 < NDI1 || q < NCH1) {
        const int r = q / CPR, col = EPC * (q % CPR);
        int64_t row = r0 + r;
        row = row < last ? row : last;
        const ST BORTH_GLOBAL* src;
        if (KYP > 0 && col < KYP) {
          src = (const ST BORTH_GLOBAL*)(gmem(a.Y) + row * a.ldy + (col + 1 < ky ? col : 0));
        } else {
          const int xc = col - KYP;
          src = gmem((const ST*)a.X) + row * a.ldx + (xc < a.k ? xc : 0);
        }
        __builtin_amdgcn_global_load_lds((const void BORTH_GLOBAL*)src,
                                         (void __attribute__((address_space(3)))*)((char*)pst + 1024 * i),
                                         16, 0, 0);
      }
    };
    auto transfer1 = [&](int64_t p) {
      if constexpr (KYP == 0) {
#pragma unroll
        for (int i = 0; i < NDI1; ++i) chunk(p * PR, i);
      } else {
        // rolled: unrolled, the chunks' lane offsets stay live across the
        // whole stream and push the Y variants into spills
#pragma unroll 1
        for (int i = 0; i < NDI1; ++i) chunk(p * PR, i);
      }
    };
    // T of a panel is stored at the start of the next panel, so that the
    // wait for a transfer (which also waits for the wave's stores) finds the
    // stores issued a panel's products earlier.
    auto store_t = [&](const d4_t* tt, int64_t r0, int nr) {
      if (!a.Q) return;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r4 + 4 * v;
        if (r < nr) {
          double BORTH_GLOBAL* qrow = gmem(a.Q) + (r0 + r) * a.ldq;
#pragma unroll
          for (int J = 0; J < KC; ++J)
            if (16 * J + c16 < a.k) qrow[16 * J + c16] = tt[J][v];
        }
      }
    };
    if (pnl < npanels) transfer1(pnl);
    d4_t tp[KC];
    int64_t prow0 = -1;
    int pnr = 0;
    while (pnl < npanels) {
      const int64_t row0 = pnl * PR;
      const int nrows = (int)(a.m - row0 < PR ? a.m - row0 : PR);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (nrows < PR) {
        for (int x = lane; x < (PR - nrows) * RS; x += 64) pst[nrows * RS + x] = (ST)0;
      }
      wave_lds_sync();
      // the previous panel's T (its registers are free before this panel's
      // operands are read)
      if (prow0 >= 0) store_t(tp, prow0, pnr);
      d4_t t[KC];
      double yv[4];  // the Y block in the result layout (Gram of [Y | T])
      if constexpr (YS > 0) {
        // projection in the paper's order, Xt = S - Y C accumulated onto S
        // on the matrix cores (result layout), then written back over S as
        // the A operand of the product with Z (binary64 panel, stride S)
        const double* pd = (const double*)pst;
#pragma unroll
        for (int J = 0; J < KC; ++J)
#pragma unroll
          for (int v = 0; v < 4; ++v) t[J][v] = pd[doff + 4 * v * S + KYP + 16 * J];
        double ay[YS > 0 ? YS : 1];
#pragma unroll
        for (int s = 0; s < YS; ++s) ay[s] = pd[aoff + 4 * s];
        if (YB) {
#pragma unroll
          for (int v = 0; v < 4; ++v) yv[v] = pd[doff + 4 * v * S];
        }
#pragma unroll
        for (int s = 0; s < YS; ++s)
#pragma unroll
          for (int J = 0; J < KC; ++J)
            t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[s], bw(0, s, J), t[J], 0, 0, 0);
        wave_lds_sync();
#pragma unroll
        for (int J = 0; J < KC; ++J)
#pragma unroll
          for (int v = 0; v < 4; ++v) ((double*)pst)[doff + 4 * v * S + KYP + 16 * J] = t[J][v];
        wave_lds_sync();
      }
#pragma unroll
      for (int J = 0; J < KC; ++J) t[J] = d4_t{0.0, 0.0, 0.0, 0.0};
      if constexpr (LATE) {
        // A operands read from the buffer as the product goes (all of them
        // in registers next to the [Y | T] Gram accumulators would spill);
        // the next transfer starts after the product, during the Gram
        const double* pd = (const double*)pst;
        if (dense) {
#pragma unroll 2
          for (int s = 0; s < KS; ++s) {
            const double av = pd[aoff + KYP + 4 * s];
#pragma unroll
            for (int J = 0; J < KC; ++J)
              t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bz(0, s, J), t[J], 0, 0, 0);
          }
        } else {
          // upper-triangular Z: k-step s meets column blocks J >= s / 4
#pragma unroll
          for (int s4 = 0; s4 < KC; ++s4) {
#pragma unroll 2
            for (int s = 4 * s4; s < 4 * s4 + 4; ++s) {
              const double av = pd[aoff + KYP + 4 * s];
#pragma unroll
              for (int J = s4; J < KC; ++J)
                t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bz(0, s, J), t[J], 0, 0, 0);
            }
          }
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (pnl + wstride < npanels) transfer1(pnl + wstride);
      } else {
      // the panel's A operands (lane l: row l % 16, column 4 s + l / 16)
      double ax[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) ax[s] = (double)pst[c16 * RS + KYP + 4 * s + r4];
      // the buffer is free once the reads are done: the next panel's
      // transfer runs during this panel's products
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      if (pnl + wstride < npanels) transfer1(pnl + wstride);
      if (dense) {
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
          for (int J = 0; J < KC; ++J)
            t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], bz(0, s, J), t[J], 0, 0, 0);
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
          for (int J = 0; J < KC; ++J)
            if (4 * s <= 16 * J + 15)
              t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], bz(0, s, J), t[J], 0, 0, 0);
      }
      }
      if (GR) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double op[T16];
          if (YB) op[0] = yv[v];
#pragma unroll
          for (int J = 0; J < KC; ++J) op[YB + J] = t[J][v];
          int idx = 0;
#pragma unroll
          for (int I = 0; I < T16; ++I)
#pragma unroll
            for (int J = I; J < T16; ++J) {
              gacc[idx] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[I], op[J], gacc[idx], 0, 0, 0);
              ++idx;
            }
        }
      }
#pragma unroll
      for (int J = 0; J < KC; ++J) tp[J] = t[J];
      prow0 = row0;
      pnr = nrows;
      pnl += wstride;
    }
    if (prow0 >= 0) store_t(tp, prow0, pnr);
  }
  if (DMA && !SB && pnl < npanels) transfer(pnl, pan0);
  int cur = 0;
  while (!SB && pnl < npanels) {
    const int64_t row0 = pnl * PR;
    const int nrows = (int)(a.m - row0 < PR ? a.m - row0 : PR);
    wave_lds_sync();  // this wave's reads of its previous panel are done
    if (DMA) {
      pan = pan0 + cur * PR * S;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      if (nrows < PR) {
        for (int x = lane; x < (PR - nrows) * S; x += 64) pan[nrows * S + x] = 0.0;
      }
      wave_lds_sync();
      // the next panel's rows fly while this one is computed
      if (pnl + wstride < npanels) transfer(pnl + wstride, pan0 + (cur ^ 1) * PR * S);
      cur ^= 1;
    } else {
    // 1. [Y | S] rows -> LDS (zero outside m, ky, k).  Loads are
    // unconditional (rows clamped to m - 1, columns to 0) so that they issue
    // back to back; out-of-range values are replaced by zero afterwards.
    if (KYP > 0) {
      const int cyc = cyin ? cy : 0;
#pragma unroll
      for (int q = 0; q < NLY; ++q) {
        const int r = ry0 + q * RY;
        const int64_t row = row0 + (r < nrows ? r : nrows - 1);
        const double v = gmem(a.Y)[row * a.ldy + cyc];
        pan[r * S + cy] = (r < nrows && cyin) ? v : 0.0;
      }
    }
    {
      const int cxc = cxin ? cx : 0;
      if (nrows == PR) {
        const ST BORTH_GLOBAL* xp = gmem((const ST*)a.X) + (row0 + rx0) * a.ldx + cxc;
        double v[NLQ];
#pragma unroll
        for (int q = 0; q < NLQ; ++q) v[q] = (double)xp[(int64_t)q * RPQ * a.ldx];
#pragma unroll
        for (int q = 0; q < NLQ; ++q) pan[(rx0 + q * RPQ) * S + KYP + cx] = cxin ? v[q] : 0.0;
      } else {
#pragma unroll
        for (int q = 0; q < NLQ; ++q) {
          const int r = rx0 + q * RPQ;
          const int64_t row = row0 + (r < nrows ? r : nrows - 1);
          const double v = (double)gmem((const ST*)a.X)[row * a.ldx + cxc];
          pan[r * S + KYP + cx] = (r < nrows && cxin) ? v : 0.0;
        }
      }
    }
    wave_lds_sync();
    }
#pragma unroll 1
    for (int b = 0; b < PR / 16; ++b) {  // 16-row blocks
      double* pb = pan + 16 * b * S;
      d4_t t[KC];
#pragma unroll
      for (int st = 0; st < NST; ++st) {
        // 1. projection in the paper's order: Xt = S_st - Y C_st, accumulated
        //    on the matrix cores into S_st itself (result layout: lane l,
        //    register v holds row l / 16 + 4 v, column 16 J + l % 16), so the
        //    subtraction is one rounding per product term on top of S; then
        //    Xt goes back to LDS as the A operand of the product with Z.
        //    S_0 is the panel, S_1 the previous stage's result (registers).
        if (YS > 0) {
#pragma unroll
          for (int J = 0; J < KC; ++J)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (st == 0) t[J][v] = pb[doff + 4 * v * S + KYP + 16 * J];
          // the A operands of every k-step first, so that the matrix-core
          // chain issues back to back
          double ay[YS > 0 ? YS : 1];
#pragma unroll
          for (int s = 0; s < YS; ++s) ay[s] = pb[aoff + 4 * s];
#pragma unroll
          for (int s = 0; s < YS; ++s) {
#pragma unroll
            for (int J = 0; J < KC; ++J)
              t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[s], bw(st, s, J), t[J], 0, 0, 0);
          }
        }
        if (YS > 0 || st > 0) {
          wave_lds_sync();
#pragma unroll
          for (int J = 0; J < KC; ++J)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (16 * J + c16 < K) pb[doff + 4 * v * S + KYP + 16 * J] = t[J][v];
          wave_lds_sync();
        }
        // 2. T = Xt Z_st
#pragma unroll
        for (int J = 0; J < KC; ++J) t[J] = d4_t{0.0, 0.0, 0.0, 0.0};
        if (ZL) {
          // with the B operands in LDS, a partly unrolled k loop bounds the
          // operand loads in flight (the registers are needed by the Gram)
#pragma unroll 2
          for (int s = 0; s < KS; ++s) {
            const double av = pb[aoff + KYP + 4 * s];
#pragma unroll
            for (int J = 0; J < KC; ++J)
              if (dense || 4 * s <= 16 * J + 15)  // upper-triangular Z: skip zero blocks
                t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bz(st, s, J), t[J], 0, 0, 0);
          }
        } else {
          // all A operands first, then the chain: upper-triangular Z (the
          // zero blocks skipped) or dense Z, one uniform branch
          double ax[KS];
#pragma unroll
          for (int s = 0; s < KS; ++s) ax[s] = pb[aoff + KYP + 4 * s];
          if (dense) {
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
              for (int J = 0; J < KC; ++J)
                t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], bz(st, s, J), t[J], 0, 0, 0);
          } else {
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
              for (int J = 0; J < KC; ++J)
                if (4 * s <= 16 * J + 15)
                  t[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], bz(st, s, J), t[J], 0, 0, 0);
          }
        }
      }
      // store T rows 16 b + l / 16 + 4 v, columns 16 J + l % 16
      if (a.Q) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * b + r4 + 4 * v;
          if (r < nrows) {
            double BORTH_GLOBAL* qrow = gmem(a.Q) + (row0 + r) * a.ldq;
#pragma unroll
            for (int J = 0; J < KC; ++J)
              if (16 * J + c16 < a.k) qrow[16 * J + c16] = t[J][v];
          }
        }
      }
      // fused Gram: the result registers are operands for the 4-row groups v
      if (GR) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double op[T16];
          if (YB) op[0] = pb[doff + 4 * v * S];  // Y block (layout of the result)
#pragma unroll
          for (int J = 0; J < KC; ++J) op[YB + J] = t[J][v];
          int idx = 0;
#pragma unroll
          for (int I = 0; I < T16; ++I)
#pragma unroll
            for (int J = I; J < T16; ++J) {
              gacc[idx] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[I], op[J], gacc[idx], 0, 0, 0);
              ++idx;
            }
        }
      }
    }
    pnl += wstride;
  }

  if (!GR) return;
  // Sum the waves' accumulators in wave order into wave 0, write the partial
  // (the buffer overlays the panels and Z / W: the first barrier below
  // orders it after every wave's last panel).
  double* red = lds;
  for (int w = 1; w < NW; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) red[(i * 4 + vv) * 64 + lane] = gacc[i][vv];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) gacc[i][vv] += red[(i * 4 + vv) * 64 + lane];
    }
  }
  if (wave != 0) return;
  // Gram block B, in-block index x -> padded Gram column (Y: 0..15, then the
  // K columns of T); -1 for padding columns of a T block narrower than 16.
  auto pcol = [&](int B, int x) -> int {
    if (YB && B == 0) return x;
    return x < KV ? YB * KYP + 16 * (B - YB) + x : -1;
  };
  double BORTH_GLOBAL* out = gmem(a.part) + (int64_t)wg * a.gE;
  int idx = 0;
#pragma unroll
  for (int I = 0; I < T16; ++I)
#pragma unroll
    for (int J = I; J < T16; ++J) {
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        // v_mfma_f64_16x16x4 D layout: lane l, register vv -> D[l/16 + 4 vv][l%16]
        const int pi = pcol(I, r4 + 4 * vv), pj = pcol(J, c16);
        if (pi >= 0 && pj >= 0 && (pi >> 2) <= (pj >> 2)) {
          const int e = tile_index_u(pi >> 2, pj >> 2, GT4) * 16 + (pi & 3) * 4 + (pj & 3);
          out[e] = gacc[idx][vv];
        }
      }
      ++idx;
    }
}

template <int K, int KYP, bool TWO, int GR, typename ST, bool BATCH, bool DMA>
__global__ void __launch_bounds__(512) update_kernel(UpdDev one, const UpdDev* __restrict__ tab,
                                                     const int* __restrict__ wg2seg) {
  extern __shared__ double lds[];
  update_body<K, KYP, TWO, GR, ST, BATCH, DMA>(one, tab, wg2seg, (int)blockIdx.x,
                                               (int)(blockDim.x >> 6), lds);
}

template <int K, int KYP, bool TWO, int GR, typename ST>
hipError_t launch_upd_t(int grid, const UpdDev& one, const UpdDev* tab, const int* map,
                        hipStream_t st, bool dma) {
  constexpr bool DC = upd_dma_class(K, KYP) && (upd_zl(K) ? !TWO : sizeof(ST) == 8);
  dma = dma && DC;
  constexpr bool F32 = sizeof(ST) == 4;
  const int NW = upd_waves(K, KYP, TWO ? 2 : 1, dma, F32);
  constexpr int KC = (K + 15) / 16;
  constexpr int T16 = (GR == 2 ? 1 : 0) + KC;
  const size_t red = GR ? sizeof(double) * T16 * (T16 + 1) / 2 * 4 * 64 : 0;
  const size_t lb = (size_t)upd_lds_bytes(K, KYP, NW, TWO ? 2 : 1, dma, F32);
  const size_t shmem = lb > red ? lb : red;
  if (dma) {
    if (tab)
      hipLaunchKernelGGL((update_kernel<K, KYP, TWO, GR, ST, true, DC>), dim3(grid), dim3(64 * NW),
                         shmem, st, one, tab, map);
    else
      hipLaunchKernelGGL((update_kernel<K, KYP, TWO, GR, ST, false, DC>), dim3(grid), dim3(64 * NW),
                         shmem, st, one, tab, map);
  } else if (tab) {
    hipLaunchKernelGGL((update_kernel<K, KYP, TWO, GR, ST, true, false>), dim3(grid), dim3(64 * NW),
                       shmem, st, one, tab, map);
  } else {
    hipLaunchKernelGGL((update_kernel<K, KYP, TWO, GR, ST, false, false>), dim3(grid), dim3(64 * NW),
                       shmem, st, one, tab, map);
  }
  return hipGetLastError();
}

// Dispatch on the Y padding class, the two-stage flag and the Gram kind.
template <int K>
hipError_t launch_upd_k(const UpdClass& c, int grid, const UpdDev& one, const UpdDev* tab,
                        const int* map, hipStream_t st) {
  if (grid < 1) return hipSuccess;
  if (c.f32) {
    if (c.two || c.KYP || c.gr == 2) return hipErrorInvalidValue;
    return c.gr ? launch_upd_t<K, 0, false, 1, float>(grid, one, tab, map, st, c.dma)
                : launch_upd_t<K, 0, false, 0, float>(grid, one, tab, map, st, c.dma);
  }
  if (c.KYP == 0) {
    if (c.gr == 2) return hipErrorInvalidValue;
    if (c.two)
      return c.gr ? launch_upd_t<K, 0, true, 1, double>(grid, one, tab, map, st, c.dma)
                  : launch_upd_t<K, 0, true, 0, double>(grid, one, tab, map, st, c.dma);
    return c.gr ? launch_upd_t<K, 0, false, 1, double>(grid, one, tab, map, st, c.dma)
                : launch_upd_t<K, 0, false, 0, double>(grid, one, tab, map, st, c.dma);
  }
  if (c.KYP == 16) {
    if (c.two) {
      if (c.gr == 2) return launch_upd_t<K, 16, true, 2, double>(grid, one, tab, map, st, c.dma);
      if (c.gr == 1) return launch_upd_t<K, 16, true, 1, double>(grid, one, tab, map, st, c.dma);
      return launch_upd_t<K, 16, true, 0, double>(grid, one, tab, map, st, c.dma);
    }
    if (c.gr == 2) return launch_upd_t<K, 16, false, 2, double>(grid, one, tab, map, st, c.dma);
    if (c.gr == 1) return launch_upd_t<K, 16, false, 1, double>(grid, one, tab, map, st, c.dma);
    return launch_upd_t<K, 16, false, 0, double>(grid, one, tab, map, st, c.dma);
  }
  // 16 < ky <= 64: single stage; a fused Gram covers T only
  if (c.KYP != 64 || c.two || c.gr == 2) return hipErrorInvalidValue;
  return c.gr ? launch_upd_t<K, 64, false, 1, double>(grid, one, tab, map, st, c.dma)
              : launch_upd_t<K, 64, false, 0, double>(grid, one, tab, map, st, c.dma);
}

}  // namespace upd
}  // namespace borth
