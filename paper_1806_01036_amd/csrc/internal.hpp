// Internal interfaces between the C-ABI layer (borth.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace borth {

// Global-memory view of a pointer.  Kernel segments are read from tables in
// device memory, so the compiler cannot infer the address space of the
// pointers they hold; without this cast their loads become flat accesses,
// which share the LDS wait counter and serialize prefetches with LDS traffic.
#define BORTH_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T BORTH_GLOBAL* gmem(T* p) {
  return (T BORTH_GLOBAL*)p;
}

// Layout of a per-workgroup partial Gram: the upper triangle of the padded
// Wp x Wp matrix (Wp = kyp + kp, a multiple of 4) split into 4x4 tiles
// (ti <= tj) enumerated row by row; entry e = tile * 16 + a * 4 + b holds
// G[4 ti + a][4 tj + b].  Column c < kyp of the padded matrix is column c of
// Y (valid if c < ky); column kyp + j is column j of X (valid if j < k).
struct GramLayout {
  int ky, kyp;  // Y columns and their padding to a multiple of 4
  int k, kp;    // X columns and their padding
  int Wp;       // kyp + kp
  int T4;       // Wp / 4
  int ntiles;   // T4 (T4 + 1) / 2
  int E;        // ntiles * 16
  int ty;       // first tile column computed: 0, or kyp / 4 for the columns of X only
};

GramLayout make_layout(int ky, int k, int kp_min);
// The tiles of [Y | X]^T X only (Y^T Y left out): the Gram sweep of a pass
// whose Y^T Y is already known.  Tiles (ti, tj), ti <= tj, tj >= kyp / 4, in
// row-major order.
GramLayout make_layout_xcols(int ky, int k, int kp_min);

// Source block for a sweep: [Y | X] rows.
struct Src {
  const double* Y;
  int64_t ldy;
  const void* X;
  int64_t ldx;
  int x_f32;  // X is fp32
  int64_t m;
  // Diagonal of B for a B-weighted Gram sweep [Y | X]^T B [Y | X] (m
  // entries), or null (B = I).  Only the VALU tile kernel takes weights.
  const double* bw = nullptr;
  // Iterated scheme: the kernels of pass `pass` do nothing once *stop is
  // non-zero and <= pass (set by an earlier pass's factor), or null.
  const int* stop = nullptr;
  int pass = 0;
  // DD tile sweeps: accumulate with Dot2 instead of the biased sums.
  int dot2 = 0;
};

// True when a kernel of pass `pass` is to be skipped (uniform per launch).
__host__ __device__ inline bool stopped(const int* stop, int pass) {
  return stop && stop[0] != 0 && pass >= stop[0];
}

struct TuneGram {
  int nwg;    // workgroups of the sweep (0 = automatic)
  int rows;   // rows per LDS panel / per wave-step (0 = automatic)
};

// ---- launchers (all enqueue on `st`, return hipError_t) -------------------
//
// Every sweep kernel can cover several independent blocks in one launch:
// block b owns workgroups [wg0, wg0 + nwg) of the grid and streams its own
// rows with that many workgroups.  A single-block launch passes its segment
// by value (tab == nullptr, wg0 = 0, nwg = grid size); a batched launch
// passes a device table of segments and a workgroup -> segment map.

// One block of a Gram sweep.
struct GramSeg {
  Src s;
  GramLayout L;
  double* part;    // nwg partials of E (FP64) or 2E (DD) doubles
  int64_t nunits;  // row panels (tile kernel) or 4-row groups (MFMA kernel)
  int P, S;        // tile kernel: rows per panel, row phases
  int wg0, nwg;
};

// Gram sweep over [Y | X]: writes nwg partials (FP64: E doubles each, DD: 2E).
// mode: 0 = FP64, 1 = DD.  Returns the number of partials in *nwg_out.
hipError_t launch_gram(const Src& s, const GramLayout& L, int mode, double* partials,
                       int64_t partial_cap_doubles, int* nwg_out, const TuneGram& tune,
                       hipStream_t st);
// Pieces of launch_gram for the batched driver.
int gram_kind(const GramLayout& L, int mode, bool weighted = false);  // 0 MFMA (binary64), 1 VALU tiles
int gram_tiles_threads(const GramLayout& L);   // 256 or 1024
// The tile sweep of a DD Gram staged by direct global-to-LDS transfers
// (biased DD, 256 threads, 16-byte aligned rows); launch_gram_segs takes
// kGramDmaArg as its thread argument for it.
// allow_dot2: Dot2 sums (s.dot2) too -- a single block's launch only (the
// batched and persistent launches run the biased sums).
bool gram_dma_ok(const Src& s, const GramLayout& L, int mode, int NT, bool allow_dot2 = false);
constexpr int kGramDmaArg = 257;
int gram_max_wg(const Src& s, const GramLayout& L, int mode, int NT, bool allow_dot2 = false);
bool gram_seg(const Src& s, const GramLayout& L, int mode, int NT, double* part, int wg0,
              int nwg, GramSeg* out, size_t* shmem, bool allow_dot2 = false);
// kind 0: NT_or_T = column blocks (Wp / 16, rounded up); kind 1: threads
// (256 or 1024), or kGramDmaArg.
hipError_t launch_gram_segs(int kind, int mode, int NT_or_T, size_t shmem, int grid,
                            const GramSeg& one, const GramSeg* tab, const int* wg2seg,
                            hipStream_t st);

// Split-BF16 Gram of an fp32 X (k <= 64, no Y): FP64 partials (E per WG).
hipError_t launch_gram_split(const Src& s, const GramLayout& L, double* partials,
                             int64_t partial_cap_doubles, int* nwg_out, const TuneGram& tune,
                             hipStream_t st);

// Reduce nwg partials (fixed order) into G_hi / G_lo, unpadded W x W with
// W = ky + k (ld = W).  mode 1 = DD partials.
struct ReduceSeg {
  GramLayout L;
  const double* part;
  int nwg;
  double* Ghi;
  double* Glo;
  const int* stop = nullptr;  // as in Src
  int pass = 0;
};
hipError_t launch_reduce(const GramLayout& L, int mode, const double* partials, int nwg,
                         double* G_hi, double* G_lo, hipStream_t st, const int* stop = nullptr,
                         int pass = 0);
// DD Gram of [Y | X] with X = X_hi + X_lo: from the DD Grams A of [Y | X_hi],
// B of [X_hi | X_lo] and C of [Y | X_lo] (unpadded), written over A.
hipError_t launch_gram_dd_combine(int ky, int k, double* Ahi, double* Alo, const double* Bhi,
                                  const double* Blo, const double* Chi, const double* Clo,
                                  hipStream_t st);
// Blocks (grid.x) of the reduction of a Gram with E entries (DD or binary64).
int reduce_blocks(int E, bool dd);
// nseg segments (grid.y); nb = the largest reduce_blocks(L.E, dd) among them.
hipError_t launch_reduce_segs(int mode, int nb, int nseg, const ReduceSeg& one,
                              const ReduceSeg* tab, hipStream_t st);

// k x k factorization, one workgroup.
struct FactorArgs {
  int ky, k, kp;            // kp: padded width of the Z / C outputs
  const double* G_hi;       // (ky + k)^2
  const double* G_lo;       // may be null
  int dd;                   // DD arithmetic
  int fact;                 // 0 Cholesky, 1 SVQB
  double shift_rel;         // > 0: add shift_rel * trace(M)
  int pass;                 // 0-based; pass 0 initializes the totals
  double* Zp;               // kp x kp (zero padded), binary64 hi words
  double* Cp;               // ky x kp  (this pass's C, rounded, zero padded)
  double* Rtot;             // 2 * k * k  (DD totals, hi then lo)
  double* Ctot;             // 2 * ky * k
  int* status;              // [code, pass, pivot, passes_run]
  double* R_out;            // optional final outputs (binary64)
  double* C_out;
  double* Z_out;            // optional unpadded Z (k x k)
  double* Rp_out;           // optional this-pass R (k x k)
  double* conv;             // optional: ||C_p||_F and ||R_p - I||_F of this pass
  // optional: a condition estimate of the projected block, max R_ii / min R_ii
  // (Cholesky) or sqrt(lambda_max / lambda_min) of M (SVQB, lifted eigenvalues)
  double* kappa;
  // DD update (Cholesky in DD only): the low words of Z_p and of the
  // projection coefficients, which are then D = 2C - S C (C corrected to
  // first order for Y^T Y != I) instead of C, in C_p and in the totals.
  double* Zplo;             // kp x kp, or null
  double* Cplo;             // ky x kp, or null (set together with Zplo)
  // SVQB: keep only the eigenpairs above k u lambda_max (stable order),
  // Z = U_r L_r^{-1/2}, R = L_r^{1/2} U_r^T; the rank goes to status[4].
  int rank_reveal;
  // Iterated scheme: skip when stopped(stop, pass); after a breakdown, or
  // (with conv) once both norms are <= stop_eps, set *stop = pass + 1.
  int* stop;
  double stop_eps;
  // SVQB without rank revelation, optional: a status word that keeps the
  // largest number of eigenvalues one pass lifted to its floor
  int* lifted;
};
hipError_t launch_factor(const FactorArgs& a, hipStream_t st);
// One workgroup per entry of the device table `tab` (n entries, all with
// k <= kmax and the same dd / fact); `one` describes the widest entry.
hipError_t launch_factor_table(const FactorArgs& one, const FactorArgs* tab, int n, hipStream_t st);

// Update sweep: rows of [Y | S] where S is X (pass 1) or Q_1; stage 1
// computes T = (S - Y C1) Z1; with two_stage, T = (T - Y C2) Z2.  The
// result is written to Q (if Q != null) and/or its Gram partials (if
// partials != null, FP64 entries): of [Y | T] (gram_with_y, ky <= 16, layout
// make_layout(ky, k, K)) or of T alone (layout make_layout(0, k, K)).
struct UpdateArgs {
  int gram_with_y;
  Src src;
  // Stage s computes T = (S - Y C_s) Z_s: Z_s kp x kp, C_s ky x kp
  // (row-major, zero padded beyond k).
  const double* C1; const double* Z1;
  const double* C2; const double* Z2;
  const double* C1lo; const double* Z1lo;  // DD stage 1 (narrow kernel only), or null
  int two_stage;
  int dense;                           // Z dense (SVQB)
  double* Q; int64_t ldq;
  double* Qlo;                         // narrow DD update: low words of Q (ldq), or null
  const double* Xlo;                   // narrow DD update: low words of X (ldx), or null
  double* partials; int64_t partial_cap_doubles;
  int gram_xcols;                      // narrow fused Gram: [Y | T]^T T only
  int gram_dd;                         //   ... in DD
  const double* bw;                    //   ... B-weighted (diagonal of B), or null
  int nwg;                             // out: partials written
  GramLayout glayout;                  // out: layout of those partials
};
hipError_t launch_update(UpdateArgs& a, const GramLayout& L, const TuneGram& tune,
                         hipStream_t st);

// Device-side argument block of the update kernels (one block's segment).
struct UpdDev {
  const double* Y;
  int64_t ldy;
  const void* X;
  int64_t ldx;
  int64_t m;
  int ky, kyp, k;  // kyp: ky rounded up to a multiple of 4 (selects the Y class)
  int gE;          // entries per partial of the fused Gram
  int zbase;       // 0 (passed at run time on purpose)
  int dense;
  double* Q;
  int64_t ldq;
  double* Qlo;  // DD update: the DD result's low words (ldq), or null
  const double* Xlo;  // DD update: low words of a DD input X (ldx), or null
  double* part;
  int64_t npanels;
  const double* C1;  // stage coefficients (ky x K C, K x K Z, zero padded)
  const double* Z1;
  const double* C2;
  const double* Z2;
  const double* C1lo;  // low words of C1 and Z1: DD arithmetic (narrow or DD kernel), or null
  const double* Z1lo;
  const double* bw;    // diagonal of B for the narrow kernel's fused Gram, or null
  const int* stop;     // as in Src
  int pass;
  int wg0, nwg;
};
// Kernel class of an update launch.
struct UpdClass {
  int K;       // padded width 4, 8, 16, 32, 64
  int KYP;     // Y class: 0, 16 or 64
  int two;     // second stage
  int gr;      // 0 no Gram, 1 Gram of T, 2 Gram of [Y | T]
  int f32;     // X stored as fp32
  int dma = 0; // panels by direct transfers (update_dma_ok); the same for every block of a launch
};
// Whether an update sweep over these rows can take its panels by direct
// global-to-LDS transfers: padded width 16 or 32 with ky <= 16 (binary64,
// 16-byte aligned rows of X and Y, even ldx, ldy, k and ky), or padded width
// 64 with ky <= 16 in one stage (binary64, the same conditions; or fp32 X
// without Y, 16-byte aligned rows, ldx and k multiples of 4).
bool update_dma_ok(const UpdDev& d, int K, int KYP, bool f32, bool two);
// Narrow blocks (k <= 8, ky <= 64), single stage, no fused Gram: the VALU
// stream kernel of update_narrow.hip.  kp: row stride of C and Z.
bool update_narrow_ok(int k, int ky, int kp);
hipError_t launch_update_narrow(const UpdDev& d, int kp, hipStream_t st);
// DD update with a DD result for 8 < k <= 64 (update_dd.hip): the same
// arithmetic as the narrow kernel's DD branch; needs Q, Qlo, C1, Z1, C1lo,
// Z1lo; single stage, no fused Gram.
bool update_dd_ok(int k, int ky, int kp);
hipError_t launch_update_dd(const UpdDev& d, int kp, hipStream_t st);
// The same sweep with the next pass's Gram columns [Y | T]^T T written as
// partials (binary64, or DD when mode = 1) in the layout G =
// make_layout_xcols(ky, k, 4), one per workgroup, at most max_wg of them;
// *nwg = partials written.  Needs ky + k <= 64 and Y dense with ky even.
bool update_narrow_gram_ok(const UpdDev& d, int kp);
hipError_t launch_update_narrow_gram(const UpdDev& d, int kp, int mode, const GramLayout& G,
                                     int64_t max_wg, int* nwg, hipStream_t st);
// One per padded width K (separate translation units, compiled in parallel).
hipError_t launch_update_k4(const UpdClass&, int grid, const UpdDev&, const UpdDev*, const int*, hipStream_t);
hipError_t launch_update_k8(const UpdClass&, int grid, const UpdDev&, const UpdDev*, const int*, hipStream_t);
hipError_t launch_update_k16(const UpdClass&, int grid, const UpdDev&, const UpdDev*, const int*, hipStream_t);
hipError_t launch_update_k32(const UpdClass&, int grid, const UpdDev&, const UpdDev*, const int*, hipStream_t);
hipError_t launch_update_k64(const UpdClass&, int grid, const UpdDev&, const UpdDev*, const int*, hipStream_t);
hipError_t launch_update_class(const UpdClass&, int grid, const UpdDev& one, const UpdDev* tab,
                               const int* wg2seg, hipStream_t st);
int update_waves(int K, int KYP, bool dma = false);  // waves per workgroup of a single-stage class
int update_rows(int K, int KYP);   // rows per wave panel
// Layout of the fused Gram of an update sweep (of [Y | T] with Y padded to
// 16 columns when with_y, else of T).
GramLayout update_gram_layout(int ky, int k, int K, bool with_y);

// Fill helper (graph-safe replacement for hipMemsetAsync).
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st);

}  // namespace borth
