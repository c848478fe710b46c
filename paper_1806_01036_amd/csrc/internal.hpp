// Internal interfaces between the C-ABI layer (borth.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace borth {

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
};

GramLayout make_layout(int ky, int k, int kp_min);

// Source block for a sweep: [Y | X] rows.
struct Src {
  const double* Y;
  int64_t ldy;
  const void* X;
  int64_t ldx;
  int x_f32;  // X is fp32
  int64_t m;
};

struct TuneGram {
  int nwg;    // workgroups of the sweep (0 = automatic)
  int rows;   // rows per LDS panel / per wave-step (0 = automatic)
};

// ---- launchers (all enqueue on `st`, return hipError_t) -------------------

// Gram sweep over [Y | X]: writes nwg partials (FP64: E doubles each, DD: 2E).
// mode: 0 = FP64, 1 = DD.  Returns the number of partials in *nwg_out.
hipError_t launch_gram(const Src& s, const GramLayout& L, int mode, double* partials,
                       int64_t partial_cap_doubles, int* nwg_out, const TuneGram& tune,
                       hipStream_t st);

// Split-BF16 Gram of an fp32 X (k <= 64, no Y): FP64 partials (E per WG).
hipError_t launch_gram_split(const Src& s, const GramLayout& L, double* partials,
                             int64_t partial_cap_doubles, int* nwg_out, const TuneGram& tune,
                             hipStream_t st);

// Reduce nwg partials (fixed order) into G_hi / G_lo, unpadded W x W with
// W = ky + k (ld = W).  mode 1 = DD partials.
hipError_t launch_reduce(const GramLayout& L, int mode, const double* partials, int nwg,
                         double* G_hi, double* G_lo, hipStream_t st);

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
  double* Cp;               // ky x kp  (hi words of this pass's C)
  double* Wp;               // ky x kp  W = -C Z (the update's Y coefficients)
  double* Rtot;             // 2 * k * k  (DD totals, hi then lo)
  double* Ctot;             // 2 * ky * k
  int* status;              // [code, pass, pivot, passes_run]
  double* R_out;            // optional final outputs (binary64)
  double* C_out;
  double* Z_out;            // optional unpadded Z (k x k)
  double* Rp_out;           // optional this-pass R (k x k)
};
hipError_t launch_factor(const FactorArgs& a, hipStream_t st);

// Update sweep: rows of [Y | S] where S is X (pass 1) or Q_1; stage 1
// computes T = (S - Y C1) Z1; with two_stage, T = (T - Y C2) Z2.  The
// result is written to Q (if Q != null) and/or its Gram partials (if
// partials != null, FP64 entries): of [Y | T] (gram_with_y, ky <= 16, layout
// make_layout(ky, k, K)) or of T alone (layout make_layout(0, k, K)).
struct UpdateArgs {
  int gram_with_y;
  Src src;
  // Stage s computes T = S Z_s + Y W_s with W_s = -C_s Z_s (== (S - Y C_s) Z_s):
  // Z_s kp x kp, W_s ky x kp (row-major, zero padded beyond k).
  const double* W1; const double* Z1;
  const double* W2; const double* Z2;
  int two_stage;
  int dense;                           // Z dense (SVQB)
  double* Q; int64_t ldq;
  double* partials; int64_t partial_cap_doubles;
  int nwg;                             // out: partials written
  GramLayout glayout;                  // out: layout of those partials
};
hipError_t launch_update(UpdateArgs& a, const GramLayout& L, const TuneGram& tune,
                         hipStream_t st);

// Device-side argument block of the update kernels.
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
  double* part;
  int64_t npanels;
};
// One per padded width K (separate translation units, compiled in parallel).
hipError_t launch_update_k4(const UpdDev&, const UpdateArgs&, int nwg, hipStream_t);
hipError_t launch_update_k8(const UpdDev&, const UpdateArgs&, int nwg, hipStream_t);
hipError_t launch_update_k16(const UpdDev&, const UpdateArgs&, int nwg, hipStream_t);
hipError_t launch_update_k32(const UpdDev&, const UpdateArgs&, int nwg, hipStream_t);
hipError_t launch_update_k64(const UpdDev&, const UpdateArgs&, int nwg, hipStream_t);

// W = -C Z (ky x kp, zero padded) for the public update entry point.
hipError_t launch_neg_cz(const double* C, const double* Z, double* W, int ky, int k, int kp,
                         hipStream_t st);

// Fill helper (graph-safe replacement for hipMemsetAsync).
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st);

// Batched path (one launch per phase over all blocks).
struct BatchDesc {
  // per block
  const double* X; int64_t ldx;
  const double* Y; int64_t ldy;
  double* Q; int64_t ldq;
  double* R; double* C;
  int64_t m;
  int k, kp, ky, kyp;
  int64_t panel0;    // first global panel index of this block
  int64_t npanels;
  int64_t part_off;  // offset (doubles) of this block's partial slots
  int nslots;        // partial slots of this block
  int64_t ws_off;    // offset (doubles) of this block's k x k workspace
};
struct BatchPlan {
  BatchDesc* d_desc;  // device array
  int nblocks;
  int64_t total_panels;
  int rows;           // rows per panel
  double* partials;
  double* ws;         // per-block small workspace
  int* status;        // 4 ints per block
  int gram_mode;      // 0 FP64, 1 DD for pass 1
  int passes;
  int project_each;
  double shift_rel;
};
hipError_t launch_batch_gram(const BatchPlan& p, int pass, hipStream_t st);
hipError_t launch_batch_factor(const BatchPlan& p, int pass, hipStream_t st);
hipError_t launch_batch_update(const BatchPlan& p, int pass, int last, hipStream_t st);
int64_t batch_ws_doubles_per_block();

}  // namespace borth
