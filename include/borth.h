/*
 * borth -- block orthonormalization of tall-skinny matrices on AMD MI355X
 * (gfx950).  C ABI.
 *
 * The operation (Sec. 4.2 of Alvermann et al., "Benefits from using mixed
 * precision computations in the ELPA-AEO and ESSEX-II eigensolver projects"):
 * given a block X (m x k) and optionally a locked orthonormal basis Y
 * (m x ky; the paper's W), phase I projects X against Y,
 *     C = Y^T X,    Xt = (I - Y Y^T) X = X - Y C,
 * and phase II orthonormalizes Xt by a k x k transform Z with Z^T M Z = I,
 * where M = Xt^T Xt is the Gram matrix:
 *     Cholesky (CholQR):  M = R^T R,  Z = R^{-1};
 *     SVQB:               M = U L U^T, Z = U L^{-1/2} U^T  (symmetric form);
 *     Q = Xt Z.
 * Repeating the two phases (Sec. 4.2) is offered as `passes` repetitions
 * (passes = 2 is CholQR2).  The Gram matrix of the first pass can be
 * accumulated in binary64, in double-double (DD, hi + lo; Sec. 4.2 carries
 * the Gram matrix and its factorization in extended precision), or as BF16
 * hi/lo split products on
 * the matrix cores (FP32 accumulation) followed by a shifted factorization;
 * later passes are binary64.  On success
 *     X = Y C + Q R,   Q^T Q = I,   Y^T Q = 0   (to working accuracy).
 *
 * Conventions for every entry point:
 *  - Matrices are row-major.  Element (i, j) of X is X[i * ldx + j];
 *    ld >= number of columns.  Small matrices (k x k, ky x k) are dense
 *    row-major with leading dimension equal to their column count.
 *  - X, Y, Q, R, C, G, Z are DEVICE pointers on the context's device, owned
 *    by the caller.  borth_opts, borth_info and borth_block arrays are HOST
 *    pointers.
 *  - All work is enqueued on the context's HIP stream and is asynchronous,
 *    except where a borth_info* is passed (then the call synchronizes the
 *    stream and fills it) or BORTH_FLAG_SYNC is set.
 *  - Argument errors return BORTH_ERR_ARG before anything is enqueued.
 *    HIP failures return BORTH_ERR_HIP; borth_last_error() has the text.
 *  - The context owns its workspace (partial Gram sums, k x k factors,
 *    status words, cached graphs); it grows on demand and is released by
 *    borth_destroy.  One context per host thread; calls on one context are
 *    serialized by its stream.
 */
#ifndef BORTH_H
#define BORTH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct borth_ctx_s* borth_ctx;

typedef enum {
  BORTH_OK = 0,
  BORTH_ERR_ARG = 1,          /* invalid argument; nothing was enqueued */
  BORTH_ERR_HIP = 2,          /* a HIP runtime call failed */
  BORTH_ERR_NOMEM = 3,        /* workspace allocation failed */
  BORTH_BREAKDOWN = 4,        /* Cholesky pivot <= 0 (see borth_info) */
  BORTH_NONFINITE = 5,        /* NaN/Inf in a Gram matrix */
  BORTH_ERR_UNSUPPORTED = 6   /* valid request this build does not implement */
} borth_status;

typedef enum { BORTH_F64 = 0, BORTH_F32 = 1 } borth_dtype;

/* Precision of the first pass's Gram accumulation (later passes: binary64). */
typedef enum {
  BORTH_GRAM_F64 = 0,        /* binary64 FMAs on the matrix cores (k >= 16) or VALU */
  BORTH_GRAM_DD = 1,         /* double-double Gram (see "DD accumulation" below), DD k x k step */
  BORTH_GRAM_SPLIT_BF16 = 2, /* X in fp32: (hi, lo) bf16 split, MFMA with fp32 accumulation */
  BORTH_GRAM_DD_DOT2 = 3     /* borth_gram only: BORTH_GRAM_DD with the Dot2 accumulation */
} borth_gram_prec;

/* DD accumulation.  A double-double Gram sweep (Sec. 4.2's extended-precision
 * Gram matrix) accumulates each product error-free in one of two ways:
 *   biased (default): every sum of a row panel runs on a power-of-two bias
 *     sigma > 2 x (rows per thread) x max|a| max|b| of the panel, so that the
 *     rounded sum's increment and the product's remainder are exact up to one
 *     rounding of u ulp(sigma): 4 VALU instructions per product, error per
 *     panel and thread about rows x u^2 sigma (~1e-31 relative to
 *     sqrt(G_ii G_jj) where few panels are summed, 5e-32 at millions of rows);
 *   Dot2 (BORTH_FLAG_DD_DOT2, BORTH_GRAM_DD_DOT2): TwoProduct and TwoSum,
 *     8 instructions per product, error about u^2 |G| per thread (~2e-32).
 * The narrow update's fused Gram columns (k <= 8) and the Gram sweeps of
 * the iterated scheme (borth_orthonormalize_iter, whose X lies close to
 * span(Y)) always use Dot2; sweeps weighted by B
 * (borth_orthonormalize_iter_b) always use the biased sums; blocks wider
 * than 88 columns always use Dot2. */

typedef enum { BORTH_CHOL = 0, BORTH_SVQB = 1 } borth_fact;

/* How later passes read the intermediate block Q_1 = Xt Z_1. */
typedef enum {
  BORTH_SCHED_AUTO = 0,
  BORTH_SCHED_MATERIALIZE = 1, /* write Q_1 into Q, re-read it: 2 reads + 2 read/writes */
  BORTH_SCHED_RECOMPUTE = 2    /* recompute Q_1 bitwise from X: 3 reads + 1 write (passes = 2) */
} borth_sched;

#define BORTH_FLAG_SYNC 1u          /* synchronize before returning */
#define BORTH_FLAG_PROJECT_ONCE 2u  /* project against Y in the first pass only (P,C,C) */
#define BORTH_FLAG_GRAPH 4u         /* capture the launch sequence in a cached hipGraph */
#define BORTH_FLAG_NO_FUSE 8u       /* iterated scheme: a separate Gram sweep in every pass */
#define BORTH_FLAG_RANK_REVEAL 16u  /* iterated scheme, SVQB: drop null directions (see below) */
#define BORTH_FLAG_DD_DOT2 32u      /* DD Gram sweeps accumulate with Dot2 (see above) */
#define BORTH_FLAG_AUTO_ESCALATE 64u /* borth_orthonormalize: repeat after a breakdown (below) */
#define BORTH_FLAG_BATCH_PERSISTENT 128u /* batched calls: one persistent launch (see below) */

typedef struct {
  int gram;       /* borth_gram_prec of pass 1 */
  int fact;       /* borth_fact */
  int passes;     /* 1, 2 (default) or 3 */
  int sched;      /* borth_sched */
  double shift;   /* first-pass Cholesky shift, relative: M + shift * trace(M) I.
                     < 0: automatic (2^-13 for the split mode, 0 otherwise);
                     NaN or infinite: BORTH_ERR_ARG. */
  unsigned flags; /* BORTH_FLAG_* */
} borth_opts;

typedef struct {
  int status;       /* borth_status of the numerical work */
  int failed_pass;  /* 1-based pass of a breakdown, 0 if none */
  int failed_pivot; /* 1-based Cholesky pivot (LAPACK potrf style), 0 if none */
  int passes_run;
  /* Estimates from the factors (single-block calls; 0 in batched calls and
   * from borth_factor):
   *   orth_est  ||R_p - I||_F of the last pass p (SVQB: its symmetric
   *             factor): how far that pass's input was from orthonormal
   *             (||Q_{p-1}^T Q_{p-1} - I||_F is about twice it); when it is
   *             far below 1 the result is orthonormal to O(k u);
   *   kappa_est from the first pass: max R_ii / min R_ii (Cholesky; a lower
   *             bound on kappa of the projected X) or sqrt(lambda_max /
   *             lambda_min) of its Gram matrix (SVQB, eigenvalues lifted to
   *             u lambda_max, or 2^-104 lambda_max in DD). */
  double orth_est;
  double kappa_est;
  int escalation;   /* BORTH_FLAG_AUTO_ESCALATE: 0 none, 1 DD Gram, 2 shifted DD */
  /* SVQB (without BORTH_FLAG_RANK_REVEAL): the largest number of eigenvalues
   * of M that one pass lifted to its floor (u lambda_max in binary64,
   * 2^-104 lambda_max in DD), i.e. directions of the block that were
   * numerically dependent; 0 for Cholesky and in batched calls (with
   * BORTH_FLAG_RANK_REVEAL such directions are dropped, not lifted, and
   * borth_iter_info reports the rank). */
  int svqb_lifted;
} borth_info;

/* Fills *opts with the defaults: DD Gram, Cholesky, 2 passes, automatic
 * schedule and shift, no flags. */
void borth_default_opts(borth_opts* opts);

/* Creates a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Allocates only small buffers. */
borth_status borth_create(borth_ctx* ctx, int device, void* hip_stream);
borth_status borth_destroy(borth_ctx ctx);
borth_status borth_set_stream(borth_ctx ctx, void* hip_stream);
const char* borth_status_string(int status);
const char* borth_last_error(borth_ctx ctx);

/* Synchronizes the stream and reports the numerical status of the last
 * orthonormalization (breakdowns are otherwise only visible here). */
borth_status borth_get_info(borth_ctx ctx, borth_info* info);

/* Gram product (TSMTTSM, phase II "M = Xt^T Xt" and the fused phase-I
 * coefficients "C = W^T X", Sec. 4.2): with V = [A | B] (m x (ka + kb)),
 *     G = V^T V   (W x W, W = ka + kb <= 128, symmetric, both halves written).
 * A: binary64 (may be NULL with ka = 0).  B: `dt_b` (BORTH_F32 only with
 * prec = BORTH_GRAM_SPLIT_BF16 and ka = 0).  prec BORTH_GRAM_DD (biased
 * accumulation) or BORTH_GRAM_DD_DOT2 writes the low words to G_lo (device,
 * W x W); G_lo may be NULL otherwise.  The summation order is fixed: results
 * are bitwise reproducible. */
borth_status borth_gram(borth_ctx ctx, int64_t m, int ka, const double* A, int64_t lda,
                        int kb, borth_dtype dt_b, const void* B, int64_t ldb, int prec,
                        double* G_hi, double* G_lo);

/* Small factorization (Sec. 4.2 phase II: a k x k transform Z with
 * Z^T M Z = I): from the Gram matrix G of [Y | X] (W x W,
 * W = ky + k, hi and optional lo words), form
 *     C = G_YX,  M = G_XX - 2 C^T C + C^T G_YY C  (= Xt^T Xt exactly),
 * add shift * trace(M) to the diagonal if shift > 0 (a NaN or infinite
 * shift is BORTH_ERR_ARG), and factor M in DD
 * (G_lo != NULL) or binary64: Cholesky M = R^T R, Z = R^{-1} (upper), or SVQB
 * Z = M^{-1/2}, R = M^{1/2} (Jacobi in the same precision; eigenvalues below
 * 2^-52 lambda_max, DD: 2^-104 lambda_max, lifted to that floor).  Outputs (device, may be NULL):
 * Z (k x k), R (k x k), C (ky x k).  info (host, may be NULL) receives the
 * breakdown pivot; passing it synchronizes. */
borth_status borth_factor(borth_ctx ctx, int ky, int k, const double* G_hi,
                          const double* G_lo, int fact, double shift, double* Z, double* R,
                          double* C, borth_info* info);

/* Basis update (TSMM): Q = (X - Y C) Z with C (ky x k) and Z (k x k,
 * upper-triangular unless z_dense != 0), binary64 FMAs.  X is `dt`
 * (fp32 is widened exactly).  Q may alias X when dt == BORTH_F64 and
 * ldq == ldx (rows are read before they are written). */
borth_status borth_update(borth_ctx ctx, int64_t m, int k, borth_dtype dt, const void* X,
                          int64_t ldx, const double* Y, int64_t ldy, int ky, const double* C,
                          const double* Z, int z_dense, double* Q, int64_t ldq);

/* The whole path: `passes` iterations of (phase I, phase II) with the first
 * Gram in opts->gram precision.  k <= 64, ky <= 64, m >= k + ky.
 * X: m x k (`dt`), Y: m x ky binary64 orthonormal (NULL if ky = 0),
 * Q: m x k binary64 output (may alias X iff dt == BORTH_F64, ldq == ldx and
 * the schedule is MATERIALIZE), R: k x k (R_p ... R_1, device, may be NULL),
 * C: ky x k total coefficients (device, may be NULL).  opts may be NULL
 * (defaults).  info (host) may be NULL; non-NULL synchronizes.  Returns the
 * numerical status when it synchronizes, else BORTH_OK once enqueued.
 *
 * BORTH_FLAG_AUTO_ESCALATE (binary64 X, Q not aliasing X; synchronizes):
 * after a breakdown the call is repeated, first with the DD Gram (if the
 * binary64 one broke down), then with the DD Gram, a first-pass shift of
 * 11 (m k + k (k + 1)) 2^-53 trace(M) and three passes (shifted CholQR3:
 * the shift bounds the condition number of the first pass's result by about
 * (11 m k u)^-1/2, which the binary64 passes after it can take; an X of
 * exact rank below k can still meet a non-positive pivot in a later pass,
 * which is then reported).  info->escalation tells which attempt ran last;
 * R and C are those of the last attempt.
 *
 * The environment variable BORTH_LOG=1 prints one line per call to stderr
 * (shape, options and, when the call synchronizes, status and estimates). */
borth_status borth_orthonormalize(borth_ctx ctx, int64_t m, int k, borth_dtype dt,
                                  const void* X, int64_t ldx, const double* Y, int64_t ldy,
                                  int ky, double* Q, int64_t ldq, double* R, double* C,
                                  const borth_opts* opts, borth_info* info);

/* borth_orthonormalize without allocation, for callers that cannot allocate
 * device memory in the call: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Arguments, results and status
 * as borth_orthonormalize, except that opts->flags must not hold
 * BORTH_FLAG_GRAPH or BORTH_FLAG_AUTO_ESCALATE (BORTH_ERR_ARG).  Every
 * workspace of the call (status words, k x k factors, per-workgroup Gram
 * partials) lives in one file-scope device array of the library, 32 MiB per
 * device, held from the first borth_create on that device until the process
 * ends; a shape whose Gram partials would not fit (only possible with
 * autotuned workgroup counts) is refused with BORTH_ERR_ARG before anything
 * is enqueued.  The call allocates nothing (no hipMalloc, hipFree, events or
 * graphs); the caller passes X, Y, Q, R, C.  All calls on one device share
 * that array and keep the last call's contents: calls that overlap on one
 * GPU (other streams, other contexts, other host threads) race.  The status
 * of an asynchronous call is read only through info or BORTH_FLAG_SYNC
 * (borth_get_info reports the context's own calls). */
borth_status borth_orthonormalize_noalloc(borth_ctx ctx, int64_t m, int k, borth_dtype dt,
                                          const void* X, int64_t ldx, const double* Y,
                                          int64_t ldy, int ky, double* Q, int64_t ldq, double* R,
                                          double* C, const borth_opts* opts, borth_info* info);

/* Outcome of the iterated scheme (borth_orthonormalize_iter). */
typedef struct {
  int converged;  /* 1 if the stop test held after passes_run passes */
  int passes_run;
  double c_norm;  /* ||C_j||_F of the last pass (its projection coefficients) */
  double r_dev;   /* ||R_j - I_r||_F of the last pass (I_r: the first r diagonal ones) */
  int rank;       /* numerical rank r of the last pass (k unless RANK_REVEAL) */
} borth_iter_info;

/* One project / orthonormalize pass with a double-double result (Sec. 4.2:
 * kernels that return DD results; the DD variant of Fig. 7): the DD Gram of
 * [Y | X], the DD factor (opts->fact, Cholesky or SVQB, with the corrected
 * projection coefficients) and a DD update (Dot2 steps on the vector ALUs),
 * rounded once into Q + Q_lo: Q (binary64, m x k, ldq) holds the rounded
 * result and Q_lo its DD low word (same layout), |Q_lo| <= ulp(Q)/2.
 * 1 <= k <= 64, 0 <= ky <= 64.  X_lo (may be NULL, same layout as X) makes
 * the input DD as well, X + X_lo: the DD Gram then also sweeps [X | X_lo]
 * and [Y | X_lo] and combines the blocks (k <= 32 and ky + k <= 64), and the
 * update starts from X + X_lo.  The other options are fixed (DD Gram, one
 * pass, no shift); opts->flags may carry BORTH_FLAG_SYNC and
 * BORTH_FLAG_DD_DOT2.  R and C: binary64 words of the factors.  Q and Q_lo
 * must not alias X, X_lo or each other.  Without X_lo and for k <= 8, Q
 * alone equals what borth_orthonormalize returns for the same DD pass (for
 * wider blocks that call updates in binary64 on the matrix cores). */
borth_status borth_orthonormalize_dd(borth_ctx ctx, int64_t m, int k, const double* X,
                                     const double* X_lo, int64_t ldx, const double* Y,
                                     int64_t ldy, int ky, double* Q, double* Q_lo, int64_t ldq,
                                     double* R, double* C, const borth_opts* opts,
                                     borth_info* info);

/* Iterated two-phase scheme (Sec. 4.2: phase I and phase II alternated until
 * the block no longer changes): pass j projects the current block S_j (X,
 * then Q) against Y and orthonormalizes it, S_{j+1} = (S_j - Y C_j) Z_j, and
 * the iteration stops once a pass changes nothing measurable,
 *     ||C_j||_F <= eps  and  ||R_j - I||_F <= eps,
 * or after max_iter passes.  Every pass's Gram matrix is taken in
 * opts->gram precision (BORTH_GRAM_F64 or BORTH_GRAM_DD; DD also for the
 * factorization), opts->fact selects Cholesky or SVQB;
 * opts->passes, sched and PROJECT_ONCE are ignored.  The first pass sweeps
 * the Gram matrix of [Y | X]; Y^T Y is kept for the later passes.  For
 * narrow blocks (k <= 8, ky + k <= 64, Y dense with ky even) each update
 * sweep writing Q also accumulates the next pass's Gram columns
 * [Y | S_{j+1}]^T S_{j+1} (fused operations, Sec. 4.2), so later passes make
 * one sweep each; otherwise, or with BORTH_FLAG_NO_FUSE in opts->flags, each
 * later pass sweeps [Y | S_j]^T S_j (NO_FUSE: the whole Gram matrix of
 * [Y | S_j]) before its update.  With BORTH_FLAG_RANK_REVEAL and SVQB, each
 * pass keeps the eigenpairs of M above k 2^-52 lambda_max (DD: k 2^-104
 * lambda_max), in their order, as Z = U_r L_r^{-1/2} (k x r, zero columns
 * after r) and R_j = L_r^{1/2} U_r^T: Q's first r columns are an
 * orthonormal basis of the projected block's numerical range, the others
 * zero, and X = Y C + Q R still holds up to the dropped directions;
 * it->rank reports r (the paper's solver resizes its subspace by this
 * rank).  Q may alias X as in borth_orthonormalize;
 * ky <= 64.  The call synchronizes after every pass to evaluate the stop
 * test.  On return X = Y C + Q R with R, C the products
 * of all passes (device, may be NULL); *it (host, required) reports the
 * passes run and the last pass's norms; info (host, may be NULL) the
 * numerical status.  Returns BORTH_OK whether or not the test was met
 * (it->converged tells), or the breakdown status. */
borth_status borth_orthonormalize_iter(borth_ctx ctx, int64_t m, int k, const double* X,
                                       int64_t ldx, const double* Y, int64_t ldy, int ky,
                                       double* Q, int64_t ldq, double* R, double* C,
                                       const borth_opts* opts, double eps, int max_iter,
                                       borth_iter_info* it, borth_info* info);

/* The iterated scheme in a B-inner product, B = diag(bdiag) symmetric
 * positive definite (Sec. 4.2: the technique carries over to B-inner
 * products).  bdiag: m positive weights (device, binary64).  Y must be
 * B-orthonormal (Y^T B Y = I, up to its own rounding: the projection uses
 * the measured Y^T B Y as in the plain case).  Every Gram sweep takes
 * [Y | S]^T B [Y | S] (the DD variant with an exact split of each weighted
 * product); the factors and the update are those of the plain scheme.  On
 * return Q^T B Q = I, Y^T B Q = 0 and X = Y C + Q R.  The Gram sweeps run on
 * the vector-ALU tile kernel (binary64 or DD) and, for narrow blocks, the
 * update's fused Gram columns; everything else as borth_orthonormalize_iter,
 * whose arguments these are. */
borth_status borth_orthonormalize_iter_b(borth_ctx ctx, int64_t m, int k, const double* X,
                                         int64_t ldx, const double* Y, int64_t ldy, int ky,
                                         const double* bdiag, double* Q, int64_t ldq, double* R,
                                         double* C, const borth_opts* opts, double eps,
                                         int max_iter, borth_iter_info* it, borth_info* info);

/* One block of a batch (all pointers device, as in borth_orthonormalize;
 * X binary64). */
typedef struct {
  int64_t m;
  int k;
  const double* X;
  int64_t ldx;
  const double* Y; /* may be NULL with ky = 0 */
  int64_t ldy;
  int ky;
  double* Q;
  int64_t ldq;
  double* R; /* may be NULL */
  double* C; /* may be NULL */
} borth_block;

/* Many independent blocks of uneven shape (e.g. the per-node bases of a
 * contour-integral eigensolver, Sec. 4.1) orthonormalized together, each
 * through the passes of borth_orthonormalize (Sec. 4.2).  Each phase of
 * every block runs in one launch over all blocks.  With
 * BORTH_FLAG_BATCH_PERSISTENT, and when every block takes the DD Gram
 * (biased sums), Cholesky, one or two passes, 5 <= k <= 64 and ky <= 16 (Y
 * projected in every pass), the whole batch runs instead as ONE persistent
 * launch: resident workgroups take (block, sweep, share) tasks from a queue
 * of opened sweeps, and the workgroup that finishes the last share of a
 * block's sweep runs that block's reduction and k x k step and opens its
 * next sweep, so no block waits for the others' phases.  Both run the
 * same arithmetic per block (one pass gives the same bits; with two, the
 * second Gram matrix is summed over the workgroup's waves in another
 * grouping).  Either launch
 * sequence is captured once into a hipGraph cached on the context
 * (BORTH_FLAG_GRAPH) and replayed.  `blocks` and
 * `infos` are host arrays of nblocks entries (infos may be NULL; non-NULL
 * synchronizes).  Rows per workgroup share come from the autotune table
 * when one is loaded. */
borth_status borth_batch_orthonormalize(borth_ctx ctx, int nblocks, const borth_block* blocks,
                                        const borth_opts* opts, borth_info* infos);

/* Times the tile/launch-shape candidates of the Gram and update kernels on
 * synthetic data resident on the device (~budget_ms in total), keeps the
 * fastest per (mode, width) in the context, and writes them as JSON to
 * cache_path (if not NULL), with the device it was measured on
 * (architecture, compute units, HIP runtime version).  borth_autotune_load
 * reads such a file; one made on another device or runtime is refused with
 * BORTH_ERR_ARG. */
borth_status borth_autotune(borth_ctx ctx, const char* cache_path, int budget_ms);
borth_status borth_autotune_load(borth_ctx ctx, const char* cache_path);

/* Average duration (ms) of the dominant kernel launches since profiling was
 * enabled, taken from HIP events on the context's stream.
 * borth_set_profiling(ctx, mask) times the first-pass Gram sweeps (mask bit
 * 0) and the update sweeps (bit 1); 0 turns timing off.  Each timed launch
 * adds two event records to the stream.  kind: 0 = first-pass Gram sweep,
 * 1 = update sweeps; returns the number of timed launches in *count. */
borth_status borth_set_profiling(borth_ctx ctx, int on);
borth_status borth_kernel_time(borth_ctx ctx, int kind, double* avg_ms, int* count);

/* Measurement helper (not part of the method): the HBM rate a plain
 * streaming kernel reaches on this device, the yardstick the sweeps are
 * compared against.  kind 0 reads nbytes from src (dst receives one word per
 * workgroup: at least 64 bytes per compute unit), kind 1 copies nbytes from
 * src to dst, kind 2 the same with non-temporal stores.  Each thread moves
 * 16-byte vectors, four in flight, in a grid-stride loop; grids of 2, 4, 8
 * and 16 workgroups of 256 threads per compute unit are timed with HIP
 * events over reps launches each (after one warm-up launch) and the fastest
 * is returned: *best_ms per launch, *best_grid (may be NULL) its grid.
 * src and dst: device, 16-byte aligned, nbytes a multiple of 16; the call
 * synchronizes. */
borth_status borth_stream_probe(borth_ctx ctx, int kind, const void* src, void* dst,
                                int64_t nbytes, int reps, double* best_ms, int* best_grid);

/* Measurement helper (not part of the method): the FP64 vector-ALU rate a
 * register-only kernel reaches on this device, the yardstick of the DD Gram
 * sweep, which is bound by FP64 VALU issue.  Each thread runs chains over 16
 * independent binary64 sums held in registers, with no memory traffic in
 * the loop: kind 0 plain FMAs, kind 1 the biased DD step of the Gram sweep
 * (fma, add, fma, add per product).  Launches of 1, 2, 4 and 8 waves per
 * SIMD are timed with HIP events (three each, after a warm-up launch) and
 * the fastest is returned: *lane_ops_per_s the FP64 lane operations per
 * second, *waves (may be NULL) its waves per SIMD.  sink: device, 8-byte
 * aligned, nbytes >= 8 x 256 x 8 bytes per compute unit (the sums are
 * written there so that nothing is elided); the call synchronizes. */
borth_status borth_valu_probe(borth_ctx ctx, int kind, void* sink, int64_t nbytes,
                              double* lane_ops_per_s, int* waves);

#ifdef __cplusplus
}
#endif
#endif /* BORTH_H */
