// C ABI of the block-orthonormalization library (see include/borth.h).
//
// Host-side orchestration of the sweeps of one orthonormalization call:
//   pass 1:  Gram sweep over [Y | X] (binary64, DD or split bf16)
//            -> fixed-order reduction -> k x k factor (DD or binary64)
//   pass p:  update sweep (X - Y C) Z with the next pass's Gram fused
//            -> reduction -> factor
//   last:    update sweep writing Q (materialized Q_1 or Q_1 recomputed).
// Everything stays on the device and on one stream; the only readback is the
// 4-int status word when the caller asks for it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ctx.hpp"

using namespace borth;

namespace {

const char* kStatusText[] = {"ok",
                             "invalid argument",
                             "HIP runtime error",
                             "out of device memory",
                             "Cholesky breakdown (non-positive pivot)",
                             "non-finite value in a Gram matrix",
                             "unsupported request"};

void invalidate_graphs(borth_ctx c) {
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

borth_status ensure(borth_ctx c, double** buf, int64_t* cap, int64_t need) {
  if (need <= *cap) return BORTH_OK;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_hip(c, e, "hipStreamSynchronize");
  if (*buf) hipFree(*buf);
  *buf = nullptr;
  *cap = 0;
  int64_t n = need + need / 4;
  e = hipMalloc((void**)buf, sizeof(double) * (size_t)n);
  if (e != hipSuccess) {
    *buf = nullptr;
    c->err = "workspace allocation failed";
    return BORTH_ERR_NOMEM;
  }
  *cap = n;
  invalidate_graphs(c);
  ++c->ws_generation;
  return BORTH_OK;
}

borth_status ensure_status(borth_ctx c, int n) {
  if (n <= c->status_cap && n <= c->h_status_cap) return BORTH_OK;
  hipStreamSynchronize(c->stream);
  if (c->status) hipFree(c->status);
  if (c->h_status) hipHostFree(c->h_status);
  c->status = nullptr;
  c->h_status = nullptr;
  int nn = n < 64 ? 64 : n;
  if (hipMalloc((void**)&c->status, sizeof(int) * nn) != hipSuccess) return BORTH_ERR_NOMEM;
  if (hipHostMalloc((void**)&c->h_status, sizeof(int) * nn, hipHostMallocDefault) != hipSuccess)
    return BORTH_ERR_NOMEM;
  c->status_cap = nn;
  c->h_status_cap = nn;
  invalidate_graphs(c);
  return BORTH_OK;
}

// Small-matrix workspace layout (doubles), for W = ky + k <= 128, kp <= 64.
struct WsLayout {
  int64_t g_hi, g_lo, zp[3], cp[3], rtot, ctot, zu, cu, zplo, cplo, total;
};
WsLayout ws_layout() {
  WsLayout w;
  int64_t o = 0;
  w.g_hi = o; o += 128 * 128;
  w.g_lo = o; o += 128 * 128;
  for (int i = 0; i < 3; ++i) { w.zp[i] = o; o += 64 * 64; }
  for (int i = 0; i < 3; ++i) { w.cp[i] = o; o += 64 * 64; }
  w.rtot = o; o += 2 * 64 * 64;
  w.ctot = o; o += 2 * 64 * 64;
  w.zu = o; o += 64 * 64;
  w.cu = o; o += 64 * 64;
  w.zplo = o; o += 64 * 64;  // low words of Z and C for a DD update
  w.cplo = o; o += 64 * 64;
  w.total = o;
  return w;
}

// Copy a rows x k matrix into a rows x kp zero-padded one (device to device).
borth_status pad_copy(borth_ctx c, double* dst, int kp, const double* src, int k, int rows) {
  if (rows == 0) return BORTH_OK;
  HIPCHK(c, hipMemcpy2DAsync(dst, sizeof(double) * kp, src, sizeof(double) * k, sizeof(double) * k,
                             rows, hipMemcpyDeviceToDevice, c->stream),
         "hipMemcpy2DAsync");
  return BORTH_OK;
}

// The orthonormalization launch sequence (enqueue only).
struct OrthoCall {
  int64_t m;
  int k, ky;
  borth_dtype dt;
  const void* X;
  int64_t ldx;
  const double* Y;
  int64_t ldy;
  double* Q;
  int64_t ldq;
  double* R;
  double* C;
  borth_opts o;
  double* Qlo;        // one DD pass on a narrow block: the result's low words, or null
  const double* Xlo;  // ... and the low words of a DD input X, or null
};

borth_status enqueue_ortho(borth_ctx c, const OrthoCall& a) {
  hipStream_t st = c->cur;
  const WsLayout W = ws_layout();
  double* ws = c->ws;
  const int kp = pow2pad(a.k);
  const int gmode = a.o.gram;
  const bool split = gmode == BORTH_GRAM_SPLIT_BF16;
  const bool dd = gmode == BORTH_GRAM_DD;
  const bool project_each = !(a.o.flags & BORTH_FLAG_PROJECT_ONCE);
  const int passes = a.o.passes;
  int sched = a.o.sched;
  if (sched == BORTH_SCHED_AUTO)
    sched = (passes == 2 && a.dt == BORTH_F64 && kp <= 32 && a.X != (const void*)a.Q)
                ? BORTH_SCHED_RECOMPUTE
                : BORTH_SCHED_MATERIALIZE;
  double shift = a.o.shift;
  if (shift < 0) shift = split ? std::ldexp(1.0, -13) : 0.0;
  const bool hasy = a.ky > 0;

  HIPCHK(c, launch_fill_int(c->status, 7, 0, st), "fill");

  // ---- pass 1: Gram sweep + reduction + factor
  Src s1{a.Y, a.ldy, a.X, a.ldx, a.dt == BORTH_F32 ? 1 : 0, a.m};
  s1.dot2 = (a.o.flags & BORTH_FLAG_DD_DOT2) ? 1 : 0;
  GramLayout L1 = make_layout(a.ky, a.k, 4);
  int nwg = 0;
  prof_begin(c, 0);
  if (split) {
    Src ss{nullptr, 0, a.X, a.ldx, 1, a.m};
    GramLayout Ls = make_layout(0, a.k, 4);
    HIPCHK(c, launch_gram_split(ss, Ls, c->part, c->part_cap, &nwg, lookup(c->tune_gram, 2, kp, 0), st),
           "gram_split");
    prof_end(c, 0);
    HIPCHK(c, launch_reduce(Ls, 0, c->part, nwg, ws + W.g_hi, nullptr, st), "reduce");
  } else {
    HIPCHK(c, launch_gram(s1, L1, dd ? 1 : 0, c->part, c->part_cap, &nwg,
                          lookup(c->tune_gram, dd ? 1 : 0, kp, hasy), st),
           "gram");
    prof_end(c, 0);
    HIPCHK(c, launch_reduce(L1, dd ? 1 : 0, c->part, nwg, ws + W.g_hi, dd ? ws + W.g_lo : nullptr, st),
           "reduce");
    if (a.Xlo) {
      // DD input X = X + X_lo: the Grams of [X | X_lo] and [Y | X_lo] as well,
      // combined with the one above into the DD Gram of [Y | X + X_lo]
      Src sb{a.X ? (const double*)a.X : nullptr, a.ldx, a.Xlo, a.ldx, 0, a.m};
      sb.dot2 = s1.dot2;
      const GramLayout Lb = make_layout(a.k, a.k, 4);
      HIPCHK(c, launch_gram(sb, Lb, 1, c->part, c->part_cap, &nwg, TuneGram{}, st), "gram (X, X_lo)");
      HIPCHK(c, launch_reduce(Lb, 1, c->part, nwg, ws + W.zp[1], ws + W.zp[2], st), "reduce");
      if (hasy) {
        Src sc{a.Y, a.ldy, a.Xlo, a.ldx, 0, a.m};
        sc.dot2 = s1.dot2;
        HIPCHK(c, launch_gram(sc, L1, 1, c->part, c->part_cap, &nwg, TuneGram{}, st), "gram (Y, X_lo)");
        HIPCHK(c, launch_reduce(L1, 1, c->part, nwg, ws + W.cp[1], ws + W.cp[2], st), "reduce");
      }
      HIPCHK(c, launch_gram_dd_combine(a.ky, a.k, ws + W.g_hi, ws + W.g_lo, ws + W.zp[1],
                                       ws + W.zp[2], ws + W.cp[1], ws + W.cp[2], st),
             "combine");
    }
  }
  // One DD pass on a narrow block, or with a DD result requested on a block
  // of up to 64 columns: the update runs in DD as well (the factor then also
  // gives the low words of Z and C).
  const bool dd_update =
      dd && passes == 1 && a.dt == BORTH_F64 && (a.k <= 8 || (a.Qlo && a.k <= 64));
  auto factor = [&](int pass, int kyp_pass, const double* ghi, const double* glo, bool ddm,
                    double shrel, bool last) -> borth_status {
    FactorArgs f;
    memset(&f, 0, sizeof(f));
    f.ky = kyp_pass;
    f.k = a.k;
    f.kp = kp;
    f.G_hi = ghi;
    f.G_lo = glo;
    f.dd = ddm ? 1 : 0;
    f.fact = a.o.fact;
    f.shift_rel = shrel;
    f.pass = pass;
    f.Zp = ws + W.zp[pass];
    f.Cp = ws + W.cp[pass];
    f.Rtot = ws + W.rtot;
    f.Ctot = ws + W.ctot;
    f.status = c->status;
    f.lifted = c->status + 6;
    f.conv = ws + W.cu;  // the last pass's ||R_p - I|| stays (orth_est)
    f.kappa = pass == 0 ? ws + W.cu + 2 : nullptr;
    f.R_out = last ? a.R : nullptr;
    f.C_out = (last && hasy) ? a.C : nullptr;
    if (dd_update && pass == 0) {
      f.Zplo = ws + W.zplo;
      f.Cplo = ws + W.cplo;
    }
    HIPCHK(c, launch_factor(f, st), "factor");
    return BORTH_OK;
  };
  borth_status r = factor(0, a.ky, ws + W.g_hi, dd ? ws + W.g_lo : nullptr, dd, shift, passes == 1);
  if (r) return r;
  // C totals when the later passes do not project: the factor of pass 0 already
  // set C_tot = C_1; later factors run with ky = 0 and leave it (C_out written by
  // the last factor only if it projects, so copy it here).
  const bool later_proj = project_each && hasy;
  if (hasy && !later_proj && passes > 1 && a.C)
    HIPCHK(c, hipMemcpyAsync(a.C, ws + W.ctot, sizeof(double) * a.ky * a.k, hipMemcpyDeviceToDevice, st),
           "copy C");

  GramLayout Lu = make_layout(a.ky, a.k, kp);
  if (passes == 1) {
    UpdateArgs u;
    memset(&u, 0, sizeof(u));
    u.src = s1;
    u.C1 = ws + W.cp[0];
    u.Z1 = ws + W.zp[0];
    if (dd_update) {
      u.C1lo = ws + W.cplo;
      u.Z1lo = ws + W.zplo;
    }
    u.dense = a.o.fact == BORTH_SVQB;
    u.Q = a.Q;
    u.ldq = a.ldq;
    if (dd_update) {
      u.Qlo = a.Qlo;
      u.Xlo = a.Xlo;
    }
    prof_begin(c, 1);
    HIPCHK(c, launch_update(u, Lu, lookup(c->tune_upd, 0, kp, hasy), st), "update");
    prof_end(c, 1);
    return BORTH_OK;
  }

  if (sched == BORTH_SCHED_RECOMPUTE && passes == 2 && !split) {
    // sweep 2: Q_1 in registers, Gram of [Y | Q_1] (or Q_1) fused
    UpdateArgs u;
    memset(&u, 0, sizeof(u));
    u.src = s1;
    u.C1 = ws + W.cp[0];
    u.Z1 = ws + W.zp[0];
    u.dense = a.o.fact == BORTH_SVQB;
    u.gram_with_y = later_proj ? 1 : 0;
    u.partials = c->part;
    u.partial_cap_doubles = c->part_cap;
    prof_begin(c, 1);
    HIPCHK(c, launch_update(u, Lu, lookup(c->tune_upd, 1, kp, hasy), st), "update2");
    prof_end(c, 1);
    HIPCHK(c, launch_reduce(u.glayout, 0, c->part, u.nwg, ws + W.g_hi, nullptr, st), "reduce2");
    r = factor(1, later_proj ? a.ky : 0, ws + W.g_hi, nullptr, false, 0.0, true);
    if (r) return r;
    // sweep 3: recompute Q_1 bitwise, apply pass 2, write Q
    UpdateArgs u3;
    memset(&u3, 0, sizeof(u3));
    u3.src = s1;
    u3.C1 = ws + W.cp[0];
    u3.Z1 = ws + W.zp[0];
    u3.C2 = ws + W.cp[1];
    u3.Z2 = ws + W.zp[1];
    u3.two_stage = 1;
    u3.dense = a.o.fact == BORTH_SVQB;
    u3.Q = a.Q;
    u3.ldq = a.ldq;
    if (!later_proj && hasy) {
      // pass 2 did not project: its C is zero (without Y no sweep reads C)
      HIPCHK(c, launch_fill_int((int*)(ws + W.cp[1]), 2 * 64 * 64, 0, st), "zero C2");
    }
    prof_begin(c, 1);
    HIPCHK(c, launch_update(u3, Lu, lookup(c->tune_upd, 2, kp, hasy), st), "update3");
    prof_end(c, 1);
    return BORTH_OK;
  }

  // materialized schedule: every pass writes its result into Q
  Src cur = s1;
  for (int p = 1; p < passes; ++p) {
    UpdateArgs u;
    memset(&u, 0, sizeof(u));
    u.src = cur;
    u.C1 = ws + W.cp[p - 1];
    u.Z1 = ws + W.zp[p - 1];
    u.dense = a.o.fact == BORTH_SVQB;
    u.Q = a.Q;
    u.ldq = a.ldq;
    u.gram_with_y = later_proj ? 1 : 0;
    u.partials = c->part;
    u.partial_cap_doubles = c->part_cap;
    prof_begin(c, 1);
    HIPCHK(c, launch_update(u, Lu, lookup(c->tune_upd, 1, kp, hasy), st), "update_p");
    prof_end(c, 1);
    HIPCHK(c, launch_reduce(u.glayout, 0, c->part, u.nwg, ws + W.g_hi, nullptr, st), "reduce_p");
    r = factor(p, later_proj ? a.ky : 0, ws + W.g_hi, nullptr, false, 0.0, p == passes - 1);
    if (r) return r;
    cur = Src{a.Y, a.ldy, a.Q, a.ldq, 0, a.m};
    if (!later_proj && hasy)
      HIPCHK(c, launch_fill_int((int*)(ws + W.cp[p]), 2 * 64 * 64, 0, st), "zero C");
  }
  UpdateArgs u;
  memset(&u, 0, sizeof(u));
  u.src = cur;
  u.C1 = ws + W.cp[passes - 1];
  u.Z1 = ws + W.zp[passes - 1];
  u.dense = a.o.fact == BORTH_SVQB;
  u.Q = a.Q;
  u.ldq = a.ldq;
  prof_begin(c, 1);
  HIPCHK(c, launch_update(u, Lu, lookup(c->tune_upd, 0, kp, hasy), st), "update_last");
  prof_end(c, 1);
  return BORTH_OK;
}

int64_t partial_need(int ky, int k, int gmode) {
  const int kp = pow2pad(k);
  GramLayout L1 = make_layout(ky, k, 4);
  GramLayout Lu = make_layout(ky <= 16 && ky > 0 ? 16 : ky, k, kp);
  int64_t e = (int64_t)L1.E * (gmode == BORTH_GRAM_DD ? 2 : 1);
  if (Lu.E > e) e = Lu.E;
  return kMaxSweepWG * e;
}

// Status words (and, when the last call left them, the estimates: ||R_p -
// I||_F of its last pass and the first pass's condition estimate, in the
// spare k x k area of the workspace).
borth_status read_status(borth_ctx c, borth_info* info) {
  HIPCHK(c, hipMemcpyAsync(c->h_status, c->status, sizeof(int) * 7, hipMemcpyDeviceToHost, c->stream),
         "status readback");
  double est[3] = {0.0, 0.0, 0.0};
  if (c->last_est)
    HIPCHK(c, hipMemcpyAsync(est, c->ws + ws_layout().cu, sizeof(est), hipMemcpyDeviceToHost, c->stream),
           "estimates readback");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (info) {
    info->status = c->h_status[0];
    info->failed_pass = c->h_status[1];
    info->failed_pivot = c->h_status[2];
    info->passes_run = c->h_status[3];
    info->orth_est = est[1];
    info->kappa_est = est[2];
    info->escalation = 0;
    info->svqb_lifted = c->h_status[6];
  }
  return (borth_status)c->h_status[0];
}

borth_status ortho_enqueue(borth_ctx c, int64_t m, int k, borth_dtype dt, const void* X,
                           int64_t ldx, const double* Y, int64_t ldy, int ky, double* Q,
                           int64_t ldq, double* R, double* C, const borth_opts& o,
                           double* Qlo = nullptr, const double* Xlo = nullptr);

bool log_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("BORTH_LOG");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  return on;
}

}  // namespace

extern "C" {

void borth_default_opts(borth_opts* o) {
  if (!o) return;
  o->gram = BORTH_GRAM_DD;
  o->fact = BORTH_CHOL;
  o->passes = 2;
  o->sched = BORTH_SCHED_AUTO;
  o->shift = -1.0;
  o->flags = 0;
}

const char* borth_status_string(int s) {
  if (s < 0 || s > 6) return "unknown status";
  return kStatusText[s];
}

borth_status borth_create(borth_ctx* out, int device, void* stream) {
  if (!out) return BORTH_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return BORTH_ERR_ARG;
  borth_ctx c = new borth_ctx_s();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->cur = c->stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return BORTH_ERR_HIP;
  }
  const WsLayout W = ws_layout();
  if (ensure(c, &c->ws, &c->ws_cap, W.total) != BORTH_OK || ensure_status(c, 64) != BORTH_OK) {
    borth_destroy(c);
    return BORTH_ERR_NOMEM;
  }
  // device address of this device's scratch array (allocation-free entry point)
  const hipError_t es = noalloc_setup(device);
  if (es != hipSuccess) c->noalloc_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(es);
  *out = c;
  return BORTH_OK;
}

borth_status borth_destroy(borth_ctx c) {
  if (!c) return BORTH_ERR_ARG;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  invalidate_graphs(c);
  if (c->part) hipFree(c->part);
  if (c->ws) hipFree(c->ws);
  if (c->status) hipFree(c->status);
  if (c->h_status) hipHostFree(c->h_status);
  batch_free_all(c);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  for (auto& p : c->ev_free) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
  for (int k = 0; k < 2; ++k)
    for (auto& p : c->ev_used[k]) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
  delete c;
  return BORTH_OK;
}

borth_status borth_set_stream(borth_ctx c, void* stream) {
  if (!c) return BORTH_ERR_ARG;
  if (c->stream == (hipStream_t)stream) return BORTH_OK;
  c->stream = (hipStream_t)stream;
  c->cur = c->stream;
  return BORTH_OK;
}

const char* borth_last_error(borth_ctx c) { return c ? c->err.c_str() : "null context"; }

borth_status borth_get_info(borth_ctx c, borth_info* info) {
  if (!c || !info) return BORTH_ERR_ARG;
  hipSetDevice(c->device);
  read_status(c, info);
  return BORTH_OK;
}

borth_status borth_gram(borth_ctx c, int64_t m, int ka, const double* A, int64_t lda, int kb,
                        borth_dtype dt_b, const void* B, int64_t ldb, int prec, double* G_hi,
                        double* G_lo) {
  if (!c) return BORTH_ERR_ARG;
  if (m < 0 || ka < 0 || kb < 1 || ka + kb > 128 || !B || !G_hi) return fail_arg(c, "shape/pointers");
  if (ka > 0 && (!A || lda < ka)) return fail_arg(c, "A");
  if (ldb < kb) return fail_arg(c, "ldb");
  if (prec < 0 || prec > 3) return fail_arg(c, "prec");
  if (prec == BORTH_GRAM_SPLIT_BF16 && (dt_b != BORTH_F32 || ka != 0 || kb > 64))
    return fail_arg(c, "split mode needs fp32 B, no A, kb <= 64");
  if (dt_b == BORTH_F32 && (prec == BORTH_GRAM_DD || prec == BORTH_GRAM_DD_DOT2))
    return fail_arg(c, "DD Gram needs binary64 input");
  hipSetDevice(c->device);
  c->cur = c->stream;
  if (m == 0) {  // empty block: G = 0 (the sweeps assume at least one row)
    const int W = ka + kb;
    HIPCHK(c, launch_fill_int((int*)G_hi, 2 * W * W, 0, c->stream), "zero G");
    if (G_lo) HIPCHK(c, launch_fill_int((int*)G_lo, 2 * W * W, 0, c->stream), "zero G");
    return BORTH_OK;
  }
  GramLayout L = make_layout(ka, kb, 4);
  borth_status r = ensure(c, &c->part, &c->part_cap, kMaxSweepWG * (int64_t)L.E * 2);
  if (r) return r;
  int nwg = 0;
  const int kp = pow2pad(kb);
  if (prec == BORTH_GRAM_SPLIT_BF16) {
    Src s{nullptr, 0, B, ldb, 1, m};
    prof_begin(c, 0);
    HIPCHK(c, launch_gram_split(s, L, c->part, c->part_cap, &nwg, lookup(c->tune_gram, 2, kp, 0), c->stream), "gram_split");
    prof_end(c, 0);
    HIPCHK(c, launch_reduce(L, 0, c->part, nwg, G_hi, G_lo, c->stream), "reduce");
  } else {
    Src s{A, lda, B, ldb, dt_b == BORTH_F32 ? 1 : 0, m};
    s.dot2 = prec == BORTH_GRAM_DD_DOT2 ? 1 : 0;
    const int mode = prec == BORTH_GRAM_DD || prec == BORTH_GRAM_DD_DOT2 ? 1 : 0;
    prof_begin(c, 0);
    HIPCHK(c, launch_gram(s, L, mode, c->part, c->part_cap, &nwg, lookup(c->tune_gram, mode, kp, ka > 0), c->stream), "gram");
    prof_end(c, 0);
    HIPCHK(c, launch_reduce(L, mode, c->part, nwg, G_hi, G_lo, c->stream), "reduce");
  }
  return BORTH_OK;
}

borth_status borth_factor(borth_ctx c, int ky, int k, const double* G_hi, const double* G_lo,
                          int fact, double shift, double* Z, double* R, double* C,
                          borth_info* info) {
  if (!c) return BORTH_ERR_ARG;
  if (k < 1 || k > 64 || ky < 0 || ky > 64 || !G_hi) return fail_arg(c, "shape");
  if (fact != BORTH_CHOL && fact != BORTH_SVQB) return fail_arg(c, "fact");
  if (!std::isfinite(shift)) return fail_arg(c, "shift");
  hipSetDevice(c->device);
  c->cur = c->stream;
  const WsLayout W = ws_layout();
  HIPCHK(c, launch_fill_int(c->status, 7, 0, c->stream), "fill");
  c->last_est = false;
  FactorArgs f;
  memset(&f, 0, sizeof(f));
  f.ky = ky;
  f.k = k;
  f.kp = pow2pad(k);
  f.G_hi = G_hi;
  f.G_lo = G_lo;
  f.dd = G_lo ? 1 : 0;
  f.fact = fact;
  f.shift_rel = shift > 0 ? shift : 0.0;
  f.pass = 0;
  f.Zp = c->ws + W.zp[0];
  f.Cp = c->ws + W.cp[0];
  f.Rtot = c->ws + W.rtot;
  f.Ctot = c->ws + W.ctot;
  f.status = c->status;
  f.lifted = c->status + 6;
  f.R_out = R;
  f.C_out = C;
  f.Z_out = Z;
  HIPCHK(c, launch_factor(f, c->stream), "factor");
  if (info) return read_status(c, info);
  return BORTH_OK;
}

borth_status borth_update(borth_ctx c, int64_t m, int k, borth_dtype dt, const void* X,
                          int64_t ldx, const double* Y, int64_t ldy, int ky, const double* C,
                          const double* Z, int z_dense, double* Q, int64_t ldq) {
  if (!c) return BORTH_ERR_ARG;
  if (m < 0 || k < 1 || k > 64 || ky < 0 || ky > 64) return fail_arg(c, "shape");
  if (!X || !Z || !Q || ldx < k || ldq < k) return fail_arg(c, "pointers/ld");
  if (ky > 0 && (!Y || !C || ldy < ky)) return fail_arg(c, "Y/C");
  if (dt == BORTH_F32 && ky > 0) return fail_arg(c, "fp32 X with a locked basis is not supported");
  if ((const void*)Q == X && (dt != BORTH_F64 || ldq != ldx)) return fail_arg(c, "aliasing");
  hipSetDevice(c->device);
  c->cur = c->stream;
  const WsLayout W = ws_layout();
  const int kp = pow2pad(k);
  double* zp = c->ws + W.zu;
  double* cp = c->ws + W.cu;  // also where the estimates of a path call live:
  c->last_est = false;        // they are gone once C is staged here
  HIPCHK(c, launch_fill_int((int*)zp, 2 * 64 * 64, 0, c->stream), "zero Z");
  HIPCHK(c, launch_fill_int((int*)cp, 2 * 64 * 64, 0, c->stream), "zero C");
  borth_status r = pad_copy(c, zp, kp, Z, k, k);
  if (r) return r;
  if (ky > 0) {
    r = pad_copy(c, cp, kp, C, k, ky);
    if (r) return r;
  }
  UpdateArgs u;
  memset(&u, 0, sizeof(u));
  u.src = Src{Y, ldy, X, ldx, dt == BORTH_F32 ? 1 : 0, m};
  u.C1 = cp;
  u.Z1 = zp;
  u.dense = z_dense ? 1 : 0;
  u.Q = Q;
  u.ldq = ldq;
  GramLayout L = make_layout(ky, k, kp);
  prof_begin(c, 1);
  HIPCHK(c, launch_update(u, L, lookup(c->tune_upd, 0, kp, ky > 0), c->stream), "update");
  prof_end(c, 1);
  return BORTH_OK;
}

}  // extern "C"

namespace {
// Argument checks shared by borth_orthonormalize and its allocation-free
// variant (nothing is enqueued before they pass).
borth_status check_ortho_args(borth_ctx c, int64_t m, int k, borth_dtype dt, const void* X,
                              int64_t ldx, const double* Y, int64_t ldy, int ky, double* Q,
                              int64_t ldq, const borth_opts& o) {
  if (k < 1 || k > 64 || ky < 0 || ky > 64 || m < (int64_t)k + ky) return fail_arg(c, "shape");
  if (!X || !Q || ldx < k || ldq < k) return fail_arg(c, "X/Q");
  if (ky > 0 && (!Y || ldy < ky)) return fail_arg(c, "Y");
  if (o.passes < 1 || o.passes > 3) return fail_arg(c, "passes");
  if (!std::isfinite(o.shift)) return fail_arg(c, "shift");
  if (o.gram < 0 || o.gram > 2 || (o.fact != BORTH_CHOL && o.fact != BORTH_SVQB)) return fail_arg(c, "opts");
  if (o.gram == BORTH_GRAM_SPLIT_BF16 && (dt != BORTH_F32 || ky > 0))
    return fail_arg(c, "split mode needs fp32 X and no locked basis");
  if (o.gram != BORTH_GRAM_SPLIT_BF16 && dt == BORTH_F32) return fail_arg(c, "fp32 X needs the split mode");
  if ((const void*)Q == X) {
    if (dt != BORTH_F64 || ldq != ldx) return fail_arg(c, "aliasing");
    if (o.sched == BORTH_SCHED_RECOMPUTE) return fail_arg(c, "recompute schedule cannot run in place");
  }
  if (ky > 16 && o.passes > 1 && !(o.flags & BORTH_FLAG_PROJECT_ONCE)) {
    c->err = "fused Gram with a locked basis supports ky <= 16";
    return BORTH_ERR_UNSUPPORTED;
  }
  if (o.sched == BORTH_SCHED_RECOMPUTE && (dt != BORTH_F64 || o.passes != 2)) return fail_arg(c, "recompute needs binary64 X and 2 passes");
  const bool escalate = (o.flags & BORTH_FLAG_AUTO_ESCALATE) != 0;
  if (escalate && (dt != BORTH_F64 || (const void*)Q == X))
    return fail_arg(c, "automatic escalation needs binary64 X and Q distinct from X");
  return BORTH_OK;
}
}  // namespace

extern "C" {

borth_status borth_orthonormalize(borth_ctx c, int64_t m, int k, borth_dtype dt, const void* X,
                                  int64_t ldx, const double* Y, int64_t ldy, int ky, double* Q,
                                  int64_t ldq, double* R, double* C, const borth_opts* opts,
                                  borth_info* info) {
  if (!c) return BORTH_ERR_ARG;
  borth_opts o;
  if (opts) o = *opts; else borth_default_opts(&o);
  {
    const borth_status ra = check_ortho_args(c, m, k, dt, X, ldx, Y, ldy, ky, Q, ldq, o);
    if (ra) return ra;
  }
  const bool escalate = (o.flags & BORTH_FLAG_AUTO_ESCALATE) != 0;
  hipSetDevice(c->device);
  borth_status r = ortho_enqueue(c, m, k, dt, X, ldx, Y, ldy, ky, Q, ldq, R, C, o);
  if (r) return r;
  const bool sync = info || escalate || (o.flags & BORTH_FLAG_SYNC);
  borth_info local;
  borth_info* inf = info ? info : &local;
  borth_status st = BORTH_OK;
  int level = 0;
  if (sync) {
    st = read_status(c, inf);
    // escalation: DD Gram, then DD Gram with a first-pass shift and three passes
    while (escalate && st == BORTH_BREAKDOWN && level < 2) {
      borth_opts o2 = o;
      o2.flags &= ~BORTH_FLAG_AUTO_ESCALATE;
      o2.gram = BORTH_GRAM_DD;
      level = o.gram == BORTH_GRAM_DD ? 2 : level + 1;
      if (level == 2) {
        if (ky > 16 && !(o.flags & BORTH_FLAG_PROJECT_ONCE)) break;  // fused Gram limit
        // the shift of shifted CholQR3 with the binary64 unit roundoff: the
        // passes after the first are binary64 and must see a first-pass
        // result with kappa^2 u < 1 even when X is rank deficient
        o2.shift = 11.0 * ((double)m * k + (double)k * (k + 1)) * std::ldexp(1.0, -53);
        o2.passes = 3;
        o2.sched = BORTH_SCHED_MATERIALIZE;
      }
      r = ortho_enqueue(c, m, k, dt, X, ldx, Y, ldy, ky, Q, ldq, R, C, o2);
      if (r) return r;
      st = read_status(c, inf);
    }
    inf->escalation = level;
  }
  if (log_enabled()) {
    std::fprintf(stderr, "borth: orthonormalize m=%lld k=%d ky=%d dt=%d gram=%d fact=%d passes=%d "
                 "sched=%d shift=%g flags=%u", (long long)m, k, ky, (int)dt, o.gram, o.fact,
                 o.passes, o.sched, o.shift, o.flags);
    if (sync)
      std::fprintf(stderr, " -> status=%d passes_run=%d orth_est=%.3e kappa_est=%.3e escalation=%d",
                   inf->status, inf->passes_run, inf->orth_est, inf->kappa_est, inf->escalation);
    std::fprintf(stderr, "\n");
  }
  return sync ? st : BORTH_OK;
}

namespace {
// Upper bound (doubles) of the Gram partials one borth_orthonormalize call
// writes, from the workgroup counts its sweeps choose (autotuned or default;
// the DD tile sweep without a tuned count fits its grid to the space given).
int64_t noalloc_partial_need(borth_ctx c, int ky, int k, const borth_opts& o) {
  const int kp = pow2pad(k);
  const bool hasy = ky > 0;
  const bool dd = o.gram == BORTH_GRAM_DD;
  auto wg = [](const TuneGram& t) { return (int64_t)(t.nwg > 0 ? t.nwg : 1024); };
  int64_t need = 0;
  if (o.gram == BORTH_GRAM_SPLIT_BF16) {
    need = wg(lookup(c->tune_gram, 2, kp, 0)) * make_layout(0, k, 4).E;
  } else {
    const GramLayout L1 = make_layout(ky, k, 4);
    const TuneGram t = lookup(c->tune_gram, dd ? 1 : 0, kp, hasy);
    const bool rows = !dd && L1.ty == 0 && L1.Wp <= 8;
    if (!rows && gram_kind(L1, dd ? 1 : 0) == 1 && t.nwg <= 0)
      need = (int64_t)L1.E * (dd ? 2 : 1);
    else
      need = wg(t) * L1.E * (dd ? 2 : 1);
  }
  if (o.passes > 1) {
    const bool later_proj = hasy && !(o.flags & BORTH_FLAG_PROJECT_ONCE);
    const GramLayout G = update_gram_layout(ky, k, kp, later_proj);
    const int64_t u = wg(lookup(c->tune_upd, 1, kp, hasy)) * G.E;
    if (u > need) need = u;
  }
  return need;
}
}  // namespace

extern "C" borth_status borth_orthonormalize_noalloc(borth_ctx c, int64_t m, int k,
                                                     borth_dtype dt, const void* X, int64_t ldx,
                                                     const double* Y, int64_t ldy, int ky,
                                                     double* Q, int64_t ldq, double* R, double* C,
                                                     const borth_opts* opts, borth_info* info) {
  if (!c) return BORTH_ERR_ARG;
  borth_opts o;
  if (opts) o = *opts; else borth_default_opts(&o);
  {
    const borth_status ra = check_ortho_args(c, m, k, dt, X, ldx, Y, ldy, ky, Q, ldq, o);
    if (ra) return ra;
  }
  if (o.flags & (BORTH_FLAG_GRAPH | BORTH_FLAG_AUTO_ESCALATE))
    return fail_arg(c, "the allocation-free call takes neither BORTH_FLAG_GRAPH nor "
                       "BORTH_FLAG_AUTO_ESCALATE");
  double* sp = noalloc_scratch(c->device);
  if (!sp) {
    c->err = "device scratch address unavailable: " + c->noalloc_err;
    return BORTH_ERR_HIP;
  }
  // scratch: [status words (64 ints)][k x k workspace][Gram partials]
  const WsLayout W = ws_layout();
  const int64_t ws_off = 32;
  const int64_t part_off = ws_off + ((W.total + 31) / 32) * 32;
  const int64_t part_cap = kNoallocScratchDoubles - part_off;
  const int64_t need = noalloc_partial_need(c, ky, k, o);
  if (need > part_cap) {
    c->err = "allocation-free call: this shape's Gram partials need " + std::to_string(need) +
             " doubles, the device scratch holds " + std::to_string(part_cap);
    return BORTH_ERR_ARG;
  }
  hipSetDevice(c->device);
  // the regular launch sequence with the context's buffers replaced by the
  // scratch for the duration of the enqueue (no profiling events: creating
  // them could allocate)
  double* const save_part = c->part;
  const int64_t save_part_cap = c->part_cap;
  double* const save_ws = c->ws;
  const int64_t save_ws_cap = c->ws_cap;
  int* const save_status = c->status;
  const int save_prof = c->prof;
  c->part = sp + part_off;
  c->part_cap = part_cap;
  c->ws = sp + ws_off;
  c->ws_cap = W.total;
  c->status = (int*)sp;
  c->prof = 0;
  c->cur = c->stream;
  const OrthoCall a{m, k, ky, dt, X, ldx, Y, ldy, Q, ldq, R, C, o, nullptr, nullptr};
  const borth_status r = enqueue_ortho(c, a);
  c->part = save_part;
  c->part_cap = save_part_cap;
  c->ws = save_ws;
  c->ws_cap = save_ws_cap;
  c->status = save_status;
  c->prof = save_prof;
  if (r) return r;
  const bool sync = info || (o.flags & BORTH_FLAG_SYNC);
  if (!sync) return BORTH_OK;
  int hs[7] = {0, 0, 0, 0, 0, 0, 0};
  double est[3] = {0.0, 0.0, 0.0};
  HIPCHK(c, hipMemcpyAsync(hs, sp, sizeof(hs), hipMemcpyDeviceToHost, c->stream), "status readback");
  HIPCHK(c, hipMemcpyAsync(est, sp + ws_off + W.cu, sizeof(est), hipMemcpyDeviceToHost, c->stream),
         "estimates readback");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (info) {
    info->status = hs[0];
    info->failed_pass = hs[1];
    info->failed_pivot = hs[2];
    info->passes_run = hs[3];
    info->orth_est = est[1];
    info->kappa_est = est[2];
    info->escalation = 0;
    info->svqb_lifted = hs[6];
  }
  return (borth_status)hs[0];
}

namespace {
// One orthonormalization enqueued on the context's stream (captured into a
// cached hipGraph with BORTH_FLAG_GRAPH); arguments already validated.
borth_status ortho_enqueue(borth_ctx c, int64_t m, int k, borth_dtype dt, const void* X,
                           int64_t ldx, const double* Y, int64_t ldy, int ky, double* Q,
                           int64_t ldq, double* R, double* C, const borth_opts& o, double* Qlo,
                           const double* Xlo) {
  borth_status r = ensure(c, &c->part, &c->part_cap, partial_need(ky, k, o.gram));
  if (r) return r;
  c->last_est = true;
  OrthoCall a{m, k, ky, dt, X, ldx, Y, ldy, Q, ldq, R, C, o, Qlo, Xlo};
  if (o.flags & BORTH_FLAG_GRAPH) {
    GraphKey key;
    key.v = {m, k, ky, (int64_t)dt, (int64_t)(intptr_t)X, ldx, (int64_t)(intptr_t)Y, ldy,
             (int64_t)(intptr_t)Q, ldq, (int64_t)(intptr_t)R, (int64_t)(intptr_t)C, o.gram, o.fact,
             o.passes, o.sched, key_bits(o.shift), (int64_t)o.flags,
             (int64_t)c->ws_generation};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      if (!c->cap_stream)
        HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
      HIPCHK(c, hipStreamSynchronize(c->stream), "sync before capture");
      const hipError_t eb = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
      if (eb != hipSuccess) return fail_hip(c, eb, "hipStreamBeginCapture");
      c->capturing = true;
      c->cur = c->cap_stream;
      r = enqueue_ortho(c, a);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
      c->capturing = false;
      c->cur = c->stream;
      if (r) { if (g) hipGraphDestroy(g); return r; }
      if (e != hipSuccess) return fail_hip(c, e, "hipStreamEndCapture");
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) return fail_hip(c, e, "hipGraphInstantiate");
      it = c->graphs.emplace(key, ex).first;
    }
    HIPCHK(c, hipGraphLaunch(it->second, c->stream), "hipGraphLaunch");
  } else {
    c->cur = c->stream;
    r = enqueue_ortho(c, a);
    if (r) return r;
  }
  return BORTH_OK;
}

// The iterated scheme, in the inner product of B = diag(bw) (bw = null: B = I).
borth_status iter_impl(borth_ctx c, int64_t m, int k, const double* X, int64_t ldx,
                       const double* Y, int64_t ldy, int ky, const double* bw, double* Q,
                       int64_t ldq, double* R, double* C, const borth_opts* opts, double eps,
                       int max_iter, borth_iter_info* it, borth_info* info) {
  if (!c) return BORTH_ERR_ARG;
  borth_opts o;
  if (opts) o = *opts; else borth_default_opts(&o);
  if (!it) return fail_arg(c, "iteration report (it) is required");
  if (k < 1 || k > 64 || ky < 0 || ky > 64 || m < (int64_t)k + ky) return fail_arg(c, "shape");
  if (!X || !Q || ldx < k || ldq < k) return fail_arg(c, "X/Q");
  if (ky > 0 && (!Y || ldy < ky)) return fail_arg(c, "Y");
  if ((const void*)Q == (const void*)X && ldq != ldx) return fail_arg(c, "aliasing");
  if (!(eps >= 0.0) || max_iter < 1 || max_iter > 64) return fail_arg(c, "eps / max_iter");
  if (o.gram != BORTH_GRAM_F64 && o.gram != BORTH_GRAM_DD) return fail_arg(c, "opts.gram");
  if (o.fact != BORTH_CHOL && o.fact != BORTH_SVQB) return fail_arg(c, "opts.fact");
  hipSetDevice(c->device);
  c->cur = c->stream;
  const bool dd = o.gram == BORTH_GRAM_DD;
  GramLayout L = make_layout(ky, k, 4);
  const GramLayout Lx = make_layout_xcols(ky, k, 4);
  borth_status r = ensure(c, &c->part, &c->part_cap, kMaxSweepWG * (int64_t)L.E * 2);
  if (r) return r;
  const WsLayout W = ws_layout();
  double* ws = c->ws;
  const int kp = pow2pad(k);
  double* conv = ws + W.cu;  // two doubles of the spare k x k area
  // status[5]: the stop word (0 = running; else the number of passes made)
  HIPCHK(c, launch_fill_int(c->status, 7, 0, c->stream), "fill");
  int* stop = c->status + 5;
  c->last_est = true;
  it->converged = 0;
  it->passes_run = 0;
  it->c_norm = it->r_dev = 0.0;
  it->rank = k;
  // Narrow blocks: each update also accumulates the next pass's Gram columns
  // (the fused operations of Sec. 4.2), so after the first pass no separate
  // sweep over the block is made.
  const bool nofuse = (o.flags & BORTH_FLAG_NO_FUSE) != 0;
  const bool rank_reveal = (o.flags & BORTH_FLAG_RANK_REVEAL) != 0 && o.fact == BORTH_SVQB;
  const bool fuse = !nofuse && k <= 8 && ky + k <= 64 &&
                    (ky == 0 || (ky % 2 == 0 && ldy == ky && ((uintptr_t)Y & 15) == 0));
  bool have_gram = false;  // the Gram of this pass's input is already reduced
  // DD on a narrow block: the updates run in DD as well
  const bool dd_update = dd && k <= 8;
  // The stop test runs on the device: the factor of the pass that meets it
  // (or breaks down) sets the stop word, and every kernel of a later pass
  // returns at once.  Passes are enqueued in chunks with one host
  // synchronization per chunk instead of one per pass.
  int chunk_end = max_iter < 3 ? max_iter : 3;
  for (int p = 0; p < max_iter; ++p) {
    const double* S = p == 0 ? X : Q;
    const int64_t lds_ = p == 0 ? ldx : ldq;
    Src src{Y, ldy, S, lds_, 0, m};
    src.stop = stop;
    src.pass = p;
    Src gsrc = src;  // the Gram sweeps take B's diagonal
    gsrc.bw = bw;
    // The iterated scheme works on X close to span(Y), where M = G_XX -
    // C^T (2C - S C) cancels down to ~kappa(X, Y)^-2 of G_XX: its DD sweeps
    // take Dot2 (error ~u^2 |G|), not the biased sums (error set by the panel
    // maxima), which left M accurate only to ~1e-6 at kappa(X, Y) = 1e12 and
    // cost a pass.  (The weighted sweep has the biased sums only.)
    gsrc.dot2 = 1;
    if (!have_gram) {
      int nwg = 0;
      // Y does not change between passes: after the first, only the columns
      // [Y | S]^T S are swept and Y^T Y stays from the first pass's reduction.
      const GramLayout Lg = (p > 0 && !nofuse) ? Lx : L;
      prof_begin(c, 0);
      HIPCHK(c, launch_gram(gsrc, Lg, dd ? 1 : 0, c->part, c->part_cap, &nwg,
                            Lg.ty > 0 ? TuneGram{} : lookup(c->tune_gram, dd ? 1 : 0, kp, ky > 0),
                            c->stream),
             "gram");
      prof_end(c, 0);
      HIPCHK(c, launch_reduce(Lg, dd ? 1 : 0, c->part, nwg, ws + W.g_hi, dd ? ws + W.g_lo : nullptr,
                              c->stream, stop, p),
             "reduce");
    }
    FactorArgs f;
    memset(&f, 0, sizeof(f));
    f.ky = ky;
    f.k = k;
    f.kp = kp;
    f.G_hi = ws + W.g_hi;
    f.G_lo = dd ? ws + W.g_lo : nullptr;
    f.dd = dd ? 1 : 0;
    f.fact = o.fact;
    f.shift_rel = 0.0;
    f.pass = p;
    f.Zp = ws + W.zp[0];
    f.Cp = ws + W.cp[0];
    f.Rtot = ws + W.rtot;
    f.Ctot = ws + W.ctot;
    f.status = c->status;
    f.lifted = c->status + 6;
    f.conv = conv;
    f.kappa = p == 0 ? conv + 2 : nullptr;
    f.rank_reveal = rank_reveal ? 1 : 0;
    f.stop = stop;
    f.stop_eps = eps;
    if (dd_update) {
      f.Zplo = ws + W.zplo;
      f.Cplo = ws + W.cplo;
    }
    HIPCHK(c, launch_factor(f, c->stream), "factor");
    UpdateArgs u;
    memset(&u, 0, sizeof(u));
    u.src = src;
    u.C1 = ws + W.cp[0];
    u.Z1 = ws + W.zp[0];
    u.dense = o.fact == BORTH_SVQB;
    u.Q = Q;
    u.ldq = ldq;
    if (dd_update) {
      u.C1lo = ws + W.cplo;
      u.Z1lo = ws + W.zplo;
    }
    if (fuse) {
      u.partials = c->part;
      u.partial_cap_doubles = c->part_cap;
      u.gram_xcols = 1;
      u.gram_dd = dd ? 1 : 0;
      u.bw = bw;
    }
    prof_begin(c, 1);
    HIPCHK(c, launch_update(u, make_layout(ky, k, kp), lookup(c->tune_upd, 0, kp, ky > 0),
                            c->stream),
           "update");
    prof_end(c, 1);
    if (fuse) {
      HIPCHK(c, launch_reduce(u.glayout, dd ? 1 : 0, c->part, u.nwg, ws + W.g_hi,
                              dd ? ws + W.g_lo : nullptr, c->stream, stop, p),
             "reduce (fused)");
      have_gram = true;
    }
    if (p + 1 < chunk_end) continue;
    // end of a chunk: status, stop word and the norms of the last pass made
    HIPCHK(c, hipMemcpyAsync(c->h_status, c->status, sizeof(int) * 6, hipMemcpyDeviceToHost,
                             c->stream),
           "status readback");
    double hn[2] = {0.0, 0.0};
    HIPCHK(c, hipMemcpyAsync(hn, conv, sizeof(hn), hipMemcpyDeviceToHost, c->stream), "norms");
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    const int done = c->h_status[5];
    it->passes_run = done ? done : p + 1;
    it->c_norm = hn[0];
    it->r_dev = hn[1];
    it->rank = rank_reveal ? c->h_status[4] : k;
    if (done) {
      it->converged = c->h_status[0] == 0;
      break;
    }
    chunk_end = p + 3 < max_iter ? p + 3 : max_iter;
  }
  // totals: R = R_j ... R_1 and C (hi words of the DD totals)
  if (R)
    HIPCHK(c, hipMemcpyAsync(R, ws + W.rtot, sizeof(double) * k * k, hipMemcpyDeviceToDevice,
                             c->stream),
           "copy R");
  if (C && ky > 0)
    HIPCHK(c, hipMemcpyAsync(C, ws + W.ctot, sizeof(double) * ky * k, hipMemcpyDeviceToDevice,
                             c->stream),
           "copy C");
  borth_info local;
  const borth_status st = read_status(c, info ? info : &local);
  if (log_enabled())
    std::fprintf(stderr, "borth: orthonormalize_iter m=%lld k=%d ky=%d weighted=%d gram=%d fact=%d "
                 "eps=%g max_iter=%d flags=%u -> status=%d converged=%d passes_run=%d c_norm=%.3e "
                 "r_dev=%.3e rank=%d kappa_est=%.3e\n", (long long)m, k, ky, bw ? 1 : 0, o.gram,
                 o.fact, eps, max_iter, o.flags, (int)st, it->converged, it->passes_run, it->c_norm,
                 it->r_dev, it->rank, (info ? info : &local)->kappa_est);
  return st;
}
}  // namespace

borth_status borth_orthonormalize_dd(borth_ctx c, int64_t m, int k, const double* X,
                                     const double* X_lo, int64_t ldx, const double* Y, int64_t ldy,
                                     int ky, double* Q, double* Q_lo, int64_t ldq, double* R,
                                     double* C, const borth_opts* opts, borth_info* info) {
  if (!c) return BORTH_ERR_ARG;
  borth_opts o;
  if (opts) o = *opts; else borth_default_opts(&o);
  if (k < 1 || k > 64 || ky < 0 || ky > 64 || m < (int64_t)k + ky) return fail_arg(c, "shape (k <= 64)");
  if (!X || !Q || !Q_lo || ldx < k || ldq < k) return fail_arg(c, "X/Q/Q_lo");
  if (ky > 0 && (!Y || ldy < ky)) return fail_arg(c, "Y");
  if ((const void*)Q == (const void*)X || (const void*)Q_lo == (const void*)X || Q_lo == Q ||
      (X_lo && ((const void*)X_lo == (const void*)Q || (const void*)X_lo == (const void*)Q_lo)))
    return fail_arg(c, "Q and Q_lo must not alias X, X_lo or each other");
  if (X_lo && (ky + k > 64 || 2 * k > 64)) return fail_arg(c, "a DD input needs ky + k <= 64 and k <= 32");
  if (o.fact != BORTH_CHOL && o.fact != BORTH_SVQB) return fail_arg(c, "opts.fact");
  o.gram = BORTH_GRAM_DD;
  o.passes = 1;
  o.sched = BORTH_SCHED_MATERIALIZE;
  o.shift = 0.0;
  o.flags &= (BORTH_FLAG_SYNC | BORTH_FLAG_DD_DOT2);
  hipSetDevice(c->device);
  if (X_lo) {  // partial sums of the [X | X_lo] sweep
    const borth_status re = ensure(c, &c->part, &c->part_cap,
                                   kMaxSweepWG * (int64_t)make_layout(k, k, 4).E * 2);
    if (re) return re;
  }
  borth_status r = ortho_enqueue(c, m, k, BORTH_F64, X, ldx, Y, ldy, ky, Q, ldq, R, C, o, Q_lo, X_lo);
  if (r) return r;
  const bool sync = info || (o.flags & BORTH_FLAG_SYNC);
  borth_info local;
  borth_info* inf = info ? info : &local;
  const borth_status st = sync ? read_status(c, inf) : BORTH_OK;
  if (log_enabled()) {
    std::fprintf(stderr, "borth: orthonormalize_dd m=%lld k=%d ky=%d fact=%d flags=%u", (long long)m,
                 k, ky, o.fact, o.flags);
    if (sync) std::fprintf(stderr, " -> status=%d kappa_est=%.3e", inf->status, inf->kappa_est);
    std::fprintf(stderr, "\n");
  }
  return st;
}

borth_status borth_orthonormalize_iter(borth_ctx c, int64_t m, int k, const double* X,
                                       int64_t ldx, const double* Y, int64_t ldy, int ky,
                                       double* Q, int64_t ldq, double* R, double* C,
                                       const borth_opts* opts, double eps, int max_iter,
                                       borth_iter_info* it, borth_info* info) {
  return iter_impl(c, m, k, X, ldx, Y, ldy, ky, nullptr, Q, ldq, R, C, opts, eps, max_iter, it,
                   info);
}

borth_status borth_orthonormalize_iter_b(borth_ctx c, int64_t m, int k, const double* X,
                                         int64_t ldx, const double* Y, int64_t ldy, int ky,
                                         const double* bdiag, double* Q, int64_t ldq, double* R,
                                         double* C, const borth_opts* opts, double eps,
                                         int max_iter, borth_iter_info* it, borth_info* info) {
  if (!c) return BORTH_ERR_ARG;
  if (!bdiag) return fail_arg(c, "bdiag");
  return iter_impl(c, m, k, X, ldx, Y, ldy, ky, bdiag, Q, ldq, R, C, opts, eps, max_iter, it,
                   info);
}

borth_status borth_set_profiling(borth_ctx c, int on) {
  if (!c) return BORTH_ERR_ARG;
  hipStreamSynchronize(c->stream);
  for (int k = 0; k < 2; ++k) {
    for (auto& p : c->ev_used[k]) c->ev_free.push_back(p);
    c->ev_used[k].clear();
  }
  c->prof = on & 3;
  return BORTH_OK;
}

borth_status borth_kernel_time(borth_ctx c, int kind, double* avg_ms, int* count) {
  if (!c || kind < 0 || kind > 1 || !avg_ms) return BORTH_ERR_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  double tot = 0.0;
  int n = 0;
  for (auto& p : c->ev_used[kind]) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      tot += ms;
      ++n;
    }
  }
  *avg_ms = n ? tot / n : 0.0;
  if (count) *count = n;
  return BORTH_OK;
}

}  // extern "C"
