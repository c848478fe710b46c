// Batched orthonormalization (borth_batch_orthonormalize) and the
// launch-shape autotuner (borth_autotune, borth_autotune_load).
//
// A batch is many independent blocks [Y_b | X_b] of uneven height and width,
// such as the per-node bases of a contour-integral eigensolver (Sec. 4.1),
// that all go through the pass structure of a single block (Sec. 4.2).
// Instead of one launch sequence per block, every phase runs as ONE launch
// per kernel class over all blocks of that class:
//   * sweeps (Gram, update): block b owns a contiguous range of the launch's
//     workgroups, sized in proportion to its rows, and the kernels find their
//     block through a workgroup -> block map, so one grid streams all blocks
//     and no launch waits on a small block's tail;
//   * reductions: one launch, one grid row per block;
//   * k x k factors: one launch, one workgroup per block, so the latency of
//     hundreds of small factorizations overlaps.
// The plan (descriptor tables, per-block workspace and partial sums, status
// words) is built once per distinct batch and cached on the context; with
// BORTH_FLAG_GRAPH the launch sequence is captured into a hipGraph and every
// later call is a single graph launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "batch_persist.hpp"
#include "ctx.hpp"

using namespace borth;

struct BatchStep {
  enum Kind { FILL, GRAM, REDUCE, FACTOR, UPDATE } kind;
  int grid = 0;          // workgroups (GRAM, UPDATE) or entries (REDUCE, FACTOR)
  int64_t tab_off = -1;  // byte offsets into the plan's device tables
  int64_t map_off = -1;
  // GRAM
  int gkind = 0, gmode = 0, garg = 0;
  size_t shmem = 0;
  // REDUCE
  int red_nb = 0;  // blocks of the reduction launch
  // FACTOR
  FactorArgs fone;
  // UPDATE
  UpdClass uc;
  // FILL
  int fill_n = 0;
};

struct BatchPlan {
  int nblocks = 0;
  char* dtab = nullptr;
  double* part = nullptr;
  double* ws = nullptr;
  int* status = nullptr;
  int* h_status = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<BatchStep> steps;
  // persistent single launch (batch_persist.hpp), when every block fits it
  bool persist = false;
  PBlock* pblocks = nullptr;  // device
  int* porder = nullptr;      // device
  int* pstate = nullptr;      // device, batch_persistent_state_ints(nb) ints
  double* pscratch = nullptr; // device, pgrid x kPersistFactorDoubles
  int pgrid = 0;
  uint64_t last_use = 0;
  int64_t bytes = 0;  // device bytes held
};

namespace {

constexpr int kMaxPlans = 8;

void free_plan(BatchPlan* p) {
  if (!p) return;
  if (p->graph) hipGraphExecDestroy(p->graph);
  if (p->dtab) hipFree(p->dtab);
  if (p->part) hipFree(p->part);
  if (p->ws) hipFree(p->ws);
  if (p->status) hipFree(p->status);
  if (p->h_status) hipHostFree(p->h_status);
  if (p->pblocks) hipFree(p->pblocks);
  if (p->porder) hipFree(p->porder);
  if (p->pstate) hipFree(p->pstate);
  if (p->pscratch) hipFree(p->pscratch);
  delete p;
}

// Host staging of the device tables: arrays appended at 256-byte alignment.
struct TableBuf {
  std::vector<char> b;
  template <typename T>
  int64_t add(const std::vector<T>& v) {
    const int64_t off = ((int64_t)b.size() + 255) & ~(int64_t)255;
    b.resize(off + sizeof(T) * v.size());
    if (!v.empty()) std::memcpy(b.data() + off, v.data(), sizeof(T) * v.size());
    return off;
  }
};

int chol_class(int k) { return k <= 8 ? 0 : k <= 16 ? 1 : k <= 32 ? 2 : k <= 48 ? 3 : 4; }

// Workgroups of each block of a group: one per `rows_per_wg` rows (the
// share a workgroup gets in a single-block sweep, so per-workgroup
// accumulation chains are as long as there), at least one, at most what the
// block can use.
// Rows per workgroup of the batched sweeps (measured defaults; an autotune
// entry's "rows" field overrides them).  The update sweeps accumulate the
// next pass's binary64 Gram, so their workgroups keep a single-block sweep's
// share (~4k rows) and the accumulation chains stay as short.
constexpr int64_t kBatchRowsUpd = 4096;
constexpr int64_t kBatchRowsGram = 4096;
std::vector<int> share_wgs(const std::vector<int64_t>& rows, const std::vector<int>& cap,
                           int64_t rows_per_wg) {
  std::vector<int> n(rows.size());
  for (size_t i = 0; i < rows.size(); ++i) {
    int64_t w = (rows[i] + rows_per_wg - 1) / rows_per_wg;
    if (w < 1) w = 1;
    if (w > cap[i]) w = cap[i];
    n[i] = (int)w;
  }
  return n;
}
// Rows per workgroup from the autotune table's "rows" field.  The tuner
// times one 2M-row block, where short shares win by filling the device; a
// batch has rows enough to fill it with default shares, and for sweeps that
// write partial sums shorter shares only add partials (measured on the
// 256-block batch with the tuner's 512-row shares: DD Gram 41.8 against
// 38.5 ms, its reduction 1.0 against 0.23 ms), so those take tuned rows only
// when longer than the default; update sweeps without a fused Gram take them
// as tuned.  A persistent plan keeps the defaults: its tasks are these
// shares.
int64_t rows_per_wg(const borth::TuneGram& t, int64_t dflt, bool partials = true) {
  if (t.rows <= 0) return dflt;
  return (!partials || t.rows > dflt) ? t.rows : dflt;
}

struct BlkWs {
  int64_t ghi, glo, zp[3], cp[3], rtot, ctot;
  int64_t part;        // offset of this block's partial region (doubles)
  int64_t part_need;   // its size
  int kp;
};

borth_status build_plan(borth_ctx c, int nb, const borth_block* B, const borth_opts& o,
                        BatchPlan** out) {
  const bool dd = o.gram == BORTH_GRAM_DD;
  const int gmode = dd ? 1 : 0;
  const bool svqb = o.fact == BORTH_SVQB;
  const bool project_each = !(o.flags & BORTH_FLAG_PROJECT_ONCE);
  const int passes = o.passes;
  const double shift0 = o.shift > 0 ? o.shift : 0.0;

  std::vector<BlkWs> W(nb);
  int64_t wsz = 0;
  auto take = [&](int64_t n) {
    const int64_t off = wsz;
    wsz += (n + 31) & ~(int64_t)31;
    return off;
  };
  for (int b = 0; b < nb; ++b) {
    const int k = B[b].k, ky = B[b].ky, w = ky + k, kp = pow2pad(k), ky1 = ky > 0 ? ky : 1;
    BlkWs& x = W[b];
    x.kp = kp;
    x.ghi = take((int64_t)w * w);
    x.glo = take((int64_t)w * w);
    for (int p = 0; p < 3; ++p) {
      x.zp[p] = p < passes ? take((int64_t)kp * kp) : -1;
      x.cp[p] = p < passes ? take((int64_t)ky1 * kp) : -1;
    }
    x.rtot = take(2 * (int64_t)k * k);
    x.ctot = take(2 * (int64_t)ky1 * k);
    x.part_need = 0;
  }

  BatchPlan* P = new BatchPlan();
  P->nblocks = nb;
  TableBuf tb;
  std::vector<BatchStep> steps;
  // what the persistent driver needs of each block: its sweeps (table
  // offsets fixed up after the upload), reductions and factors
  struct PRec {
    PBlock pb;
    int64_t tab_off[3], map_off[3];
  };
  std::vector<PRec> pr(nb);
  for (auto& r : pr) std::memset(&r, 0, sizeof(r));
  bool persistable = (o.flags & BORTH_FLAG_BATCH_PERSISTENT) && dd && !svqb && passes >= 1 &&
                     passes <= 2 && !(o.flags & BORTH_FLAG_DD_DOT2);

  {
    BatchStep s;
    s.kind = BatchStep::FILL;
    s.fill_n = 4 * nb;
    steps.push_back(s);
  }

  // ---- pass 1 Gram sweep over [Y | X]: groups by kernel shape
  std::vector<GramLayout> L1(nb);
  std::vector<int> nwg_g(nb);
  std::map<std::pair<int, int>, std::vector<int>> ggroups;
  for (int b = 0; b < nb; ++b) {
    L1[b] = make_layout(B[b].ky, B[b].k, 4);
    const int kind = gram_kind(L1[b], gmode);
    int arg = kind == 0 ? (L1[b].Wp + 15) / 16 : gram_tiles_threads(L1[b]);
    if (kind == 1) {
      Src s{B[b].Y, B[b].ldy, B[b].X, B[b].ldx, 0, B[b].m};
      s.dot2 = (o.flags & BORTH_FLAG_DD_DOT2) ? 1 : 0;
      if (gram_dma_ok(s, L1[b], gmode, arg)) arg = kGramDmaArg;
    }
    ggroups[{kind, arg}].push_back(b);
  }
  struct PendingGram {
    std::pair<int, int> key;
    std::vector<int> blocks;
  };
  std::vector<PendingGram> pend;
  for (auto& kv : ggroups) {
    const int kind = kv.first.first, arg = kv.first.second;
    const int NT = kind == 0 || arg == kGramDmaArg ? 256 : arg;
    std::vector<int64_t> rows;
    std::vector<int> cap;
    int kpmax = 4, hasy = 0;
    for (int b : kv.second) {
      Src s{B[b].Y, B[b].ldy, B[b].X, B[b].ldx, 0, B[b].m};
      s.dot2 = (o.flags & BORTH_FLAG_DD_DOT2) ? 1 : 0;
      rows.push_back(B[b].m);
      cap.push_back(gram_max_wg(s, L1[b], gmode, NT));
      kpmax = std::max(kpmax, W[b].kp);
      hasy |= B[b].ky > 0;
    }
    const std::vector<int> n =
        share_wgs(rows, cap, persistable ? kBatchRowsGram
                                         : rows_per_wg(lookup(c->tune_gram, gmode, kpmax, hasy), kBatchRowsGram));
    for (size_t i = 0; i < kv.second.size(); ++i) {
      const int b = kv.second[i];
      nwg_g[b] = n[i];
      W[b].part_need = std::max(W[b].part_need, (int64_t)n[i] * L1[b].E * (dd ? 2 : 1));
    }
    pend.push_back({kv.first, kv.second});
  }

  // ---- update sweeps: pass p = 1..passes applies Z_{p-1}, W_{p-1}
  const auto later_proj = [&](int b) { return project_each && B[b].ky > 0; };
  std::vector<std::vector<int>> nwg_u(passes + 1, std::vector<int>(nb, 0));
  std::vector<std::vector<GramLayout>> Lu(passes + 1, std::vector<GramLayout>(nb));
  std::vector<std::map<std::tuple<int, int, int>, std::vector<int>>> ugroups(passes + 1);
  std::vector<std::map<std::tuple<int, int, int>, bool>> udma(passes + 1);
  auto uclass = [&](int b, int p) {
    UpdClass uc;
    uc.K = W[b].kp;
    uc.KYP = (B[b].ky > 0 && (p - 1 == 0 || later_proj(b))) ? 16 : 0;
    uc.two = 0;
    uc.gr = p < passes ? (later_proj(b) ? 2 : 1) : 0;
    uc.f32 = 0;
    return uc;
  };
  for (int p = 1; p <= passes; ++p) {
    for (int b = 0; b < nb; ++b) {
      const UpdClass uc = uclass(b, p);
      Lu[p][b] = update_gram_layout(B[b].ky, B[b].k, uc.K, uc.gr == 2);
      ugroups[p][std::make_tuple(uc.K, uc.KYP, uc.gr)].push_back(b);
    }
    for (auto& kv : ugroups[p]) {
      const int K = std::get<0>(kv.first), KYP = std::get<1>(kv.first), gr = std::get<2>(kv.first);
      // panels by direct transfers when every block's rows allow them (not
      // in a persistent plan: its update tasks stream panels through
      // registers, and the transfers' workgroup shares would split them into
      // more, smaller tasks)
      bool dma = !persistable;
      for (int b : kv.second) {
        UpdDev d{};
        d.X = p == 1 ? (const void*)B[b].X : (const void*)B[b].Q;
        d.ldx = p == 1 ? B[b].ldx : B[b].ldq;
        d.k = B[b].k;
        if (KYP) {
          d.Y = B[b].Y;
          d.ldy = B[b].ldy;
          d.ky = B[b].ky;
        }
        dma = dma && update_dma_ok(d, K, KYP, false, false);
      }
      udma[p][kv.first] = dma;
      const int NW = update_waves(K, KYP, dma);
      std::vector<int64_t> rows;
      std::vector<int> cap;
      int hasy = 0;
      for (int b : kv.second) {
        const int64_t np = (B[b].m + update_rows(K, KYP) - 1) / update_rows(K, KYP);
        rows.push_back(B[b].m);
        cap.push_back((int)std::max<int64_t>(1, std::min<int64_t>((np + NW - 1) / NW, 1 << 20)));
        hasy |= B[b].ky > 0;
      }
      const std::vector<int> n =
          share_wgs(rows, cap, persistable ? kBatchRowsUpd
                                           : rows_per_wg(lookup(c->tune_upd, gr ? 1 : 0, K, hasy), kBatchRowsUpd,
                                                         gr != 0));
      for (size_t i = 0; i < kv.second.size(); ++i) {
        const int b = kv.second[i];
        nwg_u[p][b] = n[i];
        if (gr) W[b].part_need = std::max(W[b].part_need, (int64_t)n[i] * Lu[p][b].E);
      }
    }
  }

  // partial regions
  int64_t psz = 0;
  for (int b = 0; b < nb; ++b) {
    W[b].part = psz;
    psz += (W[b].part_need + 31) & ~(int64_t)31;
  }

  // ---- device memory
  auto cleanup = [&](borth_status st, const char* what) {
    free_plan(P);
    if (what) c->err = what;
    return st;
  };
  if (hipMalloc((void**)&P->ws, sizeof(double) * (size_t)std::max<int64_t>(wsz, 32)) != hipSuccess)
    return cleanup(BORTH_ERR_NOMEM, "batch workspace allocation failed");
  if (hipMalloc((void**)&P->part, sizeof(double) * (size_t)std::max<int64_t>(psz, 32)) != hipSuccess)
    return cleanup(BORTH_ERR_NOMEM, "batch partials allocation failed");
  if (hipMalloc((void**)&P->status, sizeof(int) * 4 * (size_t)nb) != hipSuccess)
    return cleanup(BORTH_ERR_NOMEM, "batch status allocation failed");
  if (hipHostMalloc((void**)&P->h_status, sizeof(int) * 4 * (size_t)nb, hipHostMallocDefault) !=
      hipSuccess)
    return cleanup(BORTH_ERR_NOMEM, "batch status allocation failed");
  double* ws = P->ws;
  double* part = P->part;

  // ---- Gram steps
  for (auto& g : pend) {
    const int kind = g.key.first, arg = g.key.second;
    const int NT = kind == 0 || arg == kGramDmaArg ? 256 : arg;
    std::vector<GramSeg> segs;
    std::vector<int> map;
    size_t shmem = 0;
    for (int b : g.blocks) {
      Src s{B[b].Y, B[b].ldy, B[b].X, B[b].ldx, 0, B[b].m};
      s.dot2 = (o.flags & BORTH_FLAG_DD_DOT2) ? 1 : 0;
      GramSeg gs;
      size_t sh = 0;
      if (!gram_seg(s, L1[b], gmode, NT, part + W[b].part, (int)map.size(), nwg_g[b], &gs, &sh))
        return cleanup(BORTH_ERR_UNSUPPORTED, "batch: block shape outside the Gram kernels");
      shmem = std::max(shmem, sh);
      PSweep& ps = pr[b].pb.sw[0];
      ps.kind = arg == kGramDmaArg ? 0 : 1;
      ps.ntasks = nwg_g[b];
      ps.wg0 = (int)map.size();
      pr[b].pb.nsweeps = 1;
      if (kind != 1 || (arg != kGramDmaArg && arg != 256) || sh > kPersistLds) persistable = false;
      for (int i = 0; i < nwg_g[b]; ++i) map.push_back((int)segs.size());
      segs.push_back(gs);
    }
    BatchStep s;
    s.kind = BatchStep::GRAM;
    s.gkind = kind;
    s.gmode = gmode;
    s.garg = arg;
    s.shmem = shmem;
    s.grid = (int)map.size();
    s.tab_off = tb.add(segs);
    s.map_off = tb.add(map);
    for (int b : g.blocks) {
      pr[b].tab_off[0] = s.tab_off;
      pr[b].map_off[0] = s.map_off;
    }
    steps.push_back(s);
  }

  auto add_reduce = [&](int sweep, int mode) {
    std::vector<ReduceSeg> segs(nb);
    int red_nb = 0;
    for (int b = 0; b < nb; ++b) {
      const GramLayout& L = sweep == 0 ? L1[b] : Lu[sweep][b];
      const int n = sweep == 0 ? nwg_g[b] : nwg_u[sweep][b];
      segs[b] = ReduceSeg{L, part + W[b].part, n, ws + W[b].ghi,
                          (sweep == 0 && dd) ? ws + W[b].glo : nullptr};
      red_nb = std::max(red_nb, reduce_blocks(L.E, mode == 1));
      if (sweep < 2) {
        pr[b].pb.red[sweep] = segs[b];
        pr[b].pb.red_dd[sweep] = mode;
      }
    }
    BatchStep s;
    s.kind = BatchStep::REDUCE;
    s.gmode = mode;
    s.red_nb = red_nb;
    s.grid = nb;
    s.tab_off = tb.add(segs);
    steps.push_back(s);
  };

  auto add_factor = [&](int p) {
    std::map<std::pair<int, int>, std::vector<int>> fg;
    for (int b = 0; b < nb; ++b) fg[{svqb ? 9 : chol_class(B[b].k), 0}].push_back(b);
    for (auto& kv : fg) {
      std::vector<FactorArgs> tabv;
      FactorArgs widest;
      int kmax = 0;
      for (int b : kv.second) {
        const bool proj = p == 0 || later_proj(b);
        const bool last = p == passes - 1;
        FactorArgs f;
        std::memset(&f, 0, sizeof(f));
        f.ky = proj ? B[b].ky : 0;
        f.k = B[b].k;
        f.kp = W[b].kp;
        f.G_hi = ws + W[b].ghi;
        f.G_lo = (p == 0 && dd) ? ws + W[b].glo : nullptr;
        f.dd = (p == 0 && dd) ? 1 : 0;
        f.fact = svqb ? 1 : 0;
        f.shift_rel = p == 0 ? shift0 : 0.0;
        f.pass = p;
        f.Zp = ws + W[b].zp[p];
        f.Cp = ws + W[b].cp[p];
        f.Rtot = ws + W[b].rtot;
        f.Ctot = ws + W[b].ctot;
        f.status = P->status + 4 * b;
        f.R_out = last ? B[b].R : nullptr;
        const bool c_now = B[b].ky > 0 && ((last && later_proj(b)) || (p == 0 && !later_proj(b)));
        f.C_out = c_now ? B[b].C : nullptr;
        f.Z_out = nullptr;
        f.Rp_out = nullptr;
        if (p < 2) {
          pr[b].pb.fac[p] = f;
          pr[b].pb.fac_ns[p] = f.k <= 16 ? 1 : (f.k <= 32 ? 2 : 4);
        }
        if (f.k > kmax) {
          kmax = f.k;
          widest = f;
        }
        tabv.push_back(f);
      }
      BatchStep s;
      s.kind = BatchStep::FACTOR;
      s.fone = widest;
      s.grid = (int)tabv.size();
      s.tab_off = tb.add(tabv);
      steps.push_back(s);
    }
  };

  auto add_update = [&](int p) {
    for (auto& kv : ugroups[p]) {
      std::vector<UpdDev> segs;
      std::vector<int> map;
      UpdClass uc{};
      for (int b : kv.second) {
        uc = uclass(b, p);
        uc.dma = udma[p][kv.first] ? 1 : 0;
        UpdDev d;
        std::memset(&d, 0, sizeof(d));
        const bool first = p == 1;
        d.X = first ? (const void*)B[b].X : (const void*)B[b].Q;
        d.ldx = first ? B[b].ldx : B[b].ldq;
        d.m = B[b].m;
        if (uc.KYP) {
          d.Y = B[b].Y;
          d.ldy = B[b].ldy;
          d.ky = B[b].ky;
          d.kyp = (B[b].ky + 3) & ~3;
        }
        d.k = B[b].k;
        d.gE = uc.gr ? Lu[p][b].E : 0;
        d.zbase = 0;
        d.dense = svqb ? 1 : 0;
        d.Q = B[b].Q;
        d.ldq = B[b].ldq;
        d.part = uc.gr ? part + W[b].part : nullptr;
        d.npanels = (B[b].m + update_rows(uc.K, uc.KYP) - 1) / update_rows(uc.K, uc.KYP);
        d.C1 = ws + W[b].cp[p - 1];
        d.Z1 = ws + W[b].zp[p - 1];
        d.wg0 = (int)map.size();
        d.nwg = nwg_u[p][b];
        if (p <= 2) {
          PSweep& ps = pr[b].pb.sw[p];
          ps.kind = 2;
          ps.K = uc.K;
          ps.KYP = uc.KYP;
          ps.GR = uc.gr;
          ps.nw = persist_update_waves(uc.K, uc.KYP, uc.gr);
          ps.ntasks = d.nwg;
          ps.wg0 = d.wg0;
          pr[b].pb.nsweeps = p + 1;
          if (ps.nw < 1 || uc.two || uc.f32) persistable = false;
        }
        for (int i = 0; i < d.nwg; ++i) map.push_back((int)segs.size());
        segs.push_back(d);
      }
      BatchStep s;
      s.kind = BatchStep::UPDATE;
      s.uc = uc;
      s.grid = (int)map.size();
      s.tab_off = tb.add(segs);
      s.map_off = tb.add(map);
      for (int b : kv.second) {
        pr[b].tab_off[p] = s.tab_off;
        pr[b].map_off[p] = s.map_off;
      }
      steps.push_back(s);
    }
  };

  add_reduce(0, gmode);
  add_factor(0);
  for (int p = 1; p < passes; ++p) {
    add_update(p);
    add_reduce(p, 0);
    add_factor(p);
  }
  add_update(passes);

  // ---- upload the tables
  const size_t tbytes = std::max<size_t>(tb.b.size(), 256);
  if (hipMalloc((void**)&P->dtab, tbytes) != hipSuccess)
    return cleanup(BORTH_ERR_NOMEM, "batch table allocation failed");
  if (!tb.b.empty() &&
      hipMemcpy(P->dtab, tb.b.data(), tb.b.size(), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(BORTH_ERR_HIP, "batch table upload failed");
  P->steps = std::move(steps);
  P->bytes = (int64_t)tbytes + 8 * (wsz + psz) + 16 * (int64_t)nb;

  // ---- the persistent single launch
  if (persistable) {
    const int grid = batch_persistent_grid();
    std::vector<PBlock> hb(nb);
    std::vector<int> order(nb);
    std::vector<double> work(nb);
    for (int b = 0; b < nb; ++b) {
      hb[b] = pr[b].pb;
      for (int sw = 0; sw < hb[b].nsweeps; ++sw) {
        hb[b].sw[sw].tab = P->dtab + pr[b].tab_off[sw];
        hb[b].sw[sw].map = (const int*)(P->dtab + pr[b].map_off[sw]);
      }
      order[b] = b;
      work[b] = (double)B[b].m * (B[b].ky + B[b].k);
    }
    // larger blocks first: their long sweeps start early and the tail is
    // made of small blocks
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    const size_t sbytes = sizeof(int) * (size_t)batch_persistent_state_ints(nb);
    const size_t fbytes = sizeof(double) * (size_t)std::max(grid, 1) * kPersistFactorDoubles;
    if (grid >= 1 && hipMalloc((void**)&P->pblocks, sizeof(PBlock) * nb) == hipSuccess &&
        hipMalloc((void**)&P->porder, sizeof(int) * nb) == hipSuccess &&
        hipMalloc((void**)&P->pstate, sbytes) == hipSuccess &&
        hipMalloc((void**)&P->pscratch, fbytes) == hipSuccess &&
        hipMemcpy(P->pblocks, hb.data(), sizeof(PBlock) * nb, hipMemcpyHostToDevice) == hipSuccess &&
        hipMemcpy(P->porder, order.data(), sizeof(int) * nb, hipMemcpyHostToDevice) == hipSuccess) {
      P->persist = true;
      P->pgrid = grid;
      P->bytes += (int64_t)(sizeof(PBlock) * nb + sizeof(int) * nb + sbytes + fbytes);
    } else {
      return cleanup(BORTH_ERR_NOMEM, "batch: persistent plan allocation failed");
    }
  }
  *out = P;
  return BORTH_OK;
}

borth_status run_plan(borth_ctx c, BatchPlan* P, hipStream_t st) {
  c->cur = st;
  if (P->persist) {
    const int nb = P->nblocks;
    HIPCHK(c, launch_fill_int(P->status, 4 * nb, 0, st), "batch fill");
    prof_begin(c, 0);
    HIPCHK(c, launch_batch_persistent(P->pblocks, P->porder, nb, P->pstate, P->pscratch, P->pgrid, st),
           "batch persistent");
    prof_end(c, 0);
    return BORTH_OK;
  }
  for (const BatchStep& s : P->steps) {
    switch (s.kind) {
      case BatchStep::FILL:
        HIPCHK(c, launch_fill_int(P->status, s.fill_n, 0, st), "batch fill");
        break;
      case BatchStep::GRAM: {
        const GramSeg* tab = (const GramSeg*)(P->dtab + s.tab_off);
        const int* map = (const int*)(P->dtab + s.map_off);
        GramSeg none;
        std::memset(&none, 0, sizeof(none));
        prof_begin(c, 0);
        HIPCHK(c, launch_gram_segs(s.gkind, s.gmode, s.garg, s.shmem, s.grid, none, tab, map, st),
               "batch gram");
        prof_end(c, 0);
        break;
      }
      case BatchStep::REDUCE: {
        const ReduceSeg* tab = (const ReduceSeg*)(P->dtab + s.tab_off);
        ReduceSeg none;
        std::memset(&none, 0, sizeof(none));
        HIPCHK(c, launch_reduce_segs(s.gmode, s.red_nb, s.grid, none, tab, st), "batch reduce");
        break;
      }
      case BatchStep::FACTOR: {
        const FactorArgs* tab = (const FactorArgs*)(P->dtab + s.tab_off);
        HIPCHK(c, launch_factor_table(s.fone, tab, s.grid, st), "batch factor");
        break;
      }
      case BatchStep::UPDATE: {
        const UpdDev* tab = (const UpdDev*)(P->dtab + s.tab_off);
        const int* map = (const int*)(P->dtab + s.map_off);
        UpdDev none;
        std::memset(&none, 0, sizeof(none));
        prof_begin(c, 1);
        HIPCHK(c, launch_update_class(s.uc, s.grid, none, tab, map, st), "batch update");
        prof_end(c, 1);
        break;
      }
    }
  }
  return BORTH_OK;
}

GraphKey batch_key(borth_ctx c, int nb, const borth_block* B, const borth_opts& o) {
  GraphKey k;
  k.v.reserve(11 * (size_t)nb + 8);
  k.v.push_back(nb);
  k.v.push_back(o.gram);
  k.v.push_back(o.fact);
  k.v.push_back(o.passes);
  k.v.push_back(key_bits(o.shift));
  k.v.push_back((int64_t)(o.flags & ~(unsigned)BORTH_FLAG_SYNC));
  k.v.push_back((int64_t)c->tune_generation);
  for (int b = 0; b < nb; ++b) {
    const borth_block& x = B[b];
    k.v.insert(k.v.end(), {x.m, x.k, (int64_t)(intptr_t)x.X, x.ldx, (int64_t)(intptr_t)x.Y, x.ldy,
                           x.ky, (int64_t)(intptr_t)x.Q, x.ldq, (int64_t)(intptr_t)x.R,
                           (int64_t)(intptr_t)x.C});
  }
  return k;
}

uint64_t g_use_clock = 0;

}  // namespace

void batch_free_all(borth_ctx c) {
  for (auto& kv : c->plans) free_plan(kv.second);
  c->plans.clear();
}

// The device a tuning belongs to: architecture, compute units and HIP runtime
// version (a cache made elsewhere is refused on load).
static std::string tune_device_key(borth_ctx c) {
  hipDeviceProp_t p;
  std::string arch = "unknown";
  int cus = 0, rt = 0;
  if (hipGetDeviceProperties(&p, c->device) == hipSuccess) {
    arch = p.gcnArchName;
    cus = p.multiProcessorCount;
  }
  hipRuntimeGetVersion(&rt);
  for (char& ch : arch)
    if (ch == '"' || ch == '\\') ch = '_';
  return arch + "/" + std::to_string(cus) + "cu/hip" + std::to_string(rt);
}

extern "C" {

borth_status borth_batch_orthonormalize(borth_ctx c, int nblocks, const borth_block* blocks,
                                        const borth_opts* opts, borth_info* infos) {
  if (!c) return BORTH_ERR_ARG;
  borth_opts o;
  if (opts) o = *opts; else borth_default_opts(&o);
  if (nblocks < 0 || (nblocks > 0 && !blocks)) return fail_arg(c, "blocks");
  if (nblocks == 0) return BORTH_OK;
  if (o.passes < 1 || o.passes > 3) return fail_arg(c, "passes");
  if (!std::isfinite(o.shift)) return fail_arg(c, "shift");
  if (o.gram != BORTH_GRAM_F64 && o.gram != BORTH_GRAM_DD) {
    if (o.gram == BORTH_GRAM_SPLIT_BF16) {
      c->err = "the batched path takes binary64 blocks (no split-BF16 mode)";
      return BORTH_ERR_UNSUPPORTED;
    }
    return fail_arg(c, "opts.gram");
  }
  if (o.fact != BORTH_CHOL && o.fact != BORTH_SVQB) return fail_arg(c, "opts.fact");
  for (int b = 0; b < nblocks; ++b) {
    const borth_block& x = blocks[b];
    if (x.k < 1 || x.k > 64 || x.ky < 0 || x.ky > 16 || x.m < (int64_t)x.k + x.ky)
      return fail_arg(c, "block shape (1 <= k <= 64, 0 <= ky <= 16, m >= k + ky)");
    if (!x.X || !x.Q || x.ldx < x.k || x.ldq < x.k) return fail_arg(c, "block X/Q");
    if (x.ky > 0 && (!x.Y || x.ldy < x.ky)) return fail_arg(c, "block Y");
    if ((const void*)x.Q == (const void*)x.X && x.ldq != x.ldx) return fail_arg(c, "block aliasing");
  }
  hipSetDevice(c->device);
  const GraphKey key = batch_key(c, nblocks, blocks, o);
  BatchPlan* P = nullptr;
  auto it = c->plans.find(key);
  if (it != c->plans.end()) {
    P = it->second;
  } else {
    if ((int)c->plans.size() >= kMaxPlans) {
      // drop the least recently used plan
      HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
      auto lru = c->plans.begin();
      for (auto j = c->plans.begin(); j != c->plans.end(); ++j)
        if (j->second->last_use < lru->second->last_use) lru = j;
      free_plan(lru->second);
      c->plans.erase(lru);
    }
    borth_status r = build_plan(c, nblocks, blocks, o, &P);
    if (r) return r;
    c->plans.emplace(key, P);
  }
  P->last_use = ++g_use_clock;
  if (o.flags & BORTH_FLAG_GRAPH) {
    if (!P->graph) {
      if (!c->cap_stream)
        HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
      HIPCHK(c, hipStreamSynchronize(c->stream), "sync before capture");
      const hipError_t eb = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
      if (eb != hipSuccess) return fail_hip(c, eb, "hipStreamBeginCapture");
      c->capturing = true;
      borth_status r = run_plan(c, P, c->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
      c->capturing = false;
      c->cur = c->stream;
      if (r) {
        if (g) hipGraphDestroy(g);
        return r;
      }
      if (e != hipSuccess) return fail_hip(c, e, "hipStreamEndCapture");
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) return fail_hip(c, e, "hipGraphInstantiate");
      P->graph = ex;
    }
    HIPCHK(c, hipGraphLaunch(P->graph, c->stream), "hipGraphLaunch");
  } else {
    borth_status r = run_plan(c, P, c->stream);
    if (r) return r;
  }
  c->last_est = false;
  const bool log = [] {
    const char* e = std::getenv("BORTH_LOG");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  if (!infos && !(o.flags & BORTH_FLAG_SYNC)) {
    if (log)
      std::fprintf(stderr, "borth: batch nblocks=%d gram=%d fact=%d passes=%d flags=%u persistent=%d grid=%d (async)\n",
                   nblocks, o.gram, o.fact, o.passes, o.flags, P->persist ? 1 : 0, P->pgrid);
    return BORTH_OK;
  }
  HIPCHK(c, hipMemcpyAsync(P->h_status, P->status, sizeof(int) * 4 * (size_t)nblocks,
                           hipMemcpyDeviceToHost, c->stream),
         "status readback");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  borth_status first = BORTH_OK;
  for (int b = 0; b < nblocks; ++b) {
    const int* h = P->h_status + 4 * b;
    if (infos) {
      infos[b].status = h[0];
      infos[b].failed_pass = h[1];
      infos[b].failed_pivot = h[2];
      infos[b].passes_run = h[3];
      infos[b].orth_est = 0.0;
      infos[b].kappa_est = 0.0;
      infos[b].escalation = 0;
      infos[b].svqb_lifted = 0;
    }
    if (h[0] != 0 && first == BORTH_OK) first = (borth_status)h[0];
  }
  if (log)
    std::fprintf(stderr, "borth: batch nblocks=%d gram=%d fact=%d passes=%d flags=%u persistent=%d grid=%d -> status=%d\n",
                 nblocks, o.gram, o.fact, o.passes, o.flags, P->persist ? 1 : 0, P->pgrid, (int)first);
  return first;
}

// ---------------------------------------------------------------------------
// Autotuner: for every sweep kind and width class, time each candidate grid
// size on device-resident synthetic data and keep the fastest.  The
// library's own choice (nwg 0) is a candidate, so tuning never makes a sweep
// slower than the default; a winning explicit grid also sets the rows per
// workgroup share of the batched sweeps (rows of the tuning block / nwg: the
// per-workgroup row count the single-block sweep had).

namespace {

struct TuneEntry {
  std::string op;  // "gram" or "update"
  int mode;        // gram: 0 binary64, 1 DD; update: 0 plain, 1 with fused Gram
  int kp, hasy, nwg;
  double ms;
  int rows = 0;    // rows per workgroup of batched sweeps (0: default)
};

double median(std::vector<float> v) {
  std::sort(v.begin(), v.end());
  return v.empty() ? 0.0 : v[v.size() / 2];
}

}  // namespace

borth_status borth_autotune(borth_ctx c, const char* cache_path, int budget_ms) {
  if (!c) return BORTH_ERR_ARG;
  if (budget_ms < 1) return fail_arg(c, "budget_ms");
  hipSetDevice(c->device);
  const auto t0 = std::chrono::steady_clock::now();
  auto elapsed_ms = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  const int64_t m = 1 << 21;  // rows of the synthetic block (2M)
  double *X = nullptr, *Y = nullptr, *Q = nullptr, *part = nullptr, *zw = nullptr;
  const int cand[] = {0, 256, 512, 1024, 1536, 2048, 4096};
  const int64_t part_n = 4096LL * 2 * 16 * 210;  // largest: DD, Wp = 80
  borth_status res = BORTH_OK;
  std::vector<TuneEntry> found;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  do {
    if (hipMalloc((void**)&X, sizeof(double) * m * 64) != hipSuccess ||
        hipMalloc((void**)&Y, sizeof(double) * m * 16) != hipSuccess ||
        hipMalloc((void**)&Q, sizeof(double) * m * 64) != hipSuccess ||
        hipMalloc((void**)&part, sizeof(double) * part_n) != hipSuccess ||
        hipMalloc((void**)&zw, sizeof(double) * 2 * 64 * 64) != hipSuccess) {
      c->err = "autotune allocation failed";
      res = BORTH_ERR_NOMEM;
      break;
    }
    // 0x3ff00000 in both words: every double is 1 + 2^-32 + ..., a normal number
    if (launch_fill_int((int*)X, (int)(2 * m * 64), 0x3ff00000, c->stream) != hipSuccess ||
        launch_fill_int((int*)Y, (int)(2 * m * 16), 0x3ff00000, c->stream) != hipSuccess ||
        launch_fill_int((int*)zw, 2 * 2 * 64 * 64, 0x3ff00000, c->stream) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      res = fail_hip(c, hipGetLastError(), "autotune setup");
      break;
    }
    const int kps[] = {8, 16, 32, 64};
    bool out_of_time = false;
    for (int op = 0; op < 2 && !out_of_time; ++op)
      for (int mode = 0; mode < 2 && !out_of_time; ++mode)
        for (int kp : kps)
          for (int hasy = 0; hasy < 2; ++hasy) {
            if (elapsed_ms() > budget_ms) {
              out_of_time = true;
              break;
            }
            const int ky = hasy ? 16 : 0;
            double best = 1e30;
            int best_nwg = -1;
            for (int nwg : cand) {
              std::vector<float> ts;
              for (int rep = 0; rep < 4; ++rep) {
                hipError_t e = hipEventRecord(e0, c->stream);
                if (op == 0) {
                  Src s{hasy ? Y : nullptr, 16, X, 64, 0, m};
                  GramLayout L = make_layout(ky, kp, 4);
                  int used = 0;
                  if (e == hipSuccess)
                    e = launch_gram(s, L, mode, part, part_n, &used, TuneGram{nwg, 0}, c->stream);
                } else {
                  UpdateArgs u;
                  std::memset(&u, 0, sizeof(u));
                  u.src = Src{hasy ? Y : nullptr, 16, X, 64, 0, m};
                  u.C1 = zw;
                  u.Z1 = zw;
                  u.gram_with_y = mode && hasy;
                  u.Q = Q;
                  u.ldq = 64;
                  u.partials = mode ? part : nullptr;
                  u.partial_cap_doubles = part_n;
                  GramLayout L = make_layout(ky, kp, kp);
                  if (e == hipSuccess) e = launch_update(u, L, TuneGram{nwg, 0}, c->stream);
                }
                if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                  res = fail_hip(c, e, "autotune run");
                  break;
                }
                if (rep > 0) ts.push_back(ms);  // first run warms up
              }
              if (res) break;
              const double t = median(ts);
              if (t < best) {
                best = t;
                best_nwg = nwg;
              }
            }
            if (res) break;
            if (best_nwg < 0) continue;
            TuneEntry te{op == 0 ? "gram" : "update", mode, kp, hasy, best_nwg, best};
            te.rows = best_nwg > 0 ? (int)((m + best_nwg - 1) / best_nwg) : 0;
            found.push_back(te);
          }
  } while (false);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(c->stream);
  if (X) hipFree(X);
  if (Y) hipFree(Y);
  if (Q) hipFree(Q);
  if (part) hipFree(part);
  if (zw) hipFree(zw);
  if (res) return res;
  for (const TuneEntry& t : found) {
    auto& tab = t.op == "gram" ? c->tune_gram : c->tune_upd;
    tab[std::make_tuple(t.mode, t.kp, t.hasy)] = TuneGram{t.nwg, t.rows};
  }
  ++c->tune_generation;
  ++c->ws_generation;  // cached single-block graphs were captured with the old shapes
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "w");
    if (!f) {
      c->err = std::string("cannot write ") + cache_path;
      return BORTH_ERR_ARG;
    }
    std::fprintf(f, "{\"version\": 2, \"device\": \"%s\", \"rows\": %lld, \"entries\": [\n",
                 tune_device_key(c).c_str(), (long long)m);
    for (size_t i = 0; i < found.size(); ++i) {
      const TuneEntry& t = found[i];
      std::fprintf(f, "{\"op\": \"%s\", \"mode\": %d, \"kp\": %d, \"hasy\": %d, \"nwg\": %d, \"ms\": %.6f, \"rows\": %d}%s\n",
                   t.op.c_str(), t.mode, t.kp, t.hasy, t.nwg, t.ms, t.rows,
                   i + 1 < found.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
  }
  return BORTH_OK;
}

borth_status borth_autotune_load(borth_ctx c, const char* cache_path) {
  if (!c) return BORTH_ERR_ARG;
  if (!cache_path) return fail_arg(c, "cache_path");
  FILE* f = std::fopen(cache_path, "r");
  if (!f) {
    c->err = std::string("cannot read ") + cache_path;
    return BORTH_ERR_ARG;
  }
  char line[512];
  int n = 0;
  std::vector<TuneEntry> got;
  const std::string here = tune_device_key(c);
  while (std::fgets(line, sizeof(line), f)) {
    if (const char* dp = std::strstr(line, "\"device\": \"")) {
      dp += std::strlen("\"device\": \"");
      const char* de = std::strchr(dp, '"');
      const std::string made(dp, de ? (size_t)(de - dp) : std::strlen(dp));
      if (made != here) {
        std::fclose(f);
        c->err = "autotune cache made on " + made + ", this device is " + here;
        return BORTH_ERR_ARG;
      }
      continue;
    }
    char op[16] = {0};
    TuneEntry t;
    t.rows = 0;
    if (std::sscanf(line, " {\"op\": \"%15[a-z]\", \"mode\": %d, \"kp\": %d, \"hasy\": %d, \"nwg\": %d, \"ms\": %lf",
                    op, &t.mode, &t.kp, &t.hasy, &t.nwg, &t.ms) == 6) {
      t.op = op;
      const char* rp = std::strstr(line, "\"rows\":");
      if (rp && (std::sscanf(rp, "\"rows\": %d", &t.rows) != 1 || t.rows < 0)) {
        std::fclose(f);
        c->err = "malformed autotune entry";
        return BORTH_ERR_ARG;
      }
      // nwg 0: the library's own choice
      if ((t.op != "gram" && t.op != "update") || t.mode < 0 || t.mode > 1 || t.nwg < 0 ||
          t.nwg > (1 << 20)) {
        std::fclose(f);
        c->err = "malformed autotune entry";
        return BORTH_ERR_ARG;
      }
      got.push_back(t);
      ++n;
    }
  }
  std::fclose(f);
  if (n == 0) {
    c->err = "no autotune entries found";
    return BORTH_ERR_ARG;
  }
  for (const TuneEntry& t : got) {
    if (t.nwg > kMaxSweepWG) {
      c->err = "autotune entry above the workgroup limit";
      return BORTH_ERR_ARG;
    }
  }
  for (const TuneEntry& t : got) {
    auto& tab = t.op == "gram" ? c->tune_gram : c->tune_upd;
    tab[std::make_tuple(t.mode, t.kp, t.hasy)] = TuneGram{t.nwg, t.rows};
  }
  ++c->tune_generation;
  ++c->ws_generation;
  return BORTH_OK;
}

}  // extern "C"
