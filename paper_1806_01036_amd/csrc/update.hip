// Basis update sweep (TSMM), the product of the projected block with Z
// (Sec. 4.2), with the phase-I projection folded in: T = (S - Y C) Z per
// row, S = X (first pass) or Q_1 (later passes); optionally a second stage
// and the next pass's Gram matrix fused in (matrix-core kernels in
// update_impl.hpp, one translation unit per padded width K).  Narrow
// single-stage sweeps without a fused Gram go to the vector-ALU stream kernel
// of update_narrow.hip.  This file holds the host-side dispatch.
#include "update_impl.hpp"

namespace borth {

int update_waves(int K, int KYP, bool dma) { return upd::upd_waves(K, KYP, 1, dma); }
int update_rows(int K, int KYP) { return upd::upd_rows(K, KYP); }

bool update_dma_ok(const UpdDev& d, int K, int KYP, bool f32, bool two) {
  if (!upd::upd_dma_class(K, KYP)) return false;
  if (upd::upd_zl(K)) {
    // one buffer per wave: single stage; rows of 16-byte chunks
    const int epc = f32 ? 4 : 2;
    if (two || (reinterpret_cast<uintptr_t>(d.X) & 15) || d.ldx % epc || d.k % epc) return false;
    if (d.ky > 0 && (f32 || (reinterpret_cast<uintptr_t>(d.Y) & 15) || (d.ldy & 1) || (d.ky & 1)))
      return false;
    return true;
  }
  if (f32) return false;
  if ((reinterpret_cast<uintptr_t>(d.X) & 15) || (d.ldx & 1) || (d.k & 1)) return false;
  if (d.ky > 0 && ((reinterpret_cast<uintptr_t>(d.Y) & 15) || (d.ldy & 1) || (d.ky & 1)))
    return false;
  return true;
}

GramLayout update_gram_layout(int ky, int k, int K, bool with_y) {
  GramLayout G;
  if (with_y) {
    G = make_layout(ky, k, K);
    G.kyp = 16;
    G.Wp = 16 + G.kp;
    G.T4 = G.Wp / 4;
    G.ntiles = G.T4 * (G.T4 + 1) / 2;
    G.E = 16 * G.ntiles;
  } else {
    G = make_layout(0, k, K);
  }
  return G;
}

hipError_t launch_update_class(const UpdClass& c, int grid, const UpdDev& one, const UpdDev* tab,
                               const int* wg2seg, hipStream_t st) {
  switch (c.K) {
    case 4: return launch_update_k4(c, grid, one, tab, wg2seg, st);
    case 8: return launch_update_k8(c, grid, one, tab, wg2seg, st);
    case 16: return launch_update_k16(c, grid, one, tab, wg2seg, st);
    case 32: return launch_update_k32(c, grid, one, tab, wg2seg, st);
    case 64: return launch_update_k64(c, grid, one, tab, wg2seg, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_update(UpdateArgs& a, const GramLayout& L, const TuneGram& tune,
                         hipStream_t st) {
  UpdDev d;
  d.Y = a.src.Y;
  d.ldy = a.src.ldy;
  d.X = a.src.X;
  d.ldx = a.src.ldx;
  d.m = a.src.m;
  d.ky = L.ky;
  d.kyp = L.kyp;
  d.k = L.k;
  const int K = L.kp;
  const int KYP = L.kyp == 0 ? 0 : (L.kyp <= 16 ? 16 : 64);
  // Fused Gram of [Y | T] (Y padded to 16 columns) or of T alone.
  const bool gy = a.gram_with_y && L.kyp > 0;
  if (a.partials && gy && L.kyp > 16) return hipErrorInvalidValue;
  const GramLayout G = update_gram_layout(L.ky, L.k, K, gy);
  d.gE = G.E;
  a.glayout = G;
  d.dense = a.dense;
  d.zbase = 0;
  d.Q = a.Q;
  d.ldq = a.ldq;
  d.Qlo = a.Qlo;
  d.Xlo = a.Xlo;
  d.part = a.partials;
  const int PR = upd::upd_rows(K, KYP);
  d.npanels = (a.src.m + PR - 1) / PR;
  d.C1 = a.C1;
  d.Z1 = a.Z1;
  d.C2 = a.C2;
  d.Z2 = a.Z2;
  d.C1lo = a.C1lo;
  d.Z1lo = a.Z1lo;
  d.bw = a.bw;
  d.stop = a.src.stop;
  d.pass = a.src.pass;
  if (a.bw && !(a.partials && a.gram_xcols)) return hipErrorInvalidValue;
  // DD arithmetic: the narrow kernel (k <= 8, with or without a DD result)
  // or the DD kernel (8 < k <= 64, DD result)
  if ((a.Qlo || a.Xlo) && !(a.C1lo && a.Z1lo)) return hipErrorInvalidValue;
  if ((a.C1lo || a.Z1lo) && (a.two_stage || a.src.x_f32)) return hipErrorInvalidValue;
  if ((a.C1lo || a.Z1lo) && !update_narrow_ok(L.k, L.ky, K)) {
    if (a.partials || !a.Q || !a.Qlo || !update_dd_ok(L.k, L.ky, K)) return hipErrorInvalidValue;
    a.nwg = 0;
    return launch_update_dd(d, K, st);
  }
  if (!a.partials && !a.two_stage && !a.src.x_f32 && a.Q && update_narrow_ok(L.k, L.ky, K)) {
    a.nwg = 0;
    return launch_update_narrow(d, K, st);
  }
  if (a.partials && a.gram_xcols) {
    // only the narrow kernel computes the Gram columns [Y | T]^T T
    if (a.two_stage || a.src.x_f32 || !a.Q || !update_narrow_gram_ok(d, K)) return hipErrorInvalidValue;
    a.glayout = make_layout_xcols(L.ky, L.k, 4);
    d.gE = a.glayout.E;
    const int64_t slots = a.partial_cap_doubles / ((int64_t)a.glayout.E * (a.gram_dd ? 2 : 1));
    return launch_update_narrow_gram(d, K, a.gram_dd, a.glayout, slots, &a.nwg, st);
  }
  const bool dma = update_dma_ok(d, K, KYP, a.src.x_f32 != 0, a.two_stage);
  const int NW = upd::upd_waves(K, KYP, a.two_stage ? 2 : 1, dma, a.src.x_f32 != 0);
  int nwg = tune.nwg > 0 ? tune.nwg : 1024;
  const int64_t need = (d.npanels + NW - 1) / NW;
  if (nwg > need) nwg = (int)(need > 0 ? need : 1);
  if (a.partials && (int64_t)nwg * G.E > a.partial_cap_doubles) return hipErrorInvalidValue;
  a.nwg = nwg;
  d.wg0 = 0;
  d.nwg = nwg;
  UpdClass c;
  c.K = K;
  c.KYP = KYP;
  c.two = a.two_stage ? 1 : 0;
  c.gr = !a.partials ? 0 : (gy ? 2 : 1);
  c.f32 = a.src.x_f32;
  c.dma = dma ? 1 : 0;
  return launch_update_class(c, nwg, d, nullptr, nullptr, st);
}


}  // namespace borth
