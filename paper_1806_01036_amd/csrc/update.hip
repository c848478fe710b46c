// Basis update sweep (TSMM), "Y = Xt Z" of Sec. 4.2 with the phase-I
// projection folded in:  T = (S - Y C) Z  per row, S = X (first pass) or
// Q_1 (later passes).  Optionally a second stage T = (T - Y C2) Z2 follows in
// registers (CholQR2 with Q_1 recomputed instead of stored), and the Gram
// matrix of [Y | T] needed by the next pass is accumulated from the values
// just computed ("kernel fusion ... to further reduce memory accesses",
// Sec. 4.2).
//
// Layout: a workgroup has NW waves; each wave owns a 64-row panel of [Y | S]
// in LDS (row stride Wp + 2 doubles: conflict-free 16-byte row reads).
//   1. coalesced global -> LDS load of the panel (zero-filled outside m, k, ky);
//   2. lane r computes row r: xt = s - y C (FMAs, C and Z are wave-uniform
//      and come through scalar loads), then t_j = sum_{i<=j} xt_i Z_ij (all i
//      for a dense Z), written back into the row;
//   3. coalesced LDS -> global store of T (if Q is given);
//   4. the Gram of [Y | T] over the panel on the matrix cores
//      (v_mfma_f64_16x16x4, operands read from LDS), accumulated per wave.
// The waves' Gram accumulators are summed in wave order at the end and
// written as one partial per workgroup (same tile layout as the Gram sweep).
#include "update_impl.hpp"

namespace borth {

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
  GramLayout G;
  if (gy) {
    G = make_layout(L.ky, L.k, K);
    G.kyp = 16;
    G.Wp = 16 + G.kp;
    G.T4 = G.Wp / 4;
    G.ntiles = G.T4 * (G.T4 + 1) / 2;
    G.E = 16 * G.ntiles;
  } else {
    G = make_layout(0, L.k, K);
  }
  d.gE = G.E;
  a.glayout = G;
  d.dense = a.dense;
  d.zbase = 0;
  d.Q = a.Q;
  d.ldq = a.ldq;
  d.part = a.partials;
  d.npanels = (a.src.m + 63) / 64;
  if (a.partials && gy && L.kyp > 16) return hipErrorInvalidValue;
  const int NW = upd::upd_waves(K, KYP);
  int nwg = tune.nwg > 0 ? tune.nwg : 1024;
  const int64_t need = (d.npanels + NW - 1) / NW;
  if (nwg > need) nwg = (int)(need > 0 ? need : 1);
  if (a.partials && (int64_t)nwg * G.E > a.partial_cap_doubles) return hipErrorInvalidValue;
  a.nwg = nwg;
  switch (K) {
    case 4: return launch_update_k4(d, a, nwg, st);
    case 8: return launch_update_k8(d, a, nwg, st);
    case 16: return launch_update_k16(d, a, nwg, st);
    case 32: return launch_update_k32(d, a, nwg, st);
    case 64: return launch_update_k64(d, a, nwg, st);
    default: return hipErrorInvalidValue;
  }
}


// W = -C Z for the public update entry point (C: ky x k, Z: k x k, both
// contiguous; W: ky x kp zero padded).  One thread per entry, binary64 FMAs.
__global__ void neg_cz_kernel(const double* __restrict__ C, const double* __restrict__ Z,
                              double* __restrict__ W, int ky, int k, int kp) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ky * kp) return;
  const int r = e / kp, j = e - r * kp;
  double s = 0.0;
  if (j < k)
    for (int i = 0; i < k; ++i) s = __builtin_fma(C[r * k + i], Z[i * k + j], s);
  W[e] = -s;
}

hipError_t launch_neg_cz(const double* C, const double* Z, double* W, int ky, int k, int kp,
                         hipStream_t st) {
  const int n = ky * kp;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(neg_cz_kernel, dim3((n + 255) / 256), dim3(256), 0, st, C, Z, W, ky, k, kp);
  return hipGetLastError();
}

}  // namespace borth
