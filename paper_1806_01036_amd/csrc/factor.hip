// Small k x k step of phase II (Sec. 4.2): from the Gram matrix of [Y | X]
// form the projected Gram matrix M = Xt^T Xt, factor it and build the
// transform Z with Z^T M Z = I.  Sec. 4.2 counts the work on these small
// matrices as negligible next to the sweeps, also in extended precision; on
// the GPU their cost is latency, so they run in one workgroup per block
// without leaving the device.
//
// chol_kernel (Cholesky, DD or binary64 arithmetic): one workgroup of
//   T x T threads (T = 8, 16, 32, or 24 / 32 with 2 x 2 elements a thread);
//   LDL^T elimination on [M | I] keeps R and R^{-1} in one array, one
//   barrier per eliminated column (details at the kernel).
//   Breakdown rule: unpivoted; a pivot that is not > 0 or not finite stops
//   the factorization and reports its 1-based index (LAPACK potrf style).
// svqb_kernel (binary64), svqb_dd_kernel (DD): cyclic Jacobi with parallel round-robin rotations,
//   Z = U L^{-1/2} U^T (the Procrustes-optimal, symmetric form) and
//   R = U L^{1/2} U^T; eigenvalues below tau * lambda_max (tau = 2^-52) are
//   lifted to tau * lambda_max (rank-deficient blocks stay finite).
#include "dd.hpp"
#include "factor_impl.hpp"
#include "internal.hpp"

namespace borth {

using namespace fct;

namespace {

template <bool DD, int T, int NS>
__global__ void __launch_bounds__(T * T) chol_kernel(FactorArgs one,
                                                     const FactorArgs* __restrict__ tab) {
  constexpr int KP = T * NS;
  __shared__ double s_r0[2 * 64 * 65];
  __shared__ double s_r1[2 * 64 * 65];
  __shared__ double s_row[2 * 2 * KP];
  __shared__ double s_piv[2 * 64];
  __shared__ int s_flag;
  __shared__ double s_dinv[4];
  const FactorArgs a = tab ? tab[blockIdx.x] : one;
  chol_body<DD, T, NS>(a, CholMem{s_r0, s_r1, s_row, s_piv, &s_flag, s_dinv});
}

// ---------------------------------------------------------------------------
// SVQB (binary64): M in LDS, cyclic Jacobi with round-robin parallel pairs.
__global__ void __launch_bounds__(NTF) svqb_kernel(FactorArgs one,
                                                   const FactorArgs* __restrict__ tab) {
  const FactorArgs a = tab ? tab[blockIdx.x] : one;
  if (stopped(a.stop, a.pass)) return;
  __shared__ double sM[64 * 65];
  __shared__ double sV[64 * 65];
  __shared__ double sC[64 * 65];
  __shared__ double sc[32], ss[32];
  __shared__ int sp[32], sq[32];
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  const int k = a.k, ky = a.ky, W = a.ky + a.k, kp = a.kp;
  const int LD = 65;
  if (a.status[0] != 0) {
    for (int e = tid; e < kp * kp; e += NTF) a.Zp[e] = 0.0;
    return;
  }
  // M = G_XX - C^T (2C - S C) in binary64 (hi + lo folded), in three
  // parallel steps through LDS: S and C staged, D = 2C - S C (one thread per
  // element of D), then M (one thread per element of M); every element is
  // the same fused multiply-add chain, in the same order, as one thread
  // computing it alone.
  auto g = [&](int r, int c) { return a.G_hi[r * W + c] + (a.G_lo ? a.G_lo[r * W + c] : 0.0); };
  for (int e = tid; e < ky * ky; e += NTF) sM[(e / ky) * LD + e % ky] = g(e / ky, e % ky);
  for (int e = tid; e < ky * k; e += NTF) sC[(e / k) * LD + e % k] = g(e / k, ky + e % k);
  __syncthreads();
  for (int e = tid; e < ky * k; e += NTF) {
    const int r = e / k, l = e - r * k;
    double sc2 = 0.0;
    for (int q = 0; q < ky; ++q) sc2 = __builtin_fma(sM[r * LD + q], sC[q * LD + l], sc2);
    sV[r * LD + l] = 2.0 * sC[r * LD + l] - sc2;
  }
  __syncthreads();
  double mv[(64 * 64 + NTF - 1) / NTF];
#pragma unroll
  for (int u = 0; u < (64 * 64 + NTF - 1) / NTF; ++u) {
    const int e = tid + u * NTF;
    if (e < k * k) {
      const int i = e / k, l = e - i * k;
      double v = g(ky + i, ky + l);
      for (int r = 0; r < ky; ++r) v = __builtin_fma(-sC[r * LD + i], sV[r * LD + l], v);
      mv[u] = v;
    }
  }
  __syncthreads();  // D is read; sM and sV are free
#pragma unroll
  for (int u = 0; u < (64 * 64 + NTF - 1) / NTF; ++u) {
    const int e = tid + u * NTF;
    if (e < k * k) {
      const int i = e / k, l = e - i * k;
      sM[i * LD + l] = mv[u];
      sV[i * LD + l] = (i == l) ? 1.0 : 0.0;
    }
  }
  if (tid == 0) s_flag = 0;
  __syncthreads();
  for (int e = tid; e < k * k; e += NTF)
    if (!isfinite(sM[(e / k) * LD + e % k])) s_flag = 1;
  __syncthreads();
  if (s_flag) {
    if (tid == 0) {
      a.status[0] = 5;
      a.status[1] = a.pass + 1;
      a.status[2] = 0;
      if (a.stop) a.stop[0] = a.pass + 1;
    }
    for (int e = tid; e < kp * kp; e += NTF) a.Zp[e] = 0.0;
    return;
  }
  if (a.shift_rel > 0.0) {
    if (tid == 0) {
      double tr = 0.0;
      for (int i = 0; i < k; ++i) tr += sM[i * LD + i];
      for (int i = 0; i < k; ++i) sM[i * LD + i] += a.shift_rel * tr;
    }
    __syncthreads();
  }
  // Round-robin ordering on n = k rounded up to even; index n-1 is a dummy if k odd.
  const int n = (k + 1) & ~1;
  const int npair = n / 2;
  // Rotation rule (relative threshold of Demmel and Veselic 1992): rotate the
  // pair (p, q) only if |a_pq| > u sqrt(|a_pp a_qq|); the sweeps stop after
  // one with no rotation.  Off-diagonal entries at rounding level are left
  // alone, so converged sweeps do not feed rounding noise back into V.
  for (int sweep = 0; sweep < 30; ++sweep) {
    __syncthreads();  // every thread has read the previous sweep's flag
    if (tid == 0) s_flag = 0;
    __syncthreads();
    for (int step = 0; step < n - 1; ++step) {
      if (tid < npair) {
        // round-robin: position 0 fixed, others rotate
        int pp, qq;
        const int u = tid, v = n - 1 - tid;
        auto pos = [&](int x) { return x == 0 ? 0 : 1 + (x - 1 + step) % (n - 1); };
        pp = pos(u);
        qq = pos(v);
        if (pp > qq) { const int t = pp; pp = qq; qq = t; }
        double c = 1.0, s = 0.0;
        if (qq < k) {
          const double apq = sM[pp * LD + qq];
          const double app = sM[pp * LD + pp], aqq = sM[qq * LD + qq];
          if (fabs(apq) > 0x1p-53 * sqrt(fabs(app * aqq))) {
            s_flag = 1;
            const double theta = (sM[qq * LD + qq] - sM[pp * LD + pp]) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        sp[tid] = pp; sq[tid] = qq; sc[tid] = c; ss[tid] = s;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = tid; e < npair * k; e += NTF) {
        const int pr = e / k, r = e - pr * k;
        const int p = sp[pr], q = sq[pr];
        if (q >= k) continue;
        const double c = sc[pr], s = ss[pr];
        const double arp = sM[r * LD + p], arq = sM[r * LD + q];
        sM[r * LD + p] = c * arp - s * arq;
        sM[r * LD + q] = s * arp + c * arq;
        const double vrp = sV[r * LD + p], vrq = sV[r * LD + q];
        sV[r * LD + p] = c * vrp - s * vrq;
        sV[r * LD + q] = s * vrp + c * vrq;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < npair * k; e += NTF) {
        const int pr = e / k, r = e - pr * k;
        const int p = sp[pr], q = sq[pr];
        if (q >= k) continue;
        const double c = sc[pr], s = ss[pr];
        const double apr = sM[p * LD + r], aqr = sM[q * LD + r];
        sM[p * LD + r] = c * apr - s * aqr;
        sM[q * LD + r] = s * apr + c * aqr;
      }
      __syncthreads();
    }
    if (!s_flag) break;  // read after the last step's barrier, by every thread
  }
  // eigenvalues on the diagonal; lift tiny ones, or (rank revealing) keep
  // those above k u lambda_max in their order: perm[0..rank) kept, the rest
  // dropped
  __shared__ double lam[64];
  __shared__ int perm[64];
  __shared__ int s_rank;
  if (tid == 0) {
    double lmax = 0.0;
    for (int i = 0; i < k; ++i) lmax = fmax(lmax, sM[i * LD + i]);
    const double floor_ = lmax * 2.220446049250313e-16;
    double lmin = lmax;
    int nl = 0;
    for (int i = 0; i < k; ++i) {
      double l = sM[i * LD + i];
      if (!(l > floor_)) {
        l = floor_;
        ++nl;
      }
      lam[i] = l;
      lmin = fmin(lmin, l);
    }
    if (a.kappa) a.kappa[0] = sqrt(lmax / lmin);
    if (a.lifted && !a.rank_reveal && nl > *a.lifted) *a.lifted = nl;
    int r = 0;
    if (a.rank_reveal) {
      const double thr = lmax * k * 0x1p-52;
      for (int i = 0; i < k; ++i)
        if (sM[i * LD + i] > thr) perm[r++] = i;
      int q = r;
      for (int i = 0; i < k; ++i)
        if (!(sM[i * LD + i] > thr)) perm[q++] = i;
    } else {
      for (int i = 0; i < k; ++i) perm[i] = i;
      r = k;
    }
    s_rank = r;
    if (a.rank_reveal) a.status[4] = r;  // single-block status words only
  }
  __syncthreads();
  const int rank = s_rank;
  // Z and R_p: symmetric U L^{-1/2} U^T and U L^{1/2} U^T, or (rank
  // revealing) U_r L_r^{-1/2} and L_r^{1/2} U_r^T
  auto rp_entry = [&](int i, int j) -> double {
    if (a.rank_reveal) return i < rank ? sqrt(lam[perm[i]]) * sV[j * LD + perm[i]] : 0.0;
    double r = 0.0;
    for (int l = 0; l < k; ++l) r = __builtin_fma(sV[i * LD + l] * sV[j * LD + l], sqrt(lam[l]), r);
    return r;
  };
  for (int e = tid; e < kp * kp; e += NTF) {
    const int i = e / kp, j = e - i * kp;
    double z = 0.0;
    if (i < k && j < k) {
      if (a.rank_reveal) {
        z = j < rank ? sV[i * LD + perm[j]] / sqrt(lam[perm[j]]) : 0.0;
      } else {
        for (int l = 0; l < k; ++l) z = __builtin_fma(sV[i * LD + l] * sV[j * LD + l], 1.0 / sqrt(lam[l]), z);
      }
      if (a.Z_out) a.Z_out[i * k + j] = z;
      if (a.Rp_out) a.Rp_out[i * k + j] = rp_entry(i, j);
    }
    a.Zp[e] = z;
  }
  for (int e = tid; e < ky * kp; e += NTF) {
    const int l = e / kp, j = e - l * kp;
    a.Cp[e] = j < k ? a.G_hi[l * W + ky + j] + (a.G_lo ? a.G_lo[l * W + ky + j] : 0.0) : 0.0;
  }
  __syncthreads();
  // totals in binary64 (R_p dense): C_tot += C_p R_tot_old; R_tot = R_p R_tot_old
  const bool first = (a.pass == 0);
  // R_p into sM (reuse), computed from V and lam
  for (int e = tid; e < k * k; e += NTF) {
    const int i = e / k, j = e - i * k;
    sM[i * LD + j] = rp_entry(i, j);
  }
  __syncthreads();
  double cnew[16], rnew[16];
  int cnt = 0;
  for (int e = tid; e < ky * k && cnt < 16; e += NTF, ++cnt) {
    const int l = e / k, j = e - l * k;
    const double cp = a.G_hi[l * W + ky + j] + (a.G_lo ? a.G_lo[l * W + ky + j] : 0.0);
    double ct = first ? cp : a.Ctot[e];
    if (!first)
      for (int q = 0; q < k; ++q) ct = __builtin_fma(a.G_hi[l * W + ky + q] + (a.G_lo ? a.G_lo[l * W + ky + q] : 0.0), a.Rtot[q * k + j], ct);
    cnew[cnt] = ct;
  }
  cnt = 0;
  for (int e = tid; e < k * k && cnt < 16; e += NTF, ++cnt) {
    const int i = e / k, j = e - i * k;
    double s = 0.0;
    if (first) s = sM[i * LD + j];
    else
      for (int q = 0; q < k; ++q) s = __builtin_fma(sM[i * LD + q], a.Rtot[q * k + j], s);
    rnew[cnt] = s;
  }
  __syncthreads();
  cnt = 0;
  for (int e = tid; e < ky * k && cnt < 16; e += NTF, ++cnt) {
    a.Ctot[e] = cnew[cnt];
    a.Ctot[ky * k + e] = 0.0;
    if (a.C_out) a.C_out[e] = cnew[cnt];
  }
  cnt = 0;
  for (int e = tid; e < k * k && cnt < 16; e += NTF, ++cnt) {
    a.Rtot[e] = rnew[cnt];
    a.Rtot[k * k + e] = 0.0;
    if (a.R_out) a.R_out[e] = rnew[cnt];
  }
  if (a.conv) {
    // stop test of the iterated scheme: ||C_p||_F and ||R_p - I||_F (R_p is
    // in sM), summed in a fixed order
    double rr = 0.0, cc = 0.0;
    for (int e = tid; e < k * k; e += NTF) {
      const int i = e / k, j = e - i * k;
      const double d = sM[i * LD + j] - (i == j && i < rank ? 1.0 : 0.0);
      rr = __builtin_fma(d, d, rr);
    }
    for (int e = tid; e < ky * k; e += NTF) {
      const double v = a.G_hi[(e / k) * W + ky + e % k];
      cc = __builtin_fma(v, v, cc);
    }
    wg_reduce2<NTF, false>(rr, cc, sV);
    if (tid == 0) {
      const double sr = rr, sc = cc;
      a.conv[0] = sqrt(sc);
      a.conv[1] = sqrt(sr);
      // iterated scheme: this pass is the last one when both norms are small
      if (a.stop && sqrt(sc) <= a.stop_eps && sqrt(sr) <= a.stop_eps) a.stop[0] = a.pass + 1;
    }
  }
  if (tid == 0) a.status[3] = a.pass + 1;
}

// ---------------------------------------------------------------------------
// SVQB in DD (the DD variant of Sec. 4.2 with SVQB as phase II): the
// projected Gram matrix, the cyclic Jacobi eigensolver, Z = U L^{-1/2} U^T
// and R = U L^{1/2} U^T all in DD; eigenvalues below 2^-104 lambda_max are
// lifted to that floor.  The same round-robin structure as svqb_kernel; a
// pair is rotated when |a_pq| > 2^-105 sqrt(|a_pp a_qq|).  With the low words
// of Z and C requested (DD update), the projection coefficients are the
// corrected D = 2C - S C, as in chol_kernel.
__global__ void __launch_bounds__(NTF) svqb_dd_kernel(FactorArgs one,
                                                      const FactorArgs* __restrict__ tab) {
  using A = Ar<true>;
  const FactorArgs a = tab ? tab[blockIdx.x] : one;
  if (stopped(a.stop, a.pass)) return;
  constexpr int LD = 65;
  constexpr int NE = (64 * 64 + NTF - 1) / NTF;  // per-thread share of a 64 x 64 block
  __shared__ double sMh[64 * LD], sMl[64 * LD], sVh[64 * LD], sVl[64 * LD];
  __shared__ double rch[32], rcl[32], rsh[32], rsl[32];
  __shared__ int sp[32], sq[32];
  __shared__ double lh[64], ll[64], lrh[64], lrl[64], lsh[64], lsl[64];
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  const int k = a.k, ky = a.ky, W = a.ky + a.k, kp = a.kp;
  const bool corr = a.Cplo != nullptr;
  auto zero_out = [&]() {
    for (int e = tid; e < kp * kp; e += NTF) {
      a.Zp[e] = 0.0;
      if (a.Zplo) a.Zplo[e] = 0.0;
    }
  };
  if (a.status[0] != 0) {
    zero_out();
    return;
  }
  auto g = [&](int r, int c) { return ld_g(a.G_hi, a.G_lo, r * W + c); };
  auto ldm = [&](const double* h, const double* l, int i, int j) { return dd_make(h[i * LD + j], l[i * LD + j]); };
  auto stm = [&](double* h, double* l, int i, int j, dd_t v) {
    h[i * LD + j] = v.hi;
    l[i * LD + j] = v.lo;
  };

  // Projected Gram matrix M = G_XX - C^T D, D = 2C - S C (S = G_YY, C = G_YX):
  // S into sM and C into sV, then D, then M, each element one Dot2-style
  // accumulation.  cpv: this pass's coefficients (D corrected, else C).
  dd_t cpv[NE];
  if (ky > 0) {
    for (int e = tid; e < ky * ky; e += NTF) stm(sMh, sMl, e / ky, e % ky, g(e / ky, e % ky));
    for (int e = tid; e < ky * k; e += NTF) stm(sVh, sVl, e / k, e % k, g(e / k, ky + e % k));
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + u * NTF;
      cpv[u] = dd_from(0.0);
      if (e < ky * k) {
        const int r = e / k, l = e - r * k;
        const dd_t c = ldm(sVh, sVl, r, l);
        Acc<true> acc(dd_make(2.0 * c.hi, 2.0 * c.lo));
        for (int q = 0; q < ky; ++q) acc.add(dd_neg(ldm(sMh, sMl, r, q)), ldm(sVh, sVl, q, l));
        cpv[u] = acc.get();
      }
    }
    __syncthreads();  // S is read: D goes into sM
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + u * NTF;
      if (e < ky * k) stm(sMh, sMl, e / k, e % k, cpv[u]);
    }
    __syncthreads();
    dd_t mv[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + u * NTF;
      mv[u] = dd_from(0.0);
      if (e < k * k) {
        const int i = e / k, l = e - i * k;
        if (i <= l) {
          Acc<true> acc(g(ky + i, ky + l));
          for (int r = 0; r < ky; ++r) acc.add(dd_neg(ldm(sVh, sVl, r, i)), ldm(sMh, sMl, r, l));
          mv[u] = acc.get();
        }
      }
      if (!corr && e < ky * k) cpv[u] = ldm(sVh, sVl, e / k, e % k);  // plain C
    }
    __syncthreads();  // C and D are read
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + u * NTF;
      if (e < k * k) {
        const int i = e / k, l = e - i * k;
        if (i <= l) {
          stm(sMh, sMl, i, l, mv[u]);
          stm(sMh, sMl, l, i, mv[u]);
        }
      }
    }
  } else {
    for (int e = tid; e < k * k; e += NTF) {
      const int i = e / k, l = e - i * k;
      if (i <= l) {
        const dd_t v = g(i, l);
        stm(sMh, sMl, i, l, v);
        stm(sMh, sMl, l, i, v);
      }
    }
  }
  for (int e = tid; e < k * k; e += NTF) stm(sVh, sVl, e / k, e % k, dd_from((e / k) == (e % k) ? 1.0 : 0.0));
  if (tid == 0) s_flag = 0;
  __syncthreads();
  for (int e = tid; e < k * k; e += NTF)
    if (!isfinite(sMh[(e / k) * LD + e % k]) || !isfinite(sMl[(e / k) * LD + e % k])) s_flag = 1;
  __syncthreads();
  if (s_flag) {
    if (tid == 0) {
      a.status[0] = 5;
      a.status[1] = a.pass + 1;
      a.status[2] = 0;
      if (a.stop) a.stop[0] = a.pass + 1;
    }
    zero_out();
    return;
  }
  if (a.shift_rel > 0.0) {
    if (tid == 0) {
      double tr = 0.0;
      for (int i = 0; i < k; ++i) tr += sMh[i * LD + i];
      for (int i = 0; i < k; ++i) stm(sMh, sMl, i, i, A::add(ldm(sMh, sMl, i, i), dd_from(a.shift_rel * tr)));
    }
    __syncthreads();
  }

  // Jacobi sweeps in DD.  Rank revealing after the first pass: the input
  // is a binary64 Q with r orthonormal columns, whose Gram matrix is I_r + 0
  // up to binary64 rounding; pairs below that level are not rotated, so
  // the (nearly equal) kept eigenvalues are not mixed and Q's columns stay
  // in place (the non-symmetric Z = U_r L_r^{-1/2} is not invariant to such
  // rotations, unlike the symmetric form).
  const int n = (k + 1) & ~1;
  const int npair = n / 2;
  const double rot_thr = (a.rank_reveal && a.pass > 0) ? 0x1p-53 : 0x1p-105;
  for (int sweep = 0; sweep < 40; ++sweep) {
    __syncthreads();
    if (tid == 0) s_flag = 0;
    __syncthreads();
    for (int step = 0; step < n - 1; ++step) {
      if (tid < npair) {
        const int u = tid, v = n - 1 - tid;
        auto pos = [&](int x) { return x == 0 ? 0 : 1 + (x - 1 + step) % (n - 1); };
        int pp = pos(u), qq = pos(v);
        if (pp > qq) {
          const int t = pp;
          pp = qq;
          qq = t;
        }
        dd_t c = dd_from(1.0), sn = dd_from(0.0);
        if (qq < k) {
          const dd_t apq = ldm(sMh, sMl, pp, qq);
          const dd_t app = ldm(sMh, sMl, pp, pp), aqq = ldm(sMh, sMl, qq, qq);
          if (fabs(apq.hi) > rot_thr * sqrt(fabs(app.hi * aqq.hi))) {
            s_flag = 1;
            const dd_t theta = dd_div(A::sub(aqq, app), A::add(apq, apq));
            const dd_t at = theta.hi >= 0 ? theta : dd_neg(theta);
            const dd_t den = A::add(at, A::sqrt_(A::add(A::mul(theta, theta), dd_from(1.0))));
            dd_t t = A::recip(den);
            if (theta.hi < 0) t = dd_neg(t);
            c = A::rsqrt(A::add(A::mul(t, t), dd_from(1.0)));
            sn = A::mul(t, c);
          }
        }
        sp[tid] = pp;
        sq[tid] = qq;
        rch[tid] = c.hi;
        rcl[tid] = c.lo;
        rsh[tid] = sn.hi;
        rsl[tid] = sn.lo;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J (pairs without a rotation are skipped: J = I)
      for (int e = tid; e < npair * k; e += NTF) {
        const int pr = e / k, r = e - pr * k;
        const int p = sp[pr], q = sq[pr];
        if (q >= k || (rsh[pr] == 0.0 && rsl[pr] == 0.0)) continue;
        const dd_t c = dd_make(rch[pr], rcl[pr]), sn = dd_make(rsh[pr], rsl[pr]);
        const dd_t arp = ldm(sMh, sMl, r, p), arq = ldm(sMh, sMl, r, q);
        stm(sMh, sMl, r, p, A::sub(A::mul(c, arp), A::mul(sn, arq)));
        stm(sMh, sMl, r, q, A::add(A::mul(sn, arp), A::mul(c, arq)));
        const dd_t vrp = ldm(sVh, sVl, r, p), vrq = ldm(sVh, sVl, r, q);
        stm(sVh, sVl, r, p, A::sub(A::mul(c, vrp), A::mul(sn, vrq)));
        stm(sVh, sVl, r, q, A::add(A::mul(sn, vrp), A::mul(c, vrq)));
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < npair * k; e += NTF) {
        const int pr = e / k, r = e - pr * k;
        const int p = sp[pr], q = sq[pr];
        if (q >= k || (rsh[pr] == 0.0 && rsl[pr] == 0.0)) continue;
        const dd_t c = dd_make(rch[pr], rcl[pr]), sn = dd_make(rsh[pr], rsl[pr]);
        const dd_t apr = ldm(sMh, sMl, p, r), aqr = ldm(sMh, sMl, q, r);
        stm(sMh, sMl, p, r, A::sub(A::mul(c, apr), A::mul(sn, aqr)));
        stm(sMh, sMl, q, r, A::add(A::mul(sn, apr), A::mul(c, aqr)));
      }
      __syncthreads();
    }
    if (!s_flag) break;
  }
  // eigenvalues, lifted to 2^-104 lambda_max, or (rank revealing) those
  // above k 2^-104 lambda_max kept in their order (perm[0..rank)); their
  // square roots and reciprocal square roots
  __shared__ int perm[64];
  __shared__ int s_rank;
  if (tid == 0) {
    double lmax = 0.0;
    for (int i = 0; i < k; ++i) lmax = fmax(lmax, sMh[i * LD + i]);
    const double floor_ = lmax * 0x1p-104;
    double lmin = lmax;
    int nl = 0;
    for (int i = 0; i < k; ++i) {
      dd_t l = ldm(sMh, sMl, i, i);
      if (!(l.hi > floor_)) {
        l = dd_from(floor_);
        ++nl;
      }
      lh[i] = l.hi;
      ll[i] = l.lo;
      lmin = fmin(lmin, l.hi);
    }
    if (a.kappa) a.kappa[0] = sqrt(lmax / lmin);
    if (a.lifted && !a.rank_reveal && nl > *a.lifted) *a.lifted = nl;
    int r = 0;
    if (a.rank_reveal) {
      const double thr = lmax * k * 0x1p-104;
      for (int i = 0; i < k; ++i)
        if (sMh[i * LD + i] > thr) perm[r++] = i;
      int q = r;
      for (int i = 0; i < k; ++i)
        if (!(sMh[i * LD + i] > thr)) perm[q++] = i;
    } else {
      for (int i = 0; i < k; ++i) perm[i] = i;
      r = k;
    }
    s_rank = r;
    if (a.rank_reveal) a.status[4] = r;  // single-block status words only
  }
  __syncthreads();
  const int rank = s_rank;
  if (tid < k) {
    const dd_t l = dd_make(lh[tid], ll[tid]);
    const dd_t rs = A::rsqrt(l), sq_ = A::sqrt_(l);
    lrh[tid] = rs.hi;
    lrl[tid] = rs.lo;
    lsh[tid] = sq_.hi;
    lsl[tid] = sq_.lo;
  }
  __syncthreads();
  // Z and R_p
  dd_t rv[NE];
  for (int e = tid; e < kp * kp; e += NTF) {
    const int i = e / kp, j = e - i * kp;
    dd_t z = dd_from(0.0);
    if (i < k && j < k) {
      if (a.rank_reveal) {
        if (j < rank) z = A::mul(ldm(sVh, sVl, i, perm[j]), dd_make(lrh[perm[j]], lrl[perm[j]]));
      } else {
        Acc<true> az(dd_from(0.0));
        for (int l = 0; l < k; ++l)
          az.add(A::mul(ldm(sVh, sVl, i, l), ldm(sVh, sVl, j, l)), dd_make(lrh[l], lrl[l]));
        z = az.get();
      }
      if (a.Z_out) a.Z_out[i * k + j] = z.hi;
    }
    const double zr = z.hi + z.lo;
    a.Zp[e] = zr;
    if (a.Zplo) a.Zplo[e] = (z.hi - zr) + z.lo;
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + u * NTF;
    rv[u] = dd_from(0.0);
    if (e < k * k) {
      const int i = e / k, j = e - i * k;
      if (a.rank_reveal) {
        if (i < rank) rv[u] = A::mul(dd_make(lsh[perm[i]], lsl[perm[i]]), ldm(sVh, sVl, j, perm[i]));
      } else {
        Acc<true> ar(dd_from(0.0));
        for (int l = 0; l < k; ++l)
          ar.add(A::mul(ldm(sVh, sVl, i, l), ldm(sVh, sVl, j, l)), dd_make(lsh[l], lsl[l]));
        rv[u] = ar.get();
      }
      if (a.Rp_out) a.Rp_out[e] = rv[u].hi;
    }
  }
  __syncthreads();  // V is read: R_p into sM, C_p into sV
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + u * NTF;
    if (e < k * k) stm(sMh, sMl, e / k, e % k, rv[u]);
    if (e < ky * k) stm(sVh, sVl, e / k, e % k, cpv[u]);
  }
  __syncthreads();
  // C of this pass for the update (rounded, and the remainder for a DD update)
  for (int e = tid; e < ky * kp; e += NTF) {
    const int r = e / kp, j = e - r * kp;
    const dd_t v = j < k ? ldm(sVh, sVl, r, j) : dd_from(0.0);
    const double cr = v.hi + v.lo;
    a.Cp[e] = cr;
    if (a.Cplo) a.Cplo[e] = (v.hi - cr) + v.lo;
  }
  // totals in DD: C_tot += C_p R_tot_old, R_tot = R_p R_tot_old
  const bool first = (a.pass == 0);
  dd_t cn[NE], rn[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + u * NTF;
    cn[u] = rn[u] = dd_from(0.0);
    if (e < ky * k) {
      const int l = e / k, j = e - l * k;
      if (first) {
        cn[u] = ldm(sVh, sVl, l, j);
      } else {
        Acc<true> acc(dd_make(a.Ctot[e], a.Ctot[ky * k + e]));
        for (int q = 0; q < k; ++q)
          acc.add(ldm(sVh, sVl, l, q), dd_make(a.Rtot[q * k + j], a.Rtot[k * k + q * k + j]));
        cn[u] = acc.get();
      }
    }
    if (e < k * k) {
      const int i = e / k, j = e - i * k;
      if (first) {
        rn[u] = ldm(sMh, sMl, i, j);
      } else {
        Acc<true> acc(dd_from(0.0));
        for (int q = 0; q < k; ++q)
          acc.add(ldm(sMh, sMl, i, q), dd_make(a.Rtot[q * k + j], a.Rtot[k * k + q * k + j]));
        rn[u] = acc.get();
      }
    }
  }
  __syncthreads();  // every thread has read the old totals
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + u * NTF;
    if (e < ky * k) {
      a.Ctot[e] = cn[u].hi;
      a.Ctot[ky * k + e] = cn[u].lo;
      if (a.C_out) a.C_out[e] = cn[u].hi;
    }
    if (e < k * k) {
      a.Rtot[e] = rn[u].hi;
      a.Rtot[k * k + e] = rn[u].lo;
      if (a.R_out) a.R_out[e] = rn[u].hi;
    }
  }
  if (a.conv) {
    double rr = 0.0, cc = 0.0;
    for (int e = tid; e < k * k; e += NTF) {
      const int i = e / k, j = e - i * k;
      const double d = sMh[i * LD + j] - (i == j && i < rank ? 1.0 : 0.0);
      rr = __builtin_fma(d, d, rr);
    }
    for (int e = tid; e < ky * k; e += NTF) {
      const double v = a.G_hi[(e / k) * W + ky + e % k];
      cc = __builtin_fma(v, v, cc);
    }
    wg_reduce2<NTF, false>(rr, cc, sVh);
    if (tid == 0) {
      const double sr = rr, sc = cc;
      a.conv[0] = sqrt(sc);
      a.conv[1] = sqrt(sr);
      // iterated scheme: this pass is the last one when both norms are small
      if (a.stop && sqrt(sc) <= a.stop_eps && sqrt(sr) <= a.stop_eps) a.stop[0] = a.pass + 1;
    }
  }
  if (tid == 0) a.status[3] = a.pass + 1;
}

template <bool DD>
void launch_chol(const FactorArgs& a, const FactorArgs* tab, int n, hipStream_t st) {
  if (a.k <= 8)
    hipLaunchKernelGGL((chol_kernel<DD, 8, 1>), dim3(n), dim3(64), 0, st, a, tab);
  else if (a.k <= 16)
    hipLaunchKernelGGL((chol_kernel<DD, 16, 1>), dim3(n), dim3(256), 0, st, a, tab);
  else if (a.k <= 32)
    hipLaunchKernelGGL((chol_kernel<DD, 32, 1>), dim3(n), dim3(1024), 0, st, a, tab);
  else if (a.k <= 48)
    hipLaunchKernelGGL((chol_kernel<DD, 24, 2>), dim3(n), dim3(576), 0, st, a, tab);
  else
    hipLaunchKernelGGL((chol_kernel<DD, 32, 2>), dim3(n), dim3(1024), 0, st, a, tab);
}

}  // namespace

hipError_t launch_factor_table(const FactorArgs& a, const FactorArgs* tab, int n, hipStream_t st) {
  if (a.k > 64 || a.ky > 64 || a.k < 1 || n < 1) return hipErrorInvalidValue;
  if (a.fact == 1) {
    if (a.dd)
      hipLaunchKernelGGL(svqb_dd_kernel, dim3(n), dim3(NTF), 0, st, a, tab);
    else
      hipLaunchKernelGGL(svqb_kernel, dim3(n), dim3(NTF), 0, st, a, tab);
  } else if (a.dd) {
    launch_chol<true>(a, tab, n, st);
  } else {
    launch_chol<false>(a, tab, n, st);
  }
  return hipGetLastError();
}

hipError_t launch_factor(const FactorArgs& a, hipStream_t st) {
  return launch_factor_table(a, nullptr, 1, st);
}

}  // namespace borth
