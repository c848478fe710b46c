// Small k x k step of phase II (Sec. 4.2): from the Gram matrix of [Y | X]
// form the projected Gram matrix M = Xt^T Xt, factor it and build the
// transform Z with Z^T M Z = I.  "Operations on small n_b x n_b matrices are
// cost negligible, even in extended precision" (Sec. 4.2) -- on the GPU they
// are latency, so they run in one workgroup without leaving the device.
//
// factor_kernel (Cholesky, DD or binary64 arithmetic):
//   256 threads; element (i, l) of a k x k matrix (k <= 64) lives in the
//   registers of thread (i mod 16) * 16 + (l mod 16), slot (i / 16, l / 16).
//   Right-looking Cholesky and right-looking back substitution for R^{-1}
//   broadcast one row (and one column) per step through LDS.
//   Breakdown rule: unpivoted; a pivot that is not > 0 or not finite stops
//   the factorization and reports its 1-based index (LAPACK potrf style).
// svqb_kernel (binary64): cyclic Jacobi with parallel round-robin rotations,
//   Z = U L^{-1/2} U^T (the Procrustes-optimal, symmetric form) and
//   R = U L^{1/2} U^T; eigenvalues below tau * lambda_max (tau = 2^-52) are
//   lifted to tau * lambda_max (rank-deficient blocks stay finite).
#include "dd.hpp"
#include "internal.hpp"

namespace borth {

namespace {

constexpr int NTF = 256;

struct Dd16 {
  dd_t v[4][4];
};

__device__ __forceinline__ dd_t ld_g(const double* hi, const double* lo, int idx) {
  return dd_make(hi[idx], lo ? lo[idx] : 0.0);
}

// DD or binary64 operations selected at compile time (binary64 keeps lo = 0).
template <bool DD>
struct Ar {
  static __device__ __forceinline__ dd_t add(dd_t a, dd_t b) {
    return DD ? dd_add(a, b) : dd_from(a.hi + b.hi);
  }
  static __device__ __forceinline__ dd_t sub(dd_t a, dd_t b) {
    return DD ? dd_sub(a, b) : dd_from(a.hi - b.hi);
  }
  static __device__ __forceinline__ dd_t mul(dd_t a, dd_t b) {
    return DD ? dd_mul(a, b) : dd_from(a.hi * b.hi);
  }
  // a - b c
  static __device__ __forceinline__ dd_t fnms(dd_t a, dd_t b, dd_t c) {
    return DD ? dd_sub(a, dd_mul(b, c)) : dd_from(__builtin_fma(-b.hi, c.hi, a.hi));
  }
  static __device__ __forceinline__ dd_t sqrt_(dd_t a) {
    return DD ? dd_sqrt(a) : dd_from(sqrt(a.hi));
  }
  static __device__ __forceinline__ dd_t recip(dd_t a) {
    return DD ? dd_recip(a) : dd_from(1.0 / a.hi);
  }
  static __device__ __forceinline__ dd_t rsqrt(dd_t a) {
    return DD ? dd_rsqrt(a) : dd_from(1.0 / sqrt(a.hi));
  }
};

template <bool DD>
__global__ void __launch_bounds__(NTF) factor_kernel(FactorArgs a) {
  using A = Ar<DD>;
  __shared__ double s_rowh[64], s_rowl[64], s_colh[64], s_coll[64];
  __shared__ double s_rinvh[64], s_rinvl[64];
  __shared__ double s_ch[16][64], s_cl[16][64], s_dh[16][64], s_dl[16][64];
  __shared__ double s_red[NTF];
  __shared__ double s_rjj[2];
  __shared__ int s_fail;

  const int tid = threadIdx.x;
  const int ti = tid >> 4, tj = tid & 15;
  const int k = a.k, ky = a.ky, W = a.ky + a.k, kp = a.kp;

  // A previous pass already failed: leave a zero transform and stop.
  if (a.status[0] != 0) {
    for (int e = tid; e < kp * kp; e += NTF) a.Zp[e] = 0.0;
    return;
  }

  // Load M = G_XX.
  Dd16 M;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * p, l = tj + 16 * q;
      M.v[p][q] = (i < k && l < k) ? ld_g(a.G_hi, a.G_lo, (ky + i) * W + ky + l) : dd_from(0.0);
    }

  // Phase-I correction: M = G_XX - C^T (2C - S C), C = G_YX, S = G_YY.
  for (int c0 = 0; c0 < ky; c0 += 16) {
    __syncthreads();
    for (int e = tid; e < 16 * 64; e += NTF) {
      const int r = e >> 6, j = e & 63, l = c0 + r;
      dd_t cv = dd_from(0.0), dv = dd_from(0.0);
      if (l < ky && j < k) {
        cv = ld_g(a.G_hi, a.G_lo, l * W + ky + j);
        dd_t sc = dd_from(0.0);
        for (int q = 0; q < ky; ++q)
          sc = A::add(sc, A::mul(ld_g(a.G_hi, a.G_lo, l * W + q), ld_g(a.G_hi, a.G_lo, q * W + ky + j)));
        dv = A::sub(A::add(cv, cv), sc);
      }
      s_ch[r][j] = cv.hi; s_cl[r][j] = cv.lo;
      s_dh[r][j] = dv.hi; s_dl[r][j] = dv.lo;
    }
    __syncthreads();
    const int rn = (ky - c0) < 16 ? (ky - c0) : 16;
    for (int r = 0; r < rn; ++r) {
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = ti + 16 * p, l = tj + 16 * q;
          if (i < k && l < k)
            M.v[p][q] = A::fnms(M.v[p][q], dd_make(s_ch[r][i], s_cl[r][i]), dd_make(s_dh[r][l], s_dl[r][l]));
        }
    }
  }

  // Non-finite check and optional shift s = shift_rel * trace(M).
  {
    double part = 0.0;
    int bad = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ti + 16 * p, l = tj + 16 * q;
        if (i < k && l < k) {
          if (!isfinite(M.v[p][q].hi)) bad = 1;
          if (i == l) part += M.v[p][q].hi;
        }
      }
    if (tid == 0) s_fail = 0;
    __syncthreads();
    if (bad) s_fail = 1;
    s_red[tid] = part;
    __syncthreads();
    if (s_fail) {
      if (tid == 0) {
        a.status[0] = 5;
        a.status[1] = a.pass + 1;
        a.status[2] = 0;
      }
      for (int e = tid; e < kp * kp; e += NTF) a.Zp[e] = 0.0;
      return;
    }
    if (a.shift_rel > 0.0) {
      double tr = 0.0;
      for (int t = 0; t < NTF; ++t) tr += s_red[t];  // fixed order
      const double sh = a.shift_rel * tr;
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = ti + 16 * p, l = tj + 16 * q;
          if (i < k && i == l) M.v[p][q] = A::add(M.v[p][q], dd_from(sh));
        }
    }
  }

  // Right-looking Cholesky M = R^T R (upper R stored in place).
  for (int j = 0; j < k; ++j) {
    const int pj = j >> 4, jm = j & 15;
    __syncthreads();
    if (ti == jm && tj == jm) {
      dd_t d = M.v[pj][pj];
      if (!(d.hi > 0.0) || !isfinite(d.hi)) {
        s_fail = j + 1;
      } else {
        // 1/sqrt(d) by one Newton step from the binary64 seed, then
        // sqrt(d) = d / sqrt(d)
        const dd_t ri = A::rsqrt(d);
        const dd_t r = A::mul(d, ri);
        s_rinvh[j] = ri.hi;
        s_rinvl[j] = ri.lo;
        s_rjj[0] = r.hi;
        s_rjj[1] = r.lo;
      }
    }
    __syncthreads();
    if (s_fail) break;
    const dd_t rjj = dd_make(s_rjj[0], s_rjj[1]);
    const dd_t rinv = dd_make(s_rinvh[j], s_rinvl[j]);
    __syncthreads();
    if (ti == jm) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int l = tj + 16 * q;
        if (l < k) {
          dd_t v;
          if (l > j) v = A::mul(M.v[pj][q], rinv);
          else if (l == j) v = rjj;
          else v = dd_from(0.0);
          M.v[pj][q] = v;
          s_rowh[l] = v.hi;
          s_rowl[l] = v.lo;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = ti + 16 * p;
      if (i <= j || i >= k) continue;
      const dd_t ri = dd_make(s_rowh[i], s_rowl[i]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int l = tj + 16 * q;
        if (l >= i && l < k) M.v[p][q] = A::fnms(M.v[p][q], ri, dd_make(s_rowh[l], s_rowl[l]));
      }
    }
  }
  __syncthreads();
  if (s_fail) {
    if (tid == 0) {
      a.status[0] = 4;
      a.status[1] = a.pass + 1;
      a.status[2] = s_fail;
    }
    for (int e = tid; e < kp * kp; e += NTF) a.Zp[e] = 0.0;
    return;
  }
  // Zero the strictly lower part (it held unreduced values).
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (ti + 16 * p > tj + 16 * q) M.v[p][q] = dd_from(0.0);

  // Z = R^{-1} by right-looking back substitution: T = I; for i = k-1..0:
  // Z[i][:] = T[i][:] / R_ii, then T[i'][j] -= R[i'][i] Z[i][j] for i' < i.
  Dd16 Z;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) Z.v[p][q] = dd_from((ti + 16 * p == tj + 16 * q) ? 1.0 : 0.0);
  for (int i = k - 1; i >= 0; --i) {
    const int pi = i >> 4, im = i & 15;
    __syncthreads();
    const dd_t rinv = dd_make(s_rinvh[i], s_rinvl[i]);
    if (ti == im) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = tj + 16 * q;
        if (j < k) {
          const dd_t z = (j >= i) ? A::mul(Z.v[pi][q], rinv) : dd_from(0.0);
          Z.v[pi][q] = z;
          s_rowh[j] = z.hi;
          s_rowl[j] = z.lo;
        }
      }
    }
    if (tj == im) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int ip = ti + 16 * p;
        if (ip < k) {
          s_colh[ip] = M.v[p][pi].hi;
          s_coll[ip] = M.v[p][pi].lo;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int ip = ti + 16 * p;
      if (ip >= i || ip >= k) continue;
      const dd_t r = dd_make(s_colh[ip], s_coll[ip]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = tj + 16 * q;
        if (j >= i && j < k) Z.v[p][q] = A::fnms(Z.v[p][q], r, dd_make(s_rowh[j], s_rowl[j]));
      }
    }
  }

  // Outputs: padded Z (hi words), this pass's C (hi words), optional Z / R_p.
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * p, l = tj + 16 * q;
      if (i < kp && l < kp) a.Zp[i * kp + l] = (i < k && l < k) ? Z.v[p][q].hi : 0.0;
      if (i < k && l < k) {
        if (a.Z_out) a.Z_out[i * k + l] = Z.v[p][q].hi;
        if (a.Rp_out) a.Rp_out[i * k + l] = M.v[p][q].hi;
      }
    }
  for (int e = tid; e < ky * kp; e += NTF) {
    const int l = e / kp, j = e - l * kp;
    a.Cp[e] = j < k ? a.G_hi[l * W + ky + j] + (a.G_lo ? a.G_lo[l * W + ky + j] : 0.0) : 0.0;
  }
  // W = -C Z_hi (in DD, rounded): the update applies (S - Y C) Z_hi as
  // S Z_hi + Y W.
  __syncthreads();
  for (int e = tid; e < ky * kp; e += NTF) {
    const int l = e / kp, j = e - l * kp;
    dd_t w = dd_from(0.0);
    if (j < k)
      for (int i = 0; i <= j; ++i)
        w = A::add(w, A::mul(ld_g(a.G_hi, a.G_lo, l * W + ky + i), dd_from(a.Zp[i * kp + j])));
    a.Wp[e] = -(w.hi + w.lo);
  }

  // Totals: X = Y C_tot + X_cur R_tot; after this pass
  //   C_tot += C_p R_tot_old,  R_tot = R_p R_tot_old   (DD, first pass: R_p, C_p).
  // The old R_tot is staged in LDS; R_p goes through LDS one row block at a
  // time; C_p rows go through LDS 16 at a time.
  __shared__ double s_rph[16][64], s_rpl[16][64];
  __shared__ double s_toth[64][65], s_totl[64][65];
  Dd16 Rn;
  const bool first = (a.pass == 0);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) Rn.v[p][q] = dd_from(0.0);
  if (!first) {
    for (int e = tid; e < k * k; e += NTF) {
      const int i = e / k, l = e - i * k;
      s_toth[i][l] = a.Rtot[e];
      s_totl[i][l] = a.Rtot[k * k + e];
    }
  }
  // C_tot update (needs the old R_tot).
  for (int c0 = 0; c0 < ky; c0 += 16) {
    __syncthreads();
    for (int e = tid; e < 16 * 64; e += NTF) {
      const int r = e >> 6, j = e & 63, l = c0 + r;
      const dd_t cv = (l < ky && j < k) ? ld_g(a.G_hi, a.G_lo, l * W + ky + j) : dd_from(0.0);
      s_ch[r][j] = cv.hi;
      s_cl[r][j] = cv.lo;
    }
    __syncthreads();
    const int rn = (ky - c0) < 16 ? (ky - c0) : 16;
    for (int e = tid; e < rn * k; e += NTF) {
      const int r = e / k, j = e - r * k, l = c0 + r;
      dd_t ct;
      if (first) {
        ct = dd_make(s_ch[r][j], s_cl[r][j]);
      } else {
        ct = dd_make(a.Ctot[l * k + j], a.Ctot[ky * k + l * k + j]);
        for (int q = 0; q <= j; ++q)
          ct = A::add(ct, A::mul(dd_make(s_ch[r][q], s_cl[r][q]), dd_make(s_toth[q][j], s_totl[q][j])));
      }
      a.Ctot[l * k + j] = ct.hi;  // element-private
      a.Ctot[ky * k + l * k + j] = ct.lo;
    }
  }
  for (int blk = 0; blk < 4; ++blk) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * blk, l = tj + 16 * q;
      s_rph[ti][l] = (i < k && l < k) ? M.v[blk][q].hi : 0.0;
      s_rpl[ti][l] = (i < k && l < k) ? M.v[blk][q].lo : 0.0;
    }
    __syncthreads();
    const int i = ti + 16 * blk;
    if (i < k) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int l = tj + 16 * q;
        if (l >= k || l < i) continue;
        dd_t sacc = dd_from(0.0);
        if (first) {
          sacc = dd_make(s_rph[ti][l], s_rpl[ti][l]);
        } else {
          for (int qq = i; qq <= l; ++qq)
            sacc = A::add(sacc, A::mul(dd_make(s_rph[ti][qq], s_rpl[ti][qq]),
                                       dd_make(s_toth[qq][l], s_totl[qq][l])));
        }
        Rn.v[blk][q] = sacc;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * p, l = tj + 16 * q;
      if (i < k && l < k) {
        const dd_t v = (l >= i) ? Rn.v[p][q] : dd_from(0.0);
        a.Rtot[i * k + l] = v.hi;
        a.Rtot[k * k + i * k + l] = v.lo;
        if (a.R_out) a.R_out[i * k + l] = v.hi;
      }
    }
  if (a.C_out) {
    __syncthreads();
    for (int e = tid; e < ky * k; e += NTF) a.C_out[e] = a.Ctot[e];
  }
  if (tid == 0) a.status[3] = a.pass + 1;
}

// ---------------------------------------------------------------------------
// SVQB (binary64): M in LDS, cyclic Jacobi with round-robin parallel pairs.
__global__ void __launch_bounds__(NTF) svqb_kernel(FactorArgs a) {
  __shared__ double sM[64 * 65];
  __shared__ double sV[64 * 65];
  __shared__ double sc[32], ss[32];
  __shared__ int sp[32], sq[32];
  __shared__ double s_red[NTF];
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  const int k = a.k, ky = a.ky, W = a.ky + a.k, kp = a.kp;
  const int LD = 65;
  if (a.status[0] != 0) {
    for (int e = tid; e < kp * kp; e += NTF) a.Zp[e] = 0.0;
    return;
  }
  // M = G_XX - C^T (2C - S C) in binary64 (hi + lo folded).
  for (int e = tid; e < k * k; e += NTF) {
    const int i = e / k, l = e - i * k;
    auto g = [&](int r, int c) { return a.G_hi[r * W + c] + (a.G_lo ? a.G_lo[r * W + c] : 0.0); };
    double v = g(ky + i, ky + l);
    for (int r = 0; r < ky; ++r) {
      double sc2 = 0.0;
      for (int q = 0; q < ky; ++q) sc2 = __builtin_fma(g(r, q), g(q, ky + l), sc2);
      v = __builtin_fma(-g(r, ky + i), 2.0 * g(r, ky + l) - sc2, v);
    }
    sM[i * LD + l] = v;
    sV[i * LD + l] = (i == l) ? 1.0 : 0.0;
  }
  if (tid == 0) s_flag = 0;
  __syncthreads();
  for (int e = tid; e < k * k; e += NTF)
    if (!isfinite(sM[(e / k) * LD + e % k])) s_flag = 1;
  __syncthreads();
  if (s_flag) {
    if (tid == 0) { a.status[0] = 5; a.status[1] = a.pass + 1; a.status[2] = 0; }
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
  for (int sweep = 0; sweep < 30; ++sweep) {
    // convergence test: off-diagonal mass relative to the diagonal
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < k * k; e += NTF) {
      const int i = e / k, l = e - i * k;
      const double v = sM[i * LD + l];
      if (i != l) off += v * v; else dia += v * v;
    }
    s_red[tid] = off;
    __syncthreads();
    if (tid == 0) {
      double o = 0.0;
      for (int t = 0; t < NTF; ++t) o += s_red[t];
      s_red[0] = o;
    }
    __syncthreads();
    const double offt = s_red[0];
    __syncthreads();
    s_red[tid] = dia;
    __syncthreads();
    if (tid == 0) {
      double d = 0.0;
      for (int t = 0; t < NTF; ++t) d += s_red[t];
      s_flag = (offt <= 1e-34 * d) ? 1 : 0;
    }
    __syncthreads();
    if (s_flag) break;
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
          if (apq != 0.0) {
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
  }
  // eigenvalues on the diagonal; lift tiny ones
  __shared__ double lam[64];
  if (tid == 0) {
    double lmax = 0.0;
    for (int i = 0; i < k; ++i) lmax = fmax(lmax, sM[i * LD + i]);
    const double floor_ = lmax * 2.220446049250313e-16;
    for (int i = 0; i < k; ++i) {
      double l = sM[i * LD + i];
      if (!(l > floor_)) l = floor_;
      lam[i] = l;
    }
  }
  __syncthreads();
  for (int e = tid; e < kp * kp; e += NTF) {
    const int i = e / kp, j = e - i * kp;
    double z = 0.0, r = 0.0;
    if (i < k && j < k) {
      for (int l = 0; l < k; ++l) {
        const double w = sV[i * LD + l] * sV[j * LD + l];
        z = __builtin_fma(w, 1.0 / sqrt(lam[l]), z);
        r = __builtin_fma(w, sqrt(lam[l]), r);
      }
      if (a.Z_out) a.Z_out[i * k + j] = z;
      if (a.Rp_out) a.Rp_out[i * k + j] = r;
    }
    a.Zp[e] = z;
  }
  for (int e = tid; e < ky * kp; e += NTF) {
    const int l = e / kp, j = e - l * kp;
    a.Cp[e] = j < k ? a.G_hi[l * W + ky + j] + (a.G_lo ? a.G_lo[l * W + ky + j] : 0.0) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < ky * kp; e += NTF) {
    const int l = e / kp, j = e - l * kp;
    double w = 0.0;
    if (j < k)
      for (int i = 0; i < k; ++i)
        w = __builtin_fma(a.G_hi[l * W + ky + i] + (a.G_lo ? a.G_lo[l * W + ky + i] : 0.0), a.Zp[i * kp + j], w);
    a.Wp[e] = -w;
  }
  __syncthreads();
  // totals in binary64 (R_p dense): C_tot += C_p R_tot_old; R_tot = R_p R_tot_old
  const bool first = (a.pass == 0);
  // R_p into sM (reuse), computed from V and lam
  for (int e = tid; e < k * k; e += NTF) {
    const int i = e / k, j = e - i * k;
    double r = 0.0;
    for (int l = 0; l < k; ++l) r = __builtin_fma(sV[i * LD + l] * sV[j * LD + l], sqrt(lam[l]), r);
    sM[i * LD + j] = r;
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
  if (tid == 0) a.status[3] = a.pass + 1;
}

}  // namespace

hipError_t launch_factor(const FactorArgs& a, hipStream_t st) {
  if (a.k > 64 || a.ky > 64 || a.k < 1) return hipErrorInvalidValue;
  if (a.fact == 1) {
    hipLaunchKernelGGL(svqb_kernel, dim3(1), dim3(NTF), 0, st, a);
  } else if (a.dd) {
    hipLaunchKernelGGL(factor_kernel<true>, dim3(1), dim3(NTF), 0, st, a);
  } else {
    hipLaunchKernelGGL(factor_kernel<false>, dim3(1), dim3(NTF), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace borth
