// Device code of the k x k step shared by factor.hip and the persistent
// batched kernel (batch_persistent.hip): workgroup reductions, DD / binary64
// arithmetic selectors, and the Cholesky body (its design is described at
// chol_body).
#pragma once
#include "dd.hpp"
#include "internal.hpp"

namespace borth {
namespace fct {

constexpr int NTF = 256;

// Two values per thread reduced over the workgroup (sums, or max of x and
// min of y): a shuffle tree inside each wave, then the waves' results in
// wave order by thread 0, whose x and y hold the result.  NT is a multiple
// of 64; sh holds 2 NT / 64 doubles.  Deterministic.
template <int NT, bool MAXMIN>
__device__ __forceinline__ void wg_reduce2(double& x, double& y, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double xo = __shfl_xor(x, o), yo = __shfl_xor(y, o);
    x = MAXMIN ? fmax(x, xo) : x + xo;
    y = MAXMIN ? fmin(y, yo) : y + yo;
  }
  constexpr int NW = NT / 64;
  const int w = (int)threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[w] = x;
    sh[NW + w] = y;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 1; i < NW; ++i) {
      x = MAXMIN ? fmax(x, sh[i]) : x + sh[i];
      y = MAXMIN ? fmin(y, sh[NW + i]) : y + sh[NW + i];
    }
}

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

// Accumulator of a dot product of DD operands, started from a DD value:
// Dot2 on the high words plus the binary64 cross terms a.hi b.lo + a.lo b.hi.
// Its error is O(n u^2) sum |a_i b_i|, the order of a dot product carried in
// DD arithmetic, at a third of the instructions.  Binary64 mode: one FMA.
template <bool DD>
struct Acc {
  double s, c;
  __device__ __forceinline__ explicit Acc(dd_t v) : s(v.hi), c(DD ? v.lo : 0.0) {}
  __device__ __forceinline__ void add(dd_t a, dd_t b) {
    if (DD) {
      dot2_step(s, c, a.hi, b.hi);
      c = __builtin_fma(a.hi, b.lo, __builtin_fma(a.lo, b.hi, c));
    } else {
      s = __builtin_fma(a.hi, b.hi, s);
    }
  }
  __device__ __forceinline__ dd_t get() const { return DD ? two_sum(s, c) : dd_from(s); }
};

// Cholesky factor of the k x k block in one workgroup of T x T threads; each
// thread holds the NS x NS elements (i, l) = (ti + T p, tj + T q), k <= T NS.
//
// The factorization runs as LDL^T elimination on M augmented by the
// identity: eliminating column j subtracts (M_ji / d_j) times row j from
// every row i > j, on the trailing upper part of M (l >= i) and on the
// identity's image (l <= j), which fills in as L^{-1}.  The two never
// overlap, so both share one k x k array: element (i, l) holds U = D L^T for
// l >= i and L^{-1} for l < i.  At the end R = D^{-1/2} U and
// Z = R^{-1} = L^{-T} D^{-1/2}, so the inverse needs no second sweep and the
// square roots leave the serial chain.  Each step costs one reciprocal of
// the pivot and one barrier; the owners of row j + 1 publish it through a
// double-buffered LDS row, and the owner of the pivot its reciprocal.
//
// The body runs in a workgroup of T x T threads (a launch, or a persistent
// workgroup of that size) with its working arrays at mem: in LDS for the
// kernel, in global memory for the persistent batched kernel, whose LDS is
// taken by the sweeps.
struct CholMem {
  double* r0;   // 2 x 64 x 65: C (DD) / R_p (DD)
  double* r1;   // 2 x 64 x 65: S, then D (DD) / Z (hi) / old R_tot (DD)
  double* row;  // 2 x 2 x KP: [buffer][hi, lo][column]
  double* piv;  // 2 x 64
  int* flag;
  double* dinv; // 2 x 2: [buffer][hi, lo], the reciprocal of the next pivot
};

template <bool DD, int T, int NS>
__device__ __forceinline__ void chol_body(const FactorArgs& a, const CholMem& mem) {
  using A = Ar<DD>;
  if (stopped(a.stop, a.pass)) return;
  constexpr int NT = T * T, KP = T * NS, LD = 65;
  constexpr int ND = (64 * KP + NT - 1) / NT;  // per-thread share of a ky x k block
  double(*s_r0)[64 * LD] = reinterpret_cast<double(*)[64 * LD]>(mem.r0);
  double(*s_r1)[64 * LD] = reinterpret_cast<double(*)[64 * LD]>(mem.r1);
  double(*s_row)[2][KP] = reinterpret_cast<double(*)[2][KP]>(mem.row);
  double(*s_piv)[64] = reinterpret_cast<double(*)[64]>(mem.piv);
  int& s_flag = *mem.flag;

  const int tid = threadIdx.x;
  const int ti = tid / T, tj = tid - (tid / T) * T;
  const int k = a.k, ky = a.ky, W = a.ky + a.k, kp = a.kp;
  const bool first = (a.pass == 0);

  auto zero_out = [&]() {
    for (int e = tid; e < kp * kp; e += NT) {
      a.Zp[e] = 0.0;
      if (a.Zplo) a.Zplo[e] = 0.0;
    }
  };
  // A previous pass already failed: leave a zero transform and stop.
  if (a.status[0] != 0) {
    zero_out();
    return;
  }

  // Upper part of M = G_XX; the lower part starts as the identity's image (0).
  dd_t x[NS][NS];
#pragma unroll
  for (int p = 0; p < NS; ++p)
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int i = ti + T * p, l = tj + T * q;
      x[p][q] = (i < k && l < k && l >= i) ? ld_g(a.G_hi, a.G_lo, (ky + i) * W + ky + l) : dd_from(0.0);
    }

  // Projection against Y: M = G_XX - C^T D with D = 2C - S C, C = G_YX,
  // S = G_YY; C^T D = C^T C - C^T (C - S C) expands (X - Y C)^T (X - Y C)
  // with the Gram matrix of Y as it is (no assumption Y^T Y = I).
  if (ky > 0) {
    for (int e = tid; e < ky * k; e += NT) {
      const int r = e / k, l = e - r * k;
      const dd_t c = ld_g(a.G_hi, a.G_lo, r * W + ky + l);
      s_r0[0][r * LD + l] = c.hi;
      s_r0[1][r * LD + l] = c.lo;
    }
    for (int e = tid; e < ky * ky; e += NT) {
      const int r = e / ky, q = e - r * ky;
      const dd_t sv = ld_g(a.G_hi, a.G_lo, r * W + q);
      s_r1[0][r * LD + q] = sv.hi;
      s_r1[1][r * LD + q] = sv.lo;
    }
    __syncthreads();
    dd_t dreg[ND];
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const int e = tid + NT * t;
      dreg[t] = dd_from(0.0);
      if (e < ky * k) {
        const int r = e / k, l = e - r * k;
        const dd_t c = dd_make(s_r0[0][r * LD + l], s_r0[1][r * LD + l]);
        Acc<DD> acc(dd_make(2.0 * c.hi, 2.0 * c.lo));
        for (int q = 0; q < ky; ++q)
          acc.add(dd_make(-s_r1[0][r * LD + q], -s_r1[1][r * LD + q]),
                  dd_make(s_r0[0][q * LD + l], s_r0[1][q * LD + l]));
        dreg[t] = acc.get();
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const int e = tid + NT * t;
      if (e < ky * k) {
        const int r = e / k, l = e - r * k;
        s_r1[0][r * LD + l] = dreg[t].hi;
        s_r1[1][r * LD + l] = dreg[t].lo;
        if (a.Cplo) {  // DD update: the corrected coefficients, read back below
          a.Cp[r * kp + l] = dreg[t].hi;
          a.Cplo[r * kp + l] = dreg[t].lo;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i < k && l < k && l >= i) {
          Acc<DD> acc(x[p][q]);
          for (int r = 0; r < ky; ++r)
            acc.add(dd_make(-s_r0[0][r * LD + i], -s_r0[1][r * LD + i]),
                    dd_make(s_r1[0][r * LD + l], s_r1[1][r * LD + l]));
          x[p][q] = acc.get();
        }
      }
  }

  // Non-finite check; diagonal to LDS for the trace (summed in fixed order).
  if (tid == 0) s_flag = 0;
  __syncthreads();
  {
    int bad = 0;
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i < k && l < k && l >= i) {
          if (!isfinite(x[p][q].hi) || !isfinite(x[p][q].lo)) bad = 1;
          if (i == l) s_piv[0][i] = x[p][q].hi;
        }
      }
    if (bad) s_flag = 1;
  }
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
    double tr = 0.0;
    for (int i = 0; i < k; ++i) tr += s_piv[0][i];
    const double sh = a.shift_rel * tr;
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i < k && i == l) x[p][q] = A::add(x[p][q], dd_from(sh));
      }
  }
  // Publish row 0, and the reciprocal of its pivot: the thread that holds
  // a pivot computes it once for all (every thread would otherwise repeat
  // the same DD division on every column).
  if (ti == 0) {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      s_row[0][0][tj + T * q] = x[0][q].hi;
      s_row[0][1][tj + T * q] = x[0][q].lo;
      if (tj + T * q == 0) {
        const dd_t r = A::recip(x[0][q]);
        mem.dinv[0] = r.hi;
        mem.dinv[1] = r.lo;
      }
    }
  }
  __syncthreads();

  int fail = 0;
  for (int j = 0; j < k; ++j) {
    const double* rh = s_row[j & 1][0];
    const double* rl = s_row[j & 1][1];
    const dd_t d = dd_make(rh[j], rl[j]);
    // unpivoted: a pivot that is not positive and finite stops here (the
    // value is the same in every thread, so all leave together)
    if (!(d.hi > 0.0) || !isfinite(d.hi)) {
      fail = j + 1;
      break;
    }
    const dd_t dinv = dd_make(mem.dinv[2 * (j & 1)], mem.dinv[2 * (j & 1) + 1]);
    if (tid == 0) {
      s_piv[0][j] = d.hi;
      s_piv[1][j] = d.lo;
    }
    dd_t c[NS], v[NS];
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const int i = ti + T * p;
      c[p] = (i > j) ? A::mul(dd_make(rh[i], rl[i]), dinv) : dd_from(0.0);
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int l = tj + T * q;
      v[q] = (l == j) ? dd_from(1.0) : dd_make(rh[l], rl[l]);
    }
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i > j && (l >= i || l <= j)) x[p][q] = A::fnms(x[p][q], c[p], v[q]);
      }
    const int jn = j + 1;
    if (ti == jn % T) {
#pragma unroll
      for (int p = 0; p < NS; ++p)
        if (p == jn / T) {
#pragma unroll
          for (int q = 0; q < NS; ++q) {
            s_row[jn & 1][0][tj + T * q] = x[p][q].hi;
            s_row[jn & 1][1][tj + T * q] = x[p][q].lo;
            if (tj + T * q == jn) {
              const dd_t r = A::recip(x[p][q]);
              mem.dinv[2 * (jn & 1)] = r.hi;
              mem.dinv[2 * (jn & 1) + 1] = r.lo;
            }
          }
        }
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) {
      a.status[0] = 4;
      a.status[1] = a.pass + 1;
      a.status[2] = fail;
      if (a.stop) a.stop[0] = a.pass + 1;
    }
    zero_out();
    return;
  }

  // R = D^{-1/2} U (l >= i), Z^T = D^{-1/2} L^{-1} (l <= i); x keeps R_p for
  // l >= i and Z_li for l < i.  Z (hi words) goes to LDS for the W product,
  // C (DD) too.
  dd_t rs[NS];
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    const int i = ti + T * p;
    rs[p] = i < k ? A::rsqrt(dd_make(s_piv[0][i], s_piv[1][i])) : dd_from(0.0);
  }
#pragma unroll
  for (int p = 0; p < NS; ++p)
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int i = ti + T * p, l = tj + T * q;
      if (i < k && l < k) {
        x[p][q] = A::mul(x[p][q], rs[p]);
        const dd_t z = (l < i) ? x[p][q] : (l == i ? rs[p] : dd_from(0.0));
        s_r1[0][l * LD + i] = z.hi;  // Z[l][i]
        s_r1[1][l * LD + i] = z.lo;
        if (a.Rp_out) a.Rp_out[i * k + l] = l >= i ? x[p][q].hi : 0.0;
      }
    }
  // projection coefficients of this pass: C, or for the DD update the
  // corrected D written above
  for (int e = tid; e < ky * k; e += NT) {
    const int r = e / k, l = e - r * k;
    const dd_t cv = a.Cplo ? dd_make(a.Cp[r * kp + l], a.Cplo[r * kp + l])
                           : ld_g(a.G_hi, a.G_lo, r * W + ky + l);
    s_r0[0][r * LD + l] = cv.hi;
    s_r0[1][r * LD + l] = cv.lo;
  }
  __syncthreads();
  for (int e = tid; e < kp * kp; e += NT) {
    const int i = e / kp, l = e - i * kp;
    const double z = (i < k && l < k) ? s_r1[0][i * LD + l] : 0.0;
    a.Zp[e] = z;
    if (a.Zplo) a.Zplo[e] = (i < k && l < k) ? s_r1[1][i * LD + l] : 0.0;
    if (a.Z_out && i < k && l < k) a.Z_out[i * k + l] = z;
  }
  // C of this pass, rounded, for the update (S - Y C) Z (DD update: and the
  // rounding remainder)
  for (int e = tid; e < ky * kp; e += NT) {
    const int r = e / kp, j = e - r * kp;
    const double h = s_r0[0][r * LD + (j < k ? j : 0)], lo = s_r0[1][r * LD + (j < k ? j : 0)];
    const double cr = j < k ? h + lo : 0.0;
    a.Cp[e] = cr;
    if (a.Cplo) a.Cplo[e] = j < k ? (h - cr) + lo : 0.0;
  }

  // Totals: X = Y C_tot + X_cur R_tot.  After this pass
  //   C_tot += C_p R_tot_old,  R_tot = R_p R_tot_old   (first pass: C_p, R_p).
  if (first) {
    for (int e = tid; e < ky * k; e += NT) {
      const int r = e / k, l = e - r * k;
      const double h = s_r0[0][r * LD + l], lo = s_r0[1][r * LD + l];
      a.Ctot[e] = h;
      a.Ctot[ky * k + e] = DD ? lo : 0.0;
      if (a.C_out) a.C_out[e] = h;
    }
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i < k && l < k) {
          const dd_t v = l >= i ? x[p][q] : dd_from(0.0);
          a.Rtot[i * k + l] = v.hi;
          a.Rtot[k * k + i * k + l] = v.lo;
          if (a.R_out) a.R_out[i * k + l] = v.hi;
        }
      }
  } else {
    __syncthreads();  // Z in s_r1 is no longer read
    for (int e = tid; e < k * k; e += NT) {
      const int i = e / k, l = e - i * k;
      s_r1[0][i * LD + l] = a.Rtot[e];
      s_r1[1][i * LD + l] = a.Rtot[k * k + e];
    }
    __syncthreads();
    for (int e = tid; e < ky * k; e += NT) {
      const int r = e / k, j = e - r * k;
      Acc<DD> acc(dd_make(a.Ctot[e], a.Ctot[ky * k + e]));
      for (int q = 0; q <= j; ++q)
        acc.add(dd_make(s_r0[0][r * LD + q], s_r0[1][r * LD + q]),
                dd_make(s_r1[0][q * LD + j], s_r1[1][q * LD + j]));
      const dd_t ct = acc.get();
      a.Ctot[e] = ct.hi;  // element-private
      a.Ctot[ky * k + e] = ct.lo;
      if (a.C_out) a.C_out[e] = ct.hi;
    }
    __syncthreads();  // C in s_r0 is no longer read
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i < k && l < k && l >= i) {
          s_r0[0][i * LD + l] = x[p][q].hi;
          s_r0[1][i * LD + l] = x[p][q].lo;
        }
      }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i < k && l < k) {
          dd_t v = dd_from(0.0);
          if (l >= i) {
            Acc<DD> acc(dd_from(0.0));
            for (int qq = i; qq <= l; ++qq)
              acc.add(dd_make(s_r0[0][i * LD + qq], s_r0[1][i * LD + qq]),
                      dd_make(s_r1[0][qq * LD + l], s_r1[1][qq * LD + l]));
            v = acc.get();
          }
          a.Rtot[i * k + l] = v.hi;  // element-private; the old totals are in LDS
          a.Rtot[k * k + i * k + l] = v.lo;
          if (a.R_out) a.R_out[i * k + l] = v.hi;
        }
      }
  }
  if (a.conv) {
    // stop test of the iterated scheme: ||C_p||_F (this pass's projection
    // coefficients) and ||R_p - I||_F, summed in a fixed order
    double rr = 0.0;
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i < k && l < k && l >= i) {
          const double d = x[p][q].hi - (i == l ? 1.0 : 0.0);
          rr = __builtin_fma(d, d, rr);
        }
      }
    double cc = 0.0;
    for (int e = tid; e < ky * k; e += NT) {
      const double v = a.G_hi[(e / k) * W + ky + e % k];
      cc = __builtin_fma(v, v, cc);
    }
    wg_reduce2<NT, false>(rr, cc, s_r1[0]);
    if (tid == 0) {
      const double sr = rr, sc = cc;
      a.conv[0] = sqrt(sc);
      a.conv[1] = sqrt(sr);
      // iterated scheme: this pass is the last one when both norms are small
      if (a.stop && sqrt(sc) <= a.stop_eps && sqrt(sr) <= a.stop_eps) a.stop[0] = a.pass + 1;
    }
  }
  if (a.kappa) {
    // max R_ii / min R_ii: a lower bound on the condition number of the
    // projected block (each R_ii is a distance to a span of other columns)
    double dmx = 0.0, dmn = __builtin_inf();
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = ti + T * p, l = tj + T * q;
        if (i < k && l == i) {
          const double d = fabs(x[p][q].hi);
          dmx = fmax(dmx, d);
          dmn = fmin(dmn, d);
        }
      }
    wg_reduce2<NT, true>(dmx, dmn, s_r1[0]);
    if (tid == 0) a.kappa[0] = dmx / dmn;
  }
  if (tid == 0) a.status[3] = a.pass + 1;
}

}  // namespace fct
}  // namespace borth
