/*
 * CPU oracle for block orthonormalization.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the GPU path.
 *
 * What the method computes (paper Sec. 4.2): for a block X (m x k) and an
 * orthonormal locked basis W (m x ky; called Y in this code), phase I forms
 * the projection  Xt = (I - Y Y^T) X  with coefficients C = Y^T X, phase II
 * forms the Gram matrix  M = Xt^T Xt, factors it (Cholesky M = R^T R, Z = R^{-1},
 * or SVQB  Z = M^{-1/2}) and sets  Q = Xt Z, so that Z^T M Z = I and Q^T Q = I.
 *
 * Two kinds of routines live here:
 *
 *  O1 -- the plain definitions, evaluated in IEEE binary128 (__float128,
 *        113-bit significand).  A product of two binary64 numbers is exact in
 *        binary128, so Gram sums carry only 2^-113 rounding; the thin QR factors
 *        returned by or_qr_q are the binary64 roundings of the exact factors of
 *        the stored input for every condition number below ~1e17.
 *
 *  O2 -- the paper's algorithm taken step by step in the working precision:
 *        binary64 (plain CholQR / CholQR2) or double-double (DD) in the first
 *        pass -- the projection against W, the Gram matrix and its
 *        factorization all in DD, as Sec. 4.2 describes its DD variant.  DD uses
 *        Dekker's splitting for the exact product (no FMA, so it does not share
 *        the GPU's FMA route) and Knuth's TwoSum; DD division and square root
 *        are Newton-Raphson iterations seeded by binary64, as the paper states.
 *
 * Determinism: every row sum is taken over a fixed partition of the rows into
 * at most 1024 contiguous blocks, the per-block partials are combined in block
 * order, so the results are bitwise independent of the OpenMP thread count.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 f128;

#define NPART_MAX 1024

static int64_t npart(int64_t m) { return m <= 0 ? 1 : (m < NPART_MAX ? m : NPART_MAX); }
static int64_t pbeg(int64_t m, int64_t np, int64_t b) { return (m * b) / np; }

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of the following parallel regions (results do not depend on
 * it: every sum runs over the fixed row-block partition). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static void split_q(f128 s, double* hi, double* lo) {
  double h = (double)s;
  *hi = h;
  if (lo) *lo = (double)(s - (f128)h);
}

static f128 join_q(const double* hi, const double* lo, size_t i) {
  f128 v = (f128)hi[i];
  if (lo) v += (f128)lo[i];
  return v;
}

/* ------------------------------------------------------------------------ */
/* O1: exact Gram-type product  G = A^T B  (ka x kb), binary128 accumulation. */
int or_gram_q(int64_t m, int ka, const double* A, int64_t lda, int kb,
              const double* B, int64_t ldb, double* ghi, double* glo) {
  const int64_t np = npart(m);
  const size_t n = (size_t)ka * (size_t)kb;
  f128* part = (f128*)calloc((size_t)np * n + 1, sizeof(f128));
  if (!part) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < np; ++b) {
    f128* p = part + (size_t)b * n;
    for (int64_t r = pbeg(m, np, b); r < pbeg(m, np, b + 1); ++r) {
      const double* a = A + r * lda;
      const double* c = B + r * ldb;
      for (int i = 0; i < ka; ++i) {
        const f128 ai = (f128)a[i];
        for (int j = 0; j < kb; ++j) p[(size_t)i * kb + j] += ai * (f128)c[j];
      }
    }
  }
  for (size_t e = 0; e < n; ++e) {
    f128 s = 0;
    for (int64_t b = 0; b < np; ++b) s += part[(size_t)b * n + e];
    split_q(s, &ghi[e], glo ? &glo[e] : NULL);
  }
  free(part);
  return 0;
}

/* O1: B-weighted Gram-type product  G = A^T diag(w) B  (ka x kb), the
 * B-inner products of Sec. 4.2's closing remark: each term (w_r a_ri) b_rj
 * in binary128 (w_r a_ri is exact there), accumulated as in or_gram_q. */
int or_gram_w_q(int64_t m, int ka, const double* A, int64_t lda, int kb,
                const double* B, int64_t ldb, const double* w, double* ghi, double* glo) {
  const int64_t np = npart(m);
  const size_t n = (size_t)ka * (size_t)kb;
  f128* part = (f128*)calloc((size_t)np * n + 1, sizeof(f128));
  if (!part) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < np; ++b) {
    f128* p = part + (size_t)b * n;
    for (int64_t r = pbeg(m, np, b); r < pbeg(m, np, b + 1); ++r) {
      const double* a = A + r * lda;
      const double* c = B + r * ldb;
      const f128 wr = (f128)w[r];
      for (int i = 0; i < ka; ++i) {
        const f128 ai = wr * (f128)a[i];
        for (int j = 0; j < kb; ++j) p[(size_t)i * kb + j] += ai * (f128)c[j];
      }
    }
  }
  for (size_t e = 0; e < n; ++e) {
    f128 s = 0;
    for (int64_t b = 0; b < np; ++b) s += part[(size_t)b * n + e];
    split_q(s, &ghi[e], glo ? &glo[e] : NULL);
  }
  free(part);
  return 0;
}

/* O1: Cholesky  G = R^T R  (R upper, positive diagonal) of the symmetric G
 * given as hi(+lo), in binary128.  Reads the upper triangle of G.
 * info = 0 on success, j (1-based) if the j-th pivot is not positive/finite. */
static int chol_q_inplace(int k, f128* a /* k*k, upper used; R out */) {
  for (int j = 0; j < k; ++j) {
    f128 d = a[j * k + j];
    for (int i = 0; i < j; ++i) d -= a[i * k + j] * a[i * k + j];
    if (!(d > 0) || isinfq(d) || isnanq(d)) return j + 1;
    const f128 rjj = sqrtq(d);
    a[j * k + j] = rjj;
    for (int l = j + 1; l < k; ++l) {
      f128 s = a[j * k + l];
      for (int i = 0; i < j; ++i) s -= a[i * k + j] * a[i * k + l];
      a[j * k + l] = s / rjj;
    }
    for (int l = 0; l < j; ++l) a[j * k + l] = 0;
  }
  return 0;
}

int or_chol_q(int k, const double* ghi, const double* glo, double* rhi,
              double* rlo) {
  f128* a = (f128*)malloc(sizeof(f128) * (size_t)k * k + 16);
  for (size_t e = 0; e < (size_t)k * k; ++e) a[e] = join_q(ghi, glo, e);
  int info = chol_q_inplace(k, a);
  if (info == 0)
    for (size_t e = 0; e < (size_t)k * k; ++e) split_q(a[e], &rhi[e], rlo ? &rlo[e] : NULL);
  free(a);
  return info;
}

/* O1: inverse of an upper-triangular R by back substitution, binary128. */
static void trinv_q_inplace(int k, const f128* r, f128* z) {
  memset(z, 0, sizeof(f128) * (size_t)k * k);
  for (int j = 0; j < k; ++j) {
    z[j * k + j] = 1 / r[j * k + j];
    for (int i = j - 1; i >= 0; --i) {
      f128 s = 0;
      for (int l = i + 1; l <= j; ++l) s += r[i * k + l] * z[l * k + j];
      z[i * k + j] = -s / r[i * k + i];
    }
  }
}

int or_trinv_q(int k, const double* rhi, const double* rlo, double* zhi,
               double* zlo) {
  f128* r = (f128*)malloc(sizeof(f128) * (size_t)k * k + 16);
  f128* z = (f128*)malloc(sizeof(f128) * (size_t)k * k + 16);
  for (size_t e = 0; e < (size_t)k * k; ++e) r[e] = join_q(rhi, rlo, e);
  for (int j = 0; j < k; ++j)
    if (!(r[j * k + j] != 0)) { free(r); free(z); return j + 1; }
  trinv_q_inplace(k, r, z);
  for (size_t e = 0; e < (size_t)k * k; ++e) split_q(z[e], &zhi[e], zlo ? &zlo[e] : NULL);
  free(r);
  free(z);
  return 0;
}

/* O1: basis update  Q = (X - Y C) Z  for given C (ky x k, hi+lo) and Z (k x k),
 * evaluated in binary128 and rounded once.  The product Y C and the product
 * with Z are exact definitions; only the final rounding is binary64. */
int or_update_q(int64_t m, int k, const double* X, int64_t ldx, int ky,
                const double* Y, int64_t ldy, const double* chi,
                const double* clo, const double* Z, double* Q, int64_t ldq) {
#pragma omp parallel
  {
    f128* xt = (f128*)malloc(sizeof(f128) * (size_t)(k + 1));
#pragma omp for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
      for (int j = 0; j < k; ++j) {
        f128 v = (f128)X[r * ldx + j];
        for (int l = 0; l < ky; ++l)
          v -= (f128)Y[r * ldy + l] * join_q(chi, clo, (size_t)l * k + j);
        xt[j] = v;
      }
      for (int j = 0; j < k; ++j) {
        f128 s = 0;
        for (int i = 0; i < k; ++i) s += xt[i] * (f128)Z[(size_t)i * k + j];
        Q[r * ldq + j] = (double)s;
      }
    }
    free(xt);
  }
  return 0;
}

/* binary128 Gram of a binary128 m x k array (row-major, ld = k). */
static void gram_q_of_q(int64_t m, int k, const f128* xt, f128* g) {
  const int64_t np = npart(m);
  const size_t n = (size_t)k * k;
  f128* part = (f128*)calloc((size_t)np * n + 1, sizeof(f128));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < np; ++b) {
    f128* p = part + (size_t)b * n;
    for (int64_t r = pbeg(m, np, b); r < pbeg(m, np, b + 1); ++r) {
      const f128* x = xt + (size_t)r * k;
      for (int i = 0; i < k; ++i)
        for (int j = i; j < k; ++j) p[(size_t)i * k + j] += x[i] * x[j];
    }
  }
  for (int i = 0; i < k; ++i)
    for (int j = i; j < k; ++j) {
      f128 s = 0;
      for (int64_t b = 0; b < np; ++b) s += part[(size_t)b * n + (size_t)i * k + j];
      g[i * k + j] = s;
      g[j * k + i] = s;
    }
  free(part);
}

/* O1: the exact answer.  C = Y^T X, Xt = X - Y C, G = Xt^T Xt, G = R^T R,
 * Q = Xt R^{-1} (row-wise forward substitution), all in binary128; Q, R, C and
 * (optionally) G are rounded to binary64 (G as hi+lo) at the end.
 * Returns 0, or the 1-based pivot at which binary128 Cholesky fails. */
int or_qr_q(int64_t m, int k, const double* X, int64_t ldx, int ky,
            const double* Y, int64_t ldy, double* Q, int64_t ldq, double* R,
            double* C, double* ghi, double* glo) {
  f128* c = (f128*)calloc((size_t)(ky > 0 ? ky : 1) * k, sizeof(f128));
  if (ky > 0) {
    const int64_t np = npart(m);
    const size_t n = (size_t)ky * k;
    f128* part = (f128*)calloc((size_t)np * n, sizeof(f128));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < np; ++b) {
      f128* p = part + (size_t)b * n;
      for (int64_t r = pbeg(m, np, b); r < pbeg(m, np, b + 1); ++r)
        for (int l = 0; l < ky; ++l) {
          const f128 yl = (f128)Y[r * ldy + l];
          for (int j = 0; j < k; ++j) p[(size_t)l * k + j] += yl * (f128)X[r * ldx + j];
        }
    }
    for (size_t e = 0; e < n; ++e) {
      f128 s = 0;
      for (int64_t b = 0; b < np; ++b) s += part[(size_t)b * n + e];
      c[e] = s;
    }
    free(part);
  }
  f128* xt = (f128*)malloc(sizeof(f128) * (size_t)m * k + 16);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)
    for (int j = 0; j < k; ++j) {
      f128 v = (f128)X[r * ldx + j];
      for (int l = 0; l < ky; ++l) v -= (f128)Y[r * ldy + l] * c[(size_t)l * k + j];
      xt[(size_t)r * k + j] = v;
    }
  f128* g = (f128*)malloc(sizeof(f128) * (size_t)k * k + 16);
  gram_q_of_q(m, k, xt, g);
  if (ghi)
    for (size_t e = 0; e < (size_t)k * k; ++e) split_q(g[e], &ghi[e], glo ? &glo[e] : NULL);
  int info = chol_q_inplace(k, g); /* g now holds R */
  if (info == 0) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
      f128 q[128];
      for (int j = 0; j < k; ++j) {
        f128 s = xt[(size_t)r * k + j];
        for (int i = 0; i < j; ++i) s -= q[i] * g[i * k + j];
        q[j] = s / g[j * k + j];
        Q[r * ldq + j] = (double)q[j];
      }
    }
    for (size_t e = 0; e < (size_t)k * k; ++e) R[e] = (double)g[e];
  }
  if (C)
    for (size_t e = 0; e < (size_t)ky * k; ++e) C[e] = (double)c[e];
  free(c);
  free(xt);
  free(g);
  return info;
}

/* O1: symmetric inverse square root  Z = M^{-1/2} = U L^{-1/2} U^T  of an SPD
 * M (hi+lo) by cyclic Jacobi rotations in binary128 (the SVQB transform in its
 * symmetric form, the Procrustes-optimal Z of Sec. 4.2).  Eigenvalues are
 * returned in ascending order in lam (binary64).  Returns 0, or -1 if M is not
 * positive definite to binary128 working accuracy. */
/* Cyclic Jacobi rotations in binary128 on the symmetric a (k x k): on return
 * a is diagonal to working accuracy (its diagonal holds the eigenvalues) and
 * v holds the eigenvectors as columns, a_in = v diag(a) v^T. */
static void jacobi_q(int k, f128* a, f128* v) {
  const size_t n = (size_t)k * k;
  for (size_t e = 0; e < n; ++e) v[e] = 0;
  for (int i = 0; i < k; ++i) v[i * k + i] = 1;
  f128 prev_off = -1;
  for (int sweep = 0; sweep < 80; ++sweep) {
    f128 off = 0, tot = 0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        tot += a[i * k + j] * a[i * k + j];
        if (i != j) off += a[i * k + j] * a[i * k + j];
      }
    if (off <= tot * 1e-66Q || (prev_off >= 0 && off >= prev_off)) break;
    prev_off = off;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const f128 apq = a[p * k + q];
        if (apq == 0) continue;
        const f128 theta = (a[q * k + q] - a[p * k + p]) / (2 * apq);
        const f128 t = (theta >= 0 ? 1 : -1) / (fabsq(theta) + sqrtq(theta * theta + 1));
        const f128 cs = 1 / sqrtq(t * t + 1), sn = t * cs;
        for (int r = 0; r < k; ++r) { /* columns p, q */
          const f128 arp = a[r * k + p], arq = a[r * k + q];
          a[r * k + p] = cs * arp - sn * arq;
          a[r * k + q] = sn * arp + cs * arq;
        }
        for (int r = 0; r < k; ++r) { /* rows p, q */
          const f128 apr = a[p * k + r], aqr = a[q * k + r];
          a[p * k + r] = cs * apr - sn * aqr;
          a[q * k + r] = sn * apr + cs * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const f128 vrp = v[r * k + p], vrq = v[r * k + q];
          v[r * k + p] = cs * vrp - sn * vrq;
          v[r * k + q] = sn * vrp + cs * vrq;
        }
      }
  }
}

int or_svqb_q(int k, const double* mhi, const double* mlo, double* Z,
              double* lam) {
  const size_t n = (size_t)k * k;
  f128* a = (f128*)malloc(sizeof(f128) * n + 16);
  f128* v = (f128*)calloc(n + 1, sizeof(f128));
  for (size_t e = 0; e < n; ++e) a[e] = join_q(mhi, mlo, e);
  jacobi_q(k, a, v);
  int bad = 0;
  f128* s = (f128*)malloc(sizeof(f128) * (size_t)k + 16);
  for (int i = 0; i < k; ++i) {
    if (!(a[i * k + i] > 0)) bad = 1;
    s[i] = bad ? 0 : 1 / sqrtq(a[i * k + i]);
  }
  if (!bad) {
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        f128 acc = 0;
        for (int l = 0; l < k; ++l) acc += v[i * k + l] * s[l] * v[j * k + l];
        Z[i * k + j] = (double)acc;
      }
  }
  /* ascending eigenvalues */
  if (lam) {
    f128* d = (f128*)malloc(sizeof(f128) * (size_t)k + 16);
    for (int i = 0; i < k; ++i) d[i] = a[i * k + i];
    for (int i = 1; i < k; ++i)
      for (int j = i; j > 0 && d[j - 1] > d[j]; --j) { f128 t = d[j]; d[j] = d[j - 1]; d[j - 1] = t; }
    for (int i = 0; i < k; ++i) lam[i] = (double)d[i];
    free(d);
  }
  free(s);
  free(a);
  free(v);
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Double-double arithmetic for O2, without FMA.
 * TwoSum (Knuth), TwoProduct via Dekker's splitting with 2^27 + 1; the
 * double-word sum and product follow the accurate double-word algorithms of
 * Joldes, Muller and Popescu (2017); reciprocal and square root are one Newton
 * step from a binary64 seed, evaluated in DD. */
typedef struct { double h, l; } dd;

static inline dd two_sum(double a, double b) {
  dd r;
  r.h = a + b;
  const double z = r.h - a;
  r.l = (a - (r.h - z)) + (b - z);
  return r;
}
static inline dd fast_two_sum(double a, double b) { /* |a| >= |b| or a == 0 */
  dd r;
  r.h = a + b;
  r.l = b - (r.h - a);
  return r;
}
static inline void dekker_split(double a, double* hi, double* lo) {
  const double c = 134217729.0 * a;
  const double h = c - (c - a);
  *hi = h;
  *lo = a - h;
}
static inline dd two_prod(double a, double b) {
  double ah, al, bh, bl;
  dekker_split(a, &ah, &al);
  dekker_split(b, &bh, &bl);
  dd r;
  r.h = a * b;
  r.l = ((ah * bh - r.h) + ah * bl + al * bh) + al * bl;
  return r;
}
static inline dd dd_add(dd a, dd b) {
  const dd s = two_sum(a.h, b.h);
  const dd t = two_sum(a.l, b.l);
  const double c = s.l + t.h;
  const dd v = fast_two_sum(s.h, c);
  const double w = t.l + v.l;
  return fast_two_sum(v.h, w);
}
static inline dd dd_neg(dd a) { dd r = {-a.h, -a.l}; return r; }
static inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
static inline dd dd_mul(dd a, dd b) {
  const dd c = two_prod(a.h, b.h);
  const double t = a.h * b.l + a.l * b.h;
  return fast_two_sum(c.h, c.l + t);
}
static inline dd dd_from(double a) { dd r = {a, 0.0}; return r; }
/* reciprocal: x1 = x0 + x0 (1 - b x0) */
static inline dd dd_recip(dd b) {
  const dd x0 = dd_from(1.0 / b.h);
  const dd e = dd_sub(dd_from(1.0), dd_mul(b, x0));
  return dd_add(x0, dd_mul(x0, e));
}
/* a / b = a * (1/b), then one correction q + y (a - b q) */
static inline dd dd_div(dd a, dd b) {
  const dd y = dd_recip(b);
  const dd q = dd_mul(a, y);
  const dd r = dd_sub(a, dd_mul(b, q));
  return dd_add(q, dd_mul(y, r));
}
/* sqrt(a): y = a_h * x0 with x0 ~ 1/sqrt(a_h), then y + x0 (a - y^2) / 2 */
static inline dd dd_sqrt(dd a) {
  if (!(a.h > 0)) { dd z = {a.h == 0 ? 0.0 : NAN, 0.0}; return z; }
  const double x0 = 1.0 / sqrt(a.h);
  const double y = a.h * x0;
  const dd yy = two_prod(y, y);
  const dd r = dd_sub(a, yy);
  const dd c = dd_mul(dd_from(0.5 * x0), r);
  return dd_add(dd_from(y), c);
}

/* Ogita-Rump-Oishi Dot2 over rows [r0, r1) of columns a (stride lda) and b:
 * s + c accumulates sum a_r b_r with TwoSum on s and the product/sum errors
 * in c; returned as a DD normalized by FastTwoSum. */
static dd dot2_rows(int64_t r0, int64_t r1, const double* a, int64_t lda,
                    const double* b, int64_t ldb) {
  double s = 0, c = 0;
  for (int64_t r = r0; r < r1; ++r) {
    const dd p = two_prod(a[r * lda], b[r * ldb]);
    const dd t = two_sum(s, p.h);
    s = t.h;
    c += t.l + p.l;
  }
  return fast_two_sum(s, c);
}

/* O2 Gram  G = A^T B  by Dot2 per entry, fixed row partition, partials
 * combined in block order with DD additions.  Within a block the rows are
 * visited in order for all entries at once (the same operation sequence per
 * entry as dot2_rows, only the loop nest is row-major for locality). */
int or_gram_dot2(int64_t m, int ka, const double* A, int64_t lda, int kb,
                 const double* B, int64_t ldb, double* ghi, double* glo) {
  const int64_t np = npart(m);
  const size_t n = (size_t)ka * kb;
  dd* part = (dd*)malloc(sizeof(dd) * ((size_t)np * n + 1));
#pragma omp parallel
  {
    double* s = (double*)malloc(sizeof(double) * (n + 1));
    double* c = (double*)malloc(sizeof(double) * (n + 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t b = 0; b < np; ++b) {
      for (size_t e = 0; e < n; ++e) { s[e] = 0; c[e] = 0; }
      for (int64_t r = pbeg(m, np, b); r < pbeg(m, np, b + 1); ++r) {
        const double* a = A + r * lda;
        const double* bb = B + r * ldb;
        for (int i = 0; i < ka; ++i)
          for (int j = 0; j < kb; ++j) {
            const size_t e = (size_t)i * kb + j;
            const dd p = two_prod(a[i], bb[j]);
            const dd t = two_sum(s[e], p.h);
            s[e] = t.h;
            c[e] += t.l + p.l;
          }
      }
      for (size_t e = 0; e < n; ++e) part[(size_t)b * n + e] = fast_two_sum(s[e], c[e]);
    }
    free(s);
    free(c);
  }
  for (size_t e = 0; e < n; ++e) {
    dd acc = {0, 0};
    for (int64_t b = 0; b < np; ++b) acc = dd_add(acc, part[(size_t)b * n + e]);
    ghi[e] = acc.h;
    if (glo) glo[e] = acc.l;
  }
  free(part);
  return 0;
}

/* binary64 Gram  A^T B  with plain recursive-free summation: serial within each
 * of the fixed row blocks, then block partials summed in order. */
static void gram_f64(int64_t m, int ka, const double* A, int64_t lda, int kb,
                     const double* B, int64_t ldb, double* g) {
  const int64_t np = npart(m);
  const size_t n = (size_t)ka * kb;
  double* part = (double*)calloc((size_t)np * n + 1, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < np; ++b) {
    double* p = part + (size_t)b * n;
    for (int64_t r = pbeg(m, np, b); r < pbeg(m, np, b + 1); ++r)
      for (int i = 0; i < ka; ++i)
        for (int j = 0; j < kb; ++j) p[(size_t)i * kb + j] += A[r * lda + i] * B[r * ldb + j];
  }
  for (size_t e = 0; e < n; ++e) {
    double s = 0;
    for (int64_t b = 0; b < np; ++b) s += part[(size_t)b * n + e];
    g[e] = s;
  }
  free(part);
}

int or_gram_f64(int64_t m, int ka, const double* A, int64_t lda, int kb,
                const double* B, int64_t ldb, double* g) {
  gram_f64(m, ka, A, lda, kb, B, ldb, g);
  return 0;
}

/* binary64 Cholesky with the unpivoted breakdown rule (pivot <= 0 or not
 * finite -> 1-based index). */
static int chol_f64(int k, double* a) {
  for (int j = 0; j < k; ++j) {
    double d = a[j * k + j];
    for (int i = 0; i < j; ++i) d -= a[i * k + j] * a[i * k + j];
    if (!(d > 0) || !isfinite(d)) return j + 1;
    const double rjj = sqrt(d);
    a[j * k + j] = rjj;
    for (int l = j + 1; l < k; ++l) {
      double s = a[j * k + l];
      for (int i = 0; i < j; ++i) s -= a[i * k + j] * a[i * k + l];
      a[j * k + l] = s / rjj;
    }
    for (int l = 0; l < j; ++l) a[j * k + l] = 0;
  }
  return 0;
}

static void trinv_f64(int k, const double* r, double* z) {
  memset(z, 0, sizeof(double) * (size_t)k * k);
  for (int j = 0; j < k; ++j) {
    z[j * k + j] = 1.0 / r[j * k + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0;
      for (int l = i + 1; l <= j; ++l) s += r[i * k + l] * z[l * k + j];
      z[i * k + j] = -s / r[i * k + i];
    }
  }
}

static int chol_dd(int k, dd* a) {
  for (int j = 0; j < k; ++j) {
    dd d = a[j * k + j];
    for (int i = 0; i < j; ++i) d = dd_sub(d, dd_mul(a[i * k + j], a[i * k + j]));
    if (!(d.h > 0) || !isfinite(d.h)) return j + 1;
    const dd rjj = dd_sqrt(d);
    a[j * k + j] = rjj;
    for (int l = j + 1; l < k; ++l) {
      dd s = a[j * k + l];
      for (int i = 0; i < j; ++i) s = dd_sub(s, dd_mul(a[i * k + j], a[i * k + l]));
      a[j * k + l] = dd_div(s, rjj);
    }
    for (int l = 0; l < j; ++l) a[j * k + l] = dd_from(0.0);
  }
  return 0;
}

static void trinv_dd(int k, const dd* r, dd* z) {
  for (size_t e = 0; e < (size_t)k * k; ++e) z[e] = dd_from(0.0);
  for (int j = 0; j < k; ++j) {
    z[j * k + j] = dd_recip(r[j * k + j]);
    for (int i = j - 1; i >= 0; --i) {
      dd s = {0, 0};
      for (int l = i + 1; l <= j; ++l) s = dd_add(s, dd_mul(r[i * k + l], z[l * k + j]));
      z[i * k + j] = dd_neg(dd_div(s, r[i * k + i]));
    }
  }
}

/* SVQB factor of phase II (Sec. 4.2, in the symmetric reading): the
 * eigenpairs M = U L U^T by binary128 Jacobi, Z = U L^{-1/2} U^T = M^{-1/2}
 * and R = U L^{1/2} U^T = M^{1/2}, so that Z^T M Z = I and M = R^T R.
 * Eigenvalues below floor * lambda_max are lifted to that floor (the
 * reading of the rank-deficient case: floor 2^-52 for a binary64 M, 2^-104
 * for a DD one).  a: M (k x k, binary128), destroyed.  Returns 0, or 1 + the
 * index of a non-positive eigenvalue if lambda_max itself is not positive. */
static int svqb_factor_q(int k, f128* a, f128* Z, f128* R, f128 floor_rel) {
  const size_t n = (size_t)k * k;
  f128* v = (f128*)malloc(sizeof(f128) * n + 16);
  jacobi_q(k, a, v);
  int bad = 0;
  f128 lmax = 0;
  for (int i = 0; i < k; ++i)
    if (a[i * k + i] > lmax) lmax = a[i * k + i];
  if (!(lmax > 0) || isinfq(lmax) || isnanq(lmax)) bad = 1;
  for (int i = 0; i < k && !bad; ++i)
    if (!(a[i * k + i] >= floor_rel * lmax)) a[i * k + i] = floor_rel * lmax;
  if (!bad)
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        f128 z = 0, r = 0;
        for (int l = 0; l < k; ++l) {
          const f128 w = v[i * k + l] * v[j * k + l];
          z += w / sqrtq(a[l * k + l]);
          r += w * sqrtq(a[l * k + l]);
        }
        Z[i * k + j] = z;
        R[i * k + j] = r;
      }
  free(v);
  return bad;
}

/* One binary64 pass (phase I then phase II):  C = Y^T X, Xt = X - Y C,
 * M = Xt^T Xt, then Cholesky M = R^T R, Z = R^{-1} (fact 0) or SVQB
 * Z = M^{-1/2}, R = M^{1/2} (fact 1, factored in binary128 from the binary64
 * M), Q = Xt Z.  X may alias Q. */
static int pass_f64(int64_t m, int k, const double* X, int64_t ldx, int ky,
                    const double* Y, int64_t ldy, double* Q, int64_t ldq,
                    double* R, double* C, int exact_gram, int fact, int fused) {
  double* xt = (double*)malloc(sizeof(double) * ((size_t)m * k + 1));
  if (ky > 0) gram_f64(m, ky, Y, ldy, k, X, ldx, C);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)
    for (int j = 0; j < k; ++j) {
      double v = X[r * ldx + j];
      for (int l = 0; l < ky; ++l) v -= Y[r * ldy + l] * C[(size_t)l * k + j];
      xt[(size_t)r * k + j] = v;
    }
  /* exact_gram: M is the binary128 Gram matrix of Xt rounded once to
   * binary64 -- the most accurate M a binary64 pass can be given, so the
   * pass's orthogonality loss is then due to the Cholesky factor and the
   * update alone. */
  if (exact_gram) {
    or_gram_q(m, k, xt, k, k, xt, k, R, NULL);
  } else if (fused && ky > 0) {
    /* fused operations: M from the Gram matrix of [Y | X] of one sweep,
     * M = X^T X - 2 C^T C + C^T (Y^T Y) C (= Xt^T Xt in exact arithmetic) */
    double* syy = (double*)malloc(sizeof(double) * ((size_t)ky * ky + 1));
    double* sc = (double*)malloc(sizeof(double) * ((size_t)ky * k + 1));
    gram_f64(m, k, X, ldx, k, X, ldx, R);
    gram_f64(m, ky, Y, ldy, ky, Y, ldy, syy);
    for (int l = 0; l < ky; ++l)
      for (int j = 0; j < k; ++j) {
        double v = 0;
        for (int q = 0; q < ky; ++q) v += syy[(size_t)l * ky + q] * C[(size_t)q * k + j];
        sc[(size_t)l * k + j] = v;
      }
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        double v = R[(size_t)i * k + j];
        for (int l = 0; l < ky; ++l)
          v -= C[(size_t)l * k + i] * (2.0 * C[(size_t)l * k + j] - sc[(size_t)l * k + j]);
        R[(size_t)i * k + j] = v;
      }
    free(syy);
    free(sc);
  } else {
    gram_f64(m, k, xt, k, k, xt, k, R);
  }
  double* z = (double*)malloc(sizeof(double) * (size_t)k * k + 8);
  if (fact == 1) {
    const size_t n = (size_t)k * k;
    f128* a = (f128*)malloc(sizeof(f128) * n + 16);
    f128* zq = (f128*)malloc(sizeof(f128) * n + 16);
    f128* rq = (f128*)malloc(sizeof(f128) * n + 16);
    for (size_t e = 0; e < n; ++e) a[e] = (f128)R[e];
    const int bad = svqb_factor_q(k, a, zq, rq, ldexpq(1, -52));
    for (size_t e = 0; e < n; ++e) { z[e] = (double)zq[e]; R[e] = (double)rq[e]; }
    free(a); free(zq); free(rq);
    if (bad) { free(z); free(xt); return bad; }
  } else {
    const int info = chol_f64(k, R);
    if (info) { free(z); free(xt); return info; }
    trinv_f64(k, R, z);
  }
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)
    for (int j = 0; j < k; ++j) {
      double s = 0;
      const int iend = fact == 1 ? k - 1 : j;  /* dense Z, or upper-triangular */
      for (int i = 0; i <= iend; ++i) s += xt[(size_t)r * k + i] * z[(size_t)i * k + j];
      Q[r * ldq + j] = s;
    }
  free(z);
  free(xt);
  return 0;
}

/* One DD pass: the same steps with every quantity in DD -- C by Dot2, Xt kept
 * as DD, M from the DD Xt, DD Cholesky and DD inverse, Q = Xt Z rounded to
 * binary64 once.  R and C are returned as hi/lo pairs.
 *
 * corrected: the projection coefficients are D = 2C - S C with S = Y^T Y (by
 * Dot2), the first-order expansion of (Y^T Y)^{-1} Y^T X, so that the part of
 * Xt left in span(Y) is O(||S - I||^2) instead of O(||S - I||) when the stored
 * Y is orthonormal only to binary64 accuracy; D replaces C in Xt and in the
 * returned coefficients.  For an exactly orthonormal Y, D = C. */
static int pass_dd(int64_t m, int k, const double* X, int64_t ldx, int ky,
                   const double* Y, int64_t ldy, double* Q, int64_t ldq,
                   dd* R, dd* C, int corrected, int fact, int fused) {
  const int64_t np = npart(m);
  if (ky > 0) {
    for (int l = 0; l < ky; ++l)
      for (int j = 0; j < k; ++j) {
        dd s = {0, 0};
        for (int64_t b = 0; b < np; ++b)
          s = dd_add(s, dot2_rows(pbeg(m, np, b), pbeg(m, np, b + 1), Y + l, ldy, X + j, ldx));
        C[(size_t)l * k + j] = s;
      }
  }
  dd* C0 = NULL; /* the plain coefficients, kept for the fused M */
  if (ky > 0 && fused) {
    C0 = (dd*)malloc(sizeof(dd) * ((size_t)ky * k + 1));
    memcpy(C0, C, sizeof(dd) * (size_t)ky * k);
  }
  if (ky > 0 && corrected) {
    dd* S = (dd*)malloc(sizeof(dd) * ((size_t)ky * ky + 1));
    for (int l = 0; l < ky; ++l)
      for (int q = 0; q < ky; ++q) {
        dd s = {0, 0};
        for (int64_t b = 0; b < np; ++b)
          s = dd_add(s, dot2_rows(pbeg(m, np, b), pbeg(m, np, b + 1), Y + l, ldy, Y + q, ldy));
        S[(size_t)l * ky + q] = s;
      }
    dd* D = (dd*)malloc(sizeof(dd) * ((size_t)ky * k + 1));
    for (int l = 0; l < ky; ++l)
      for (int j = 0; j < k; ++j) {
        dd s = dd_add(C[(size_t)l * k + j], C[(size_t)l * k + j]);
        for (int q = 0; q < ky; ++q) s = dd_sub(s, dd_mul(S[(size_t)l * ky + q], C[(size_t)q * k + j]));
        D[(size_t)l * k + j] = s;
      }
    memcpy(C, D, sizeof(dd) * (size_t)ky * k);
    free(D);
    free(S);
  }
  dd* xt = (dd*)malloc(sizeof(dd) * ((size_t)m * k + 1));
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)
    for (int j = 0; j < k; ++j) {
      dd v = dd_from(X[r * ldx + j]);
      for (int l = 0; l < ky; ++l) v = dd_sub(v, dd_mul(dd_from(Y[r * ldy + l]), C[(size_t)l * k + j]));
      xt[(size_t)r * k + j] = v;
    }
  const size_t n = (size_t)k * k;
  if (C0) {
    /* fused operations: M from the DD Gram matrix of [Y | X] of one sweep
     * (Dot2 sums), M = X^T X - C^T D with D the (corrected) coefficients
     * (= Xt^T Xt to second order in ||Y^T Y - I||) */
    for (int i = 0; i < k; ++i)
      for (int j = i; j < k; ++j) {
        dd s = {0, 0};
        for (int64_t b = 0; b < np; ++b)
          s = dd_add(s, dot2_rows(pbeg(m, np, b), pbeg(m, np, b + 1), X + i, ldx, X + j, ldx));
        for (int l = 0; l < ky; ++l) s = dd_sub(s, dd_mul(C0[(size_t)l * k + i], C[(size_t)l * k + j]));
        R[(size_t)i * k + j] = s;
        R[(size_t)j * k + i] = s;
      }
    free(C0);
  } else {
    /* M = Xt^T Xt with DD inputs: sum of DD products, DD accumulation per
     * row block, blocks combined in order. */
    dd* part = (dd*)malloc(sizeof(dd) * ((size_t)np * n + 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < np; ++b) {
      dd* p = part + (size_t)b * n;
      for (size_t e = 0; e < n; ++e) p[e] = dd_from(0.0);
      for (int64_t r = pbeg(m, np, b); r < pbeg(m, np, b + 1); ++r)
        for (int i = 0; i < k; ++i)
          for (int j = i; j < k; ++j)
            p[(size_t)i * k + j] = dd_add(p[(size_t)i * k + j], dd_mul(xt[(size_t)r * k + i], xt[(size_t)r * k + j]));
    }
    for (int i = 0; i < k; ++i)
      for (int j = i; j < k; ++j) {
        dd s = {0, 0};
        for (int64_t b = 0; b < np; ++b) s = dd_add(s, part[(size_t)b * n + (size_t)i * k + j]);
        R[(size_t)i * k + j] = s;
        R[(size_t)j * k + i] = s;
      }
    free(part);
  }
  dd* z = (dd*)malloc(sizeof(dd) * (n + 1));
  if (fact == 1) {
    /* SVQB factored in binary128 from the DD M, rounded to DD */
    f128* a = (f128*)malloc(sizeof(f128) * n + 16);
    f128* zq = (f128*)malloc(sizeof(f128) * n + 16);
    f128* rq = (f128*)malloc(sizeof(f128) * n + 16);
    for (size_t e = 0; e < n; ++e) a[e] = (f128)R[e].h + (f128)R[e].l;
    const int bad = svqb_factor_q(k, a, zq, rq, ldexpq(1, -104));
    for (size_t e = 0; e < n; ++e) {
      split_q(zq[e], &z[e].h, &z[e].l);
      split_q(rq[e], &R[e].h, &R[e].l);
    }
    free(a); free(zq); free(rq);
    if (bad) { free(z); free(xt); return bad; }
  } else {
    const int info = chol_dd(k, R);
    if (info) { free(z); free(xt); return info; }
    trinv_dd(k, R, z);
  }
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)
    for (int j = 0; j < k; ++j) {
      dd s = {0, 0};
      const int iend = fact == 1 ? k - 1 : j;  /* dense Z, or upper-triangular */
      for (int i = 0; i <= iend; ++i) s = dd_add(s, dd_mul(xt[(size_t)r * k + i], z[(size_t)i * k + j]));
      Q[r * ldq + j] = s.h + s.l;
    }
  free(z);
  free(xt);
  return 0;
}

/* O2 driver: `passes` repetitions of (phase I if ky > 0 and (pass == 0 or
 * project_each_pass), then phase II).  The first pass runs in DD when dd_first
 * is 1 (with the corrected coefficients of pass_dd when dd_corrected is
 * set), in binary64 with the exactly rounded Gram matrix when dd_first is 2,
 * later passes in binary64 -- the iterated two-phase scheme of
 * Sec. 4.2 cut to `passes` iterations (passes = 2 is CholQR2).
 * Outputs: Q (m x k), R = R_p ... R_1 (k x k, hi/lo), C = total projection
 * coefficients (ky x k, hi/lo) with X = Y C + Q R.  Returns 0, or
 * 100 * (pass + 1) + pivot on breakdown. */
int or_cholqr_steps(int64_t m, int k, const double* X, int64_t ldx, int ky,
                    const double* Y, int64_t ldy, int dd_first, int dd_corrected, int passes,
                    int project_each_pass, double* Q, int64_t ldq, double* rhi,
                    double* rlo, double* chi, double* clo) {
  const size_t n = (size_t)k * k;
  dd* rtot = (dd*)malloc(sizeof(dd) * (n + 1));
  dd* ctot = (dd*)malloc(sizeof(dd) * ((size_t)(ky > 0 ? ky : 1) * k + 1));
  for (size_t e = 0; e < n; ++e) rtot[e] = dd_from(0.0);
  for (int i = 0; i < k; ++i) rtot[i * k + i] = dd_from(1.0);
  for (size_t e = 0; e < (size_t)ky * k; ++e) ctot[e] = dd_from(0.0);
  double* cur = (double*)malloc(sizeof(double) * ((size_t)m * k + 1));
  for (int64_t r = 0; r < m; ++r)
    for (int j = 0; j < k; ++j) cur[(size_t)r * k + j] = X[r * ldx + j];
  dd* rp = (dd*)malloc(sizeof(dd) * (n + 1));
  dd* cp = (dd*)malloc(sizeof(dd) * ((size_t)(ky > 0 ? ky : 1) * k + 1));
  double* rf = (double*)malloc(sizeof(double) * (n + 1));
  double* cf = (double*)malloc(sizeof(double) * ((size_t)(ky > 0 ? ky : 1) * k + 1));
  int status = 0;
  for (int p = 0; p < passes && !status; ++p) {
    const int kyp = (ky > 0 && (p == 0 || project_each_pass)) ? ky : 0;
    int info;
    if (p == 0 && dd_first == 1) {
      info = pass_dd(m, k, cur, k, kyp, Y, ldy, cur, k, rp, cp, dd_corrected, 0, 0);
    } else {
      info = pass_f64(m, k, cur, k, kyp, Y, ldy, cur, k, rf, cf, p == 0 && dd_first == 2, 0, 0);
      for (size_t e = 0; e < n; ++e) rp[e] = dd_from(rf[e]);
      for (size_t e = 0; e < (size_t)kyp * k; ++e) cp[e] = dd_from(cf[e]);
    }
    if (info) { status = 100 * (p + 1) + info; break; }
    /* X_cur = Y C_p + Q_p R_p  =>  C_tot += C_p R_tot, R_tot = R_p R_tot */
    for (int l = 0; l < kyp; ++l)
      for (int j = 0; j < k; ++j) {
        dd s = ctot[(size_t)l * k + j];
        for (int i = 0; i <= j; ++i) s = dd_add(s, dd_mul(cp[(size_t)l * k + i], rtot[(size_t)i * k + j]));
        ctot[(size_t)l * k + j] = s;
      }
    dd* nr = (dd*)malloc(sizeof(dd) * (n + 1));
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        dd s = {0, 0};
        for (int l = i; l <= j; ++l) s = dd_add(s, dd_mul(rp[(size_t)i * k + l], rtot[(size_t)l * k + j]));
        nr[(size_t)i * k + j] = (j >= i) ? s : dd_from(0.0);
      }
    memcpy(rtot, nr, sizeof(dd) * n);
    free(nr);
  }
  if (!status) {
    for (int64_t r = 0; r < m; ++r)
      for (int j = 0; j < k; ++j) Q[r * ldq + j] = cur[(size_t)r * k + j];
    for (size_t e = 0; e < n; ++e) { rhi[e] = rtot[e].h; if (rlo) rlo[e] = rtot[e].l; }
    for (size_t e = 0; e < (size_t)ky * k; ++e) {
      if (chi) chi[e] = ctot[e].h;
      if (clo) clo[e] = ctot[e].l;
    }
  }
  free(rtot); free(ctot); free(cur); free(rp); free(cp); free(rf); free(cf);
  return status;
}

/* O2 iterated scheme (Sec. 4.2: phase I and phase II alternated until the
 * block no longer changes): pass j projects the current block S_j (X, then
 * the previous result) against Y and orthonormalizes it, S_{j+1} =
 * (S_j - Y C_j) Z_j, with the Gram matrix and the factor in binary64
 * (dd = 0) or DD (dd = 1, the corrected coefficients of pass_dd), by
 * Cholesky (fact 0) or SVQB (fact 1, symmetric Z = M^{-1/2}); fused: M from
 * the Gram matrix of [Y | S] of one sweep (the fused operations of Sec. 4.2)
 * instead of the Gram matrix of the projected block.  The pass is
 * applied, then the iteration stops once ||C_j||_F <= eps and
 * ||R_j - I||_F <= eps (the reading of the stop test, with R_j the pass's
 * factor: triangular, or M^{1/2}), or after max_iter passes.
 * Outputs: Q (m x k), R = R_j ... R_1 and C = the total coefficients (dense,
 * hi/lo), X = Y C + Q R; out[0] = passes run, out[1] = 1 if the test held,
 * out[2] = ||C_j||_F, out[3] = ||R_j - I||_F of the last pass.  Returns 0, or
 * 100 * pass + pivot (1-based) on a breakdown. */
int or_iterate(int64_t m, int k, const double* X, int64_t ldx, int ky, const double* Y,
               int64_t ldy, int dd_mode, int fact, int fused, double eps, int max_iter, double* Q,
               int64_t ldq, double* rhi, double* rlo, double* chi, double* clo, double* out) {
  const size_t n = (size_t)k * k;
  const size_t nc = (size_t)(ky > 0 ? ky : 1) * k;
  dd* rtot = (dd*)malloc(sizeof(dd) * (n + 1));
  dd* ctot = (dd*)malloc(sizeof(dd) * (nc + 1));
  dd* rp = (dd*)malloc(sizeof(dd) * (n + 1));
  dd* cp = (dd*)malloc(sizeof(dd) * (nc + 1));
  dd* tmp = (dd*)malloc(sizeof(dd) * (n + nc + 1));
  double* rf = (double*)malloc(sizeof(double) * (n + 1));
  double* cf = (double*)malloc(sizeof(double) * (nc + 1));
  double* cur = (double*)malloc(sizeof(double) * ((size_t)m * k + 1));
  for (size_t e = 0; e < n; ++e) rtot[e] = dd_from(0.0);
  for (int i = 0; i < k; ++i) rtot[i * k + i] = dd_from(1.0);
  for (size_t e = 0; e < nc; ++e) ctot[e] = dd_from(0.0);
  for (int64_t r = 0; r < m; ++r)
    for (int j = 0; j < k; ++j) cur[(size_t)r * k + j] = X[r * ldx + j];
  int status = 0, passes = 0, conv = 0;
  double cn = 0, rd = 0;
  for (int p = 0; p < max_iter; ++p) {
    int info;
    if (dd_mode) {
      info = pass_dd(m, k, cur, k, ky, Y, ldy, cur, k, rp, cp, 1, fact, fused);
    } else {
      info = pass_f64(m, k, cur, k, ky, Y, ldy, cur, k, rf, cf, 0, fact, fused);
      for (size_t e = 0; e < n; ++e) rp[e] = dd_from(rf[e]);
      for (size_t e = 0; e < (size_t)ky * k; ++e) cp[e] = dd_from(cf[e]);
    }
    passes = p + 1;
    if (info) { status = 100 * (p + 1) + info; break; }
    /* this pass's norms */
    double c2 = 0, r2 = 0;
    for (size_t e = 0; e < (size_t)ky * k; ++e) { const double v = cp[e].h + cp[e].l; c2 += v * v; }
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        const double v = (rp[i * k + j].h - (i == j ? 1.0 : 0.0)) + rp[i * k + j].l;
        r2 += v * v;
      }
    cn = sqrt(c2);
    rd = sqrt(r2);
    /* totals: C_tot += C_p R_tot, R_tot = R_p R_tot (dense products in DD) */
    for (int l = 0; l < ky; ++l)
      for (int j = 0; j < k; ++j) {
        dd acc = ctot[(size_t)l * k + j];
        for (int i = 0; i < k; ++i) acc = dd_add(acc, dd_mul(cp[(size_t)l * k + i], rtot[(size_t)i * k + j]));
        tmp[(size_t)l * k + j] = acc;
      }
    for (size_t e = 0; e < (size_t)ky * k; ++e) ctot[e] = tmp[e];
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        dd acc = {0, 0};
        for (int l = 0; l < k; ++l) acc = dd_add(acc, dd_mul(rp[(size_t)i * k + l], rtot[(size_t)l * k + j]));
        tmp[(size_t)i * k + j] = acc;
      }
    for (size_t e = 0; e < n; ++e) rtot[e] = tmp[e];
    if (cn <= eps && rd <= eps) { conv = 1; break; }
  }
  for (int64_t r = 0; r < m; ++r)
    for (int j = 0; j < k; ++j) Q[r * ldq + j] = cur[(size_t)r * k + j];
  for (size_t e = 0; e < n; ++e) { rhi[e] = rtot[e].h; if (rlo) rlo[e] = rtot[e].l; }
  for (size_t e = 0; e < (size_t)ky * k; ++e) {
    if (chi) chi[e] = ctot[e].h;
    if (clo) clo[e] = ctot[e].l;
  }
  out[0] = passes;
  out[1] = conv;
  out[2] = cn;
  out[3] = rd;
  free(rtot); free(ctot); free(rp); free(cp); free(tmp); free(rf); free(cf); free(cur);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Quality measures of a computed factorization  X = Y C + Q R:
 *   out[0] = ||Q^T Q - I||_F          (orthogonality loss, omega)
 *   out[1] = ||X - Y C - Q R||_F / ||X||_F   (reconstruction, rho)
 *   out[2] = ||Y^T Q||_F              (orthogonality against the locked basis)
 *   out[3] = ||X||_F
 * The Gram matrices are taken by Dot2 (error ~ u^2), the residual entries by a
 * compensated dot product, so the measures are accurate far below 1e-16.
 * If E is non-NULL it receives Q^T Q - I (k x k, binary64). */
int or_metrics(int64_t m, int k, const double* Q, int64_t ldq, const double* X,
               int64_t ldx, int ky, const double* Y, int64_t ldy,
               const double* R, const double* C, double* out, double* E) {
  const size_t n = (size_t)k * k;
  double* ghi = (double*)malloc(sizeof(double) * (n + 1));
  double* glo = (double*)malloc(sizeof(double) * (n + 1));
  or_gram_dot2(m, k, Q, ldq, k, Q, ldq, ghi, glo);
  double om = 0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      dd g = {ghi[i * k + j], glo[i * k + j]};
      if (i == j) g = dd_sub(g, dd_from(1.0));
      const double v = g.h + g.l;
      if (E) E[i * k + j] = v;
      om += v * v;
    }
  out[0] = sqrt(om);
  double oy = 0;
  if (ky > 0) {
    double* yq = (double*)malloc(sizeof(double) * ((size_t)ky * k + 1));
    double* yql = (double*)malloc(sizeof(double) * ((size_t)ky * k + 1));
    or_gram_dot2(m, ky, Y, ldy, k, Q, ldq, yq, yql);
    for (size_t e = 0; e < (size_t)ky * k; ++e) {
      const double v = yq[e] + yql[e];
      oy += v * v;
    }
    free(yq);
    free(yql);
  }
  out[2] = sqrt(oy);
  const int64_t np = npart(m);
  double* pr = (double*)calloc((size_t)np + 1, sizeof(double));
  double* px = (double*)calloc((size_t)np + 1, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < np; ++b) {
    double sr = 0, sx = 0;
    for (int64_t r = pbeg(m, np, b); r < pbeg(m, np, b + 1); ++r)
      for (int j = 0; j < k; ++j) {
        double s = X[r * ldx + j], c = 0;
        for (int l = 0; l < ky; ++l) {
          const dd p = two_prod(-Y[r * ldy + l], C[(size_t)l * k + j]);
          const dd t = two_sum(s, p.h);
          s = t.h;
          c += t.l + p.l;
        }
        for (int i = 0; i < k; ++i) {
          const dd p = two_prod(-Q[r * ldq + i], R[(size_t)i * k + j]);
          const dd t = two_sum(s, p.h);
          s = t.h;
          c += t.l + p.l;
        }
        const double res = s + c;
        sr += res * res;
        sx += X[r * ldx + j] * X[r * ldx + j];
      }
    pr[b] = sr;
    px[b] = sx;
  }
  double sr = 0, sx = 0;
  for (int64_t b = 0; b < np; ++b) { sr += pr[b]; sx += px[b]; }
  out[3] = sqrt(sx);
  out[1] = sx > 0 ? sqrt(sr) / sqrt(sx) : sqrt(sr);
  free(pr); free(px); free(ghi); free(glo);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Split-BF16 Gram model: x -> h = bf16_rne(x), l = bf16_rne(x - h) (in fp32);
 * G ~ H^T H + H^T L + L^T H, each product exact in fp32, accumulated in fp32
 * over chunks of `chunk` rows, chunk results summed in binary64.  This pins
 * the error level of the split mode, not its bits. */
static float bf16_rne(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return x; /* inf/nan passthrough */
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  float r;
  memcpy(&r, &u, 4);
  return r;
}

int or_gram_split_bf16(int64_t m, int k, const float* X, int64_t ldx,
                       int64_t chunk, double* G) {
  const size_t n = (size_t)k * k;
  for (size_t e = 0; e < n; ++e) G[e] = 0;
  float* acc = (float*)calloc(n + 1, sizeof(float));
  float* h = (float*)malloc(sizeof(float) * ((size_t)k + 1));
  float* l = (float*)malloc(sizeof(float) * ((size_t)k + 1));
  int64_t inchunk = 0;
  for (int64_t r = 0; r < m; ++r) {
    for (int j = 0; j < k; ++j) {
      const float x = X[r * ldx + j];
      h[j] = bf16_rne(x);
      l[j] = bf16_rne(x - h[j]);
    }
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        acc[(size_t)i * k + j] += h[i] * h[j];
        acc[(size_t)i * k + j] += h[i] * l[j];
        acc[(size_t)i * k + j] += l[i] * h[j];
      }
    if (++inchunk == chunk || r == m - 1) {
      for (size_t e = 0; e < n; ++e) { G[e] += (double)acc[e]; acc[e] = 0; }
      inchunk = 0;
    }
  }
  free(acc); free(h); free(l);
  return 0;
}
