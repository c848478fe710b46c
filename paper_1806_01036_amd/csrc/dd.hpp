// Double-double (DD) arithmetic for gfx950, FMA based.
//
// A DD value is an unevaluated sum hi + lo of two binary64 numbers with
// |lo| <= ulp(hi)/2 (the representation the paper's extended-precision
// kernels use, Sec. 4.2).  The exact transformations are:
//   two_sum      Knuth's branch-free error-free sum,
//   fast_two_sum Dekker's sum for |a| >= |b|,
//   two_prod     exact product via one FMA.
// dd_add / dd_mul follow the accurate double-word algorithms of Joldes,
// Muller and Popescu (2017); dd_recip / dd_div / dd_sqrt are single
// Newton-Raphson corrections from a binary64 seed, as Sec. 4.2 prescribes.
//
// Every translation unit that includes this header must be compiled with
// floating-point contraction disabled (-ffp-contract=off): a contracted
// `a*b - c` inside two_sum or fast_two_sum destroys the error terms.
#pragma once
#include <hip/hip_runtime.h>

struct dd_t {
  double hi, lo;
};

__device__ __forceinline__ dd_t dd_make(double h, double l) { return dd_t{h, l}; }
__device__ __forceinline__ dd_t dd_from(double a) { return dd_t{a, 0.0}; }

__device__ __forceinline__ dd_t two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return dd_t{s, e};
}

__device__ __forceinline__ dd_t fast_two_sum(double a, double b) {
  const double s = a + b;
  const double e = b - (s - a);
  return dd_t{s, e};
}

__device__ __forceinline__ dd_t two_prod(double a, double b) {
  const double p = a * b;
  const double e = __builtin_fma(a, b, -p);
  return dd_t{p, e};
}

__device__ __forceinline__ dd_t dd_add(dd_t a, dd_t b) {
  const dd_t s = two_sum(a.hi, b.hi);
  const dd_t t = two_sum(a.lo, b.lo);
  const double c = s.lo + t.hi;
  const dd_t v = fast_two_sum(s.hi, c);
  const double w = t.lo + v.lo;
  return fast_two_sum(v.hi, w);
}

__device__ __forceinline__ dd_t dd_neg(dd_t a) { return dd_t{-a.hi, -a.lo}; }
__device__ __forceinline__ dd_t dd_sub(dd_t a, dd_t b) { return dd_add(a, dd_neg(b)); }

__device__ __forceinline__ dd_t dd_mul(dd_t a, dd_t b) {
  dd_t c = two_prod(a.hi, b.hi);
  const double t = __builtin_fma(a.hi, b.lo, a.lo * b.hi);
  return fast_two_sum(c.hi, c.lo + t);
}

__device__ __forceinline__ dd_t dd_mul_d(dd_t a, double b) {
  dd_t c = two_prod(a.hi, b);
  return fast_two_sum(c.hi, __builtin_fma(a.lo, b, c.lo));
}

// 1/b: x1 = x0 + x0 (1 - b x0), the residual 1 - b x0 formed in DD.
__device__ __forceinline__ dd_t dd_recip(dd_t b) {
  const double x0 = 1.0 / b.hi;
  const dd_t e = dd_sub(dd_from(1.0), dd_mul_d(b, x0));
  return dd_add(dd_from(x0), dd_mul_d(e, x0));
}

// a/b = a (1/b) corrected once: q + y (a - b q).
__device__ __forceinline__ dd_t dd_div(dd_t a, dd_t b) {
  const dd_t y = dd_recip(b);
  const dd_t q = dd_mul(a, y);
  const dd_t r = dd_sub(a, dd_mul(b, q));
  return dd_add(q, dd_mul(y, r));
}

// 1/sqrt(a): y1 = y0 + y0 (1 - a y0^2) / 2 from y0 = 1/sqrt(a.hi), the
// residual 1 - a y0^2 formed in DD.
__device__ __forceinline__ dd_t dd_rsqrt(dd_t a) {
  const double y0 = 1.0 / sqrt(a.hi);
  const dd_t y2 = two_prod(y0, y0);
  const dd_t e = dd_sub(dd_from(1.0), dd_mul(a, y2));
  return dd_add(dd_from(y0), dd_mul_d(e, 0.5 * y0));
}

// sqrt(a) = y + x0 (a - y^2)/2 with x0 ~ 1/sqrt(a.hi), y = a.hi x0.
__device__ __forceinline__ dd_t dd_sqrt(dd_t a) {
  if (!(a.hi > 0.0)) return dd_t{a.hi == 0.0 ? 0.0 : __builtin_nan(""), 0.0};
  const double x0 = 1.0 / sqrt(a.hi);
  const double y = a.hi * x0;
  const dd_t r = dd_sub(a, two_prod(y, y));
  return dd_add(dd_from(y), dd_mul_d(r, 0.5 * x0));
}

// Dot2 accumulation step (Ogita-Rump-Oishi) with the product error folded
// into the TwoSum correction: (s, c) += a*b.  The second difference of
// TwoSum, p - bb, and the product error a*b - p are combined exactly in
// one FMA, a*b - bb; its rounding is O(u^2 |a b|), the order of Dot2's own
// error term.  8 VALU instructions.
__device__ __forceinline__ void dot2_step(double& s, double& c, double a, double b) {
  const double p = a * b;
  const double sn = s + p;
  const double bb = sn - s;
  const double d1 = s - (sn - bb);
  const double d2 = __builtin_fma(a, b, -bb);
  c = c + (d1 + d2);
  s = sn;
}

// Normalize a Dot2 accumulator (s, c) into a DD value without assuming
// |s| >= |c| (s may have cancelled).
__device__ __forceinline__ dd_t dot2_finish(double s, double c) { return two_sum(s, c); }
