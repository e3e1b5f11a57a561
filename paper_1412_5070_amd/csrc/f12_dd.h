// Double-double arithmetic for gfx950 device code (and host code).
// A value is hi + lo with |lo| <= ulp(hi)/2; error-free transforms use fma.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace f12 {

// Error-free transforms need every product and sum rounded on its own: the
// device compiler's default contraction (-ffp-contract=fast) would fuse a
// product from one statement into the next addition and break them.
#define F12_NO_CONTRACT _Pragma("clang fp contract(off)")

struct dd {
  double hi, lo;
};

__host__ __device__ inline dd dd_make(double x) { return dd{x, 0.0}; }

__host__ __device__ inline dd two_sum(double a, double b) {
  F12_NO_CONTRACT;
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return dd{s, e};
}

__host__ __device__ inline dd quick_two_sum(double a, double b) {
  F12_NO_CONTRACT;
  double s = a + b;
  return dd{s, b - (s - a)};
}

__host__ __device__ inline dd two_prod(double a, double b) {
  F12_NO_CONTRACT;
  double p = a * b;
  return dd{p, fma(a, b, -p)};
}

__host__ __device__ inline dd dd_add(dd a, dd b) {
  F12_NO_CONTRACT;
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}

__host__ __device__ inline dd dd_add(dd a, double b) {
  F12_NO_CONTRACT;
  dd s = two_sum(a.hi, b);
  s.lo += a.lo;
  return quick_two_sum(s.hi, s.lo);
}

__host__ __device__ inline dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
__host__ __device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

__host__ __device__ inline dd dd_mul(dd a, dd b) {
  F12_NO_CONTRACT;
  dd p = two_prod(a.hi, b.hi);
  p.lo = fma(a.hi, b.lo, fma(a.lo, b.hi, p.lo));
  return quick_two_sum(p.hi, p.lo);
}

__host__ __device__ inline dd dd_mul(dd a, double b) {
  F12_NO_CONTRACT;
  dd p = two_prod(a.hi, b);
  p.lo = fma(a.lo, b, p.lo);
  return quick_two_sum(p.hi, p.lo);
}

// a + b*c in DD
__host__ __device__ inline dd dd_fma(dd a, dd b, dd c) { return dd_add(a, dd_mul(b, c)); }

__host__ __device__ inline dd dd_div(dd a, dd b) {
  F12_NO_CONTRACT;
  double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul(b, q1));
  double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul(b, q2));
  double q3 = r.hi / b.hi;
  dd q = quick_two_sum(q1, q2);
  return dd_add(q, q3);
}

__host__ __device__ inline dd dd_div(dd a, double b) {
  F12_NO_CONTRACT;
  double q1 = a.hi / b;
  dd p = two_prod(q1, b);
  dd s = two_sum(a.hi, -p.hi);
  s.lo = s.lo - p.lo + a.lo;
  double q2 = (s.hi + s.lo) / b;
  return quick_two_sum(q1, q2);
}

__host__ __device__ inline dd dd_sqrt(dd a) {
  F12_NO_CONTRACT;
  if (a.hi <= 0.0) return dd{0.0, 0.0};
  double x = sqrt(a.hi);
  dd xx = two_prod(x, x);
  double r = ((a.hi - xx.hi) - xx.lo + a.lo) / (2.0 * x);
  return quick_two_sum(x, r);
}

// ln 2 to DD
__host__ __device__ inline dd dd_ln2() { return dd{6.931471805599452862e-01, 2.319046813846299558e-17}; }

// exp(a): a = k ln2 + r, |r| <= ln2/2, r/512, Taylor to 1e-34, square 9 times.
__host__ __device__ inline dd dd_exp(dd a) {
  F12_NO_CONTRACT;
  if (a.hi < -745.0) return dd{0.0, 0.0};
  if (a.hi > 709.0) return dd{INFINITY, 0.0};
  double k = rint(a.hi / 6.931471805599452862e-01);
  dd r = dd_sub(a, dd_mul(dd_ln2(), k));
  r.hi = ldexp(r.hi, -9);
  r.lo = ldexp(r.lo, -9);
  // s = exp(r) - 1
  dd term = r;
  dd s = r;
  for (int i = 2; i <= 12; ++i) {
    term = dd_div(dd_mul(term, r), (double)i);
    s = dd_add(s, term);
  }
  for (int i = 0; i < 9; ++i) s = dd_add(dd_mul(s, s), dd_mul(s, 2.0));
  s = dd_add(s, 1.0);
  int ki = (int)k;
  return dd{ldexp(s.hi, ki), ldexp(s.lo, ki)};
}

// log(a) for a > 0: Newton y <- y + a exp(-y) - 1, twice from the binary64 log.
__host__ __device__ inline dd dd_log(dd a) {
  F12_NO_CONTRACT;
  dd y = dd_make(log(a.hi));
  for (int i = 0; i < 2; ++i) {
    dd e = dd_exp(dd_neg(y));
    y = dd_add(dd_add(y, dd_mul(a, e)), -1.0);
  }
  return y;
}

__host__ __device__ inline double dd_to_double(dd a) { return a.hi + a.lo; }

}  // namespace f12
