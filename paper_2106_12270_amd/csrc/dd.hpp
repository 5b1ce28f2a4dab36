// Double-double arithmetic for the device.
//
// A value is the unevaluated sum hi + lo of two binary64 numbers with
// |lo| <= ulp(hi)/2, about 106 significant bits.  The alias-table build keeps
// the total weight W, the bucket size W/N, every prefix sum, split residual
// ("spill") and running residual in this format: the paper fixes only the
// 64-bit type for weights and table rows, and plain binary64 sums lose the
// per-item mass bound at the table sizes served here.
//
// Building blocks: Knuth's TwoSum, Dekker's FastTwoSum and the exact product
// via fused multiply-add; the accurate addition of Hida, Li & Bailey's QD
// library.  The whole library is compiled with -ffp-contract=off, so every
// + and * below is one correctly rounded IEEE operation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amdalias {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd dd_make(double hi, double lo) {
  dd r;
  r.hi = hi;
  r.lo = lo;
  return r;
}

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double v = s - a;
  return dd_make(s, (a - (s - v)) + (b - v));
}

// |a| >= |b| (or a == 0)
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  double s = a + b;
  return dd_make(s, b - (s - a));
}

__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return dd_make(p, __fma_rn(a, b, -p));
}

__device__ __forceinline__ dd operator+(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd operator-(dd a) { return dd_make(-a.hi, -a.lo); }
__device__ __forceinline__ dd operator-(dd a, dd b) { return a + (-b); }

__device__ __forceinline__ dd add_d(dd a, double b) {
  dd s = two_sum(a.hi, b);
  s.lo += a.lo;
  return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return quick_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd div_d(dd a, double b) {
  double q1 = a.hi / b;
  dd p = two_prod(q1, b);
  dd s = two_sum(a.hi, -p.hi);
  s.lo -= p.lo;
  s.lo += a.lo;
  double q2 = (s.hi + s.lo) / b;
  return quick_two_sum(q1, q2);
}

__device__ __forceinline__ bool le(dd a, dd b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo <= b.lo);
}

// a / b rounded to one binary64: long-division step q1, remainder-based
// correction q2, one rounding of q1 + q2 (the correctly rounded quotient
// whenever a and b are plain doubles).
__device__ __forceinline__ double quot(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = a - mul_d(b, q1);
  double q2 = r.hi / b.hi;
  return q1 + q2;
}

// Divisor prepared once for many quotients: its dd value, the correctly
// rounded reciprocal of its high part, and whether that reciprocal may be
// used (no overflow or underflow near it).
struct Divisor {
  double hi, lo, inv;
  bool mk;
};

__device__ __forceinline__ Divisor make_divisor(dd b) {
  Divisor d;
  d.hi = b.hi;
  d.lo = b.lo;
  d.inv = 1.0 / b.hi;
  d.mk = b.hi >= 0x1p-1000 && b.hi <= 0x1p+1000;
  return d;
}

// a / b rounded to one binary64 without a division.  Markstein's correction
// (P. Markstein, IBM J. Res. Dev. 34(1), 1990): with y = RN(1/b) and
// q0 = RN(a * y), within one ulp of a/b, the remainder r = a - b*q0 is exact
// (one fma) and RN(q0 + r*y) is the correctly rounded a/b.  The low parts of
// a and b enter the remainder as first-order terms.  So the result is the
// correctly rounded quotient whenever a and b are plain doubles, and within
// one unit in the last place of the dd quotient otherwise.  Outside the range
// where the theorem's no-underflow assumption holds, an IEEE division step
// with the same remainder correction is used.
__device__ __forceinline__ double quot_fast(dd a, const Divisor &b) {
  if (b.mk && (a.hi == 0.0 || fabs(a.hi) >= 0x1p-900)) {
    const double q0 = a.hi * b.inv;
    const double r = __fma_rn(-b.hi, q0, a.hi);
    const double e = (r + a.lo) - b.lo * q0;
    return __fma_rn(e, b.inv, q0);
  }
  const double q1 = a.hi / b.hi;
  const dd p = two_prod(b.hi, q1);
  const double e = (((a.hi - p.hi) - p.lo) + a.lo) - b.lo * q1;
  return q1 + e * b.inv;
}

// Addition without the renormalisation of the low parts (QD's sloppy add):
// error bounded by a few units of 2^-104 times |a| + |b|, exact whenever the
// operands and the sum fit in the two components.
__device__ __forceinline__ dd add_fast(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  return quick_two_sum(s.hi, s.lo + (a.lo + b.lo));
}

__device__ __forceinline__ double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

// ---------------------------------------------------------------------------
// Wave64 shuffles of dd values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ dd shfl_up(dd v, int d) {
  return dd_make(__shfl_up(v.hi, d, 64), __shfl_up(v.lo, d, 64));
}
__device__ __forceinline__ dd shfl_xor(dd v, int m) {
  return dd_make(__shfl_xor(v.hi, m, 64), __shfl_xor(v.lo, m, 64));
}
__device__ __forceinline__ dd shfl(dd v, int src) {
  return dd_make(__shfl(v.hi, src, 64), __shfl(v.lo, src, 64));
}

// Inclusive scan across the 64 lanes (Hillis-Steele, fixed pattern: the
// result depends only on the inputs, never on timing).
__device__ __forceinline__ dd wave_inclusive_scan(dd v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    dd o = shfl_up(v, d);
    if (lane >= d) v = o + v;
  }
  return v;
}

// Sum over the 64 lanes (butterfly; every lane gets the same value).
__device__ __forceinline__ dd wave_sum(dd v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    dd o = shfl_xor(v, m);
    // combine in lane order so both partners compute the identical sum
    v = ((__lane_id() & m) == 0) ? (v + o) : (o + v);
  }
  return v;
}

// wave_sum for terms of one sign (all partial sums then have that sign, and
// the same-sign addition add_fast keeps the full dd accuracy).
__device__ __forceinline__ dd wave_sum_fast(dd v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    dd o = shfl_xor(v, m);
    v = ((__lane_id() & m) == 0) ? add_fast(v, o) : add_fast(o, v);
  }
  return v;
}

}  // namespace amdalias
