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

// ---------------------------------------------------------------------------
// Wave64 inclusive scans with DPP lane moves (VALU modifiers, no LDS
// round trip): shifts of 1, 2, 4, 8 lanes inside each 16-lane row, then the
// last lane of row 0 / row 2 into rows 1 / 3 (row_bcast:15) and the last lane
// of row 1 into rows 2 and 3 (row_bcast:31).  Lanes without a source read 0,
// the identity of every sum here.  The combination order is fixed, so the
// result depends only on the inputs.
// ---------------------------------------------------------------------------
enum : int {
  kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118,
  kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138
};

template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xF, true);
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = dpp_u32<kCtrl, kRowMask>((uint32_t)v);
  const uint32_t hi = dpp_u32<kCtrl, kRowMask>((uint32_t)(v >> 32));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double v) {
  return __longlong_as_double((long long)dpp_u64<kCtrl, kRowMask>((uint64_t)__double_as_longlong(v)));
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ dd dpp_dd(dd v) {
  return dd_make(dpp_f64<kCtrl, kRowMask>(v.hi), dpp_f64<kCtrl, kRowMask>(v.lo));
}

// one step of a (segmented) scan: this lane's (v, f) combined with the
// DPP-moved value of an earlier lane: v stays if a segment starts here
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void dpp_seg_step(dd &v, uint32_t &f) {
  const dd o = dpp_dd<kCtrl, kRowMask>(v);
  const uint32_t of = dpp_u32<kCtrl, kRowMask>(f);
  if (!f) v = add_fast(o, v);
  f |= of;
}

// inclusive scan of same-sign dd values; f != 0 marks a lane whose value
// starts a new segment (earlier lanes are not added to it or to later lanes)
__device__ __forceinline__ void wave_seg_scan_dd(dd &v, uint32_t &f) {
  dpp_seg_step<kDppRowShr1, 0xF>(v, f);
  dpp_seg_step<kDppRowShr2, 0xF>(v, f);
  dpp_seg_step<kDppRowShr4, 0xF>(v, f);
  dpp_seg_step<kDppRowShr8, 0xF>(v, f);
  dpp_seg_step<kDppRowBcast15, 0xA>(v, f);
  dpp_seg_step<kDppRowBcast31, 0xC>(v, f);
}

// inclusive scan of same-sign dd values (no segments)
__device__ __forceinline__ dd wave_scan_dd(dd v) {
  v = add_fast(dpp_dd<kDppRowShr1, 0xF>(v), v);
  v = add_fast(dpp_dd<kDppRowShr2, 0xF>(v), v);
  v = add_fast(dpp_dd<kDppRowShr4, 0xF>(v), v);
  v = add_fast(dpp_dd<kDppRowShr8, 0xF>(v), v);
  v = add_fast(dpp_dd<kDppRowBcast15, 0xA>(v), v);
  v = add_fast(dpp_dd<kDppRowBcast31, 0xC>(v), v);
  return v;
}

__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t v) {
  v += dpp_u32<kDppRowShr1, 0xF>(v);
  v += dpp_u32<kDppRowShr2, 0xF>(v);
  v += dpp_u32<kDppRowShr4, 0xF>(v);
  v += dpp_u32<kDppRowShr8, 0xF>(v);
  v += dpp_u32<kDppRowBcast15, 0xA>(v);
  v += dpp_u32<kDppRowBcast31, 0xC>(v);
  return v;
}

// the value of the previous lane (0 in lane 0)
__device__ __forceinline__ dd wave_prev_dd(dd v) { return dpp_dd<kDppWaveShr1, 0xF>(v); }
__device__ __forceinline__ uint32_t wave_prev_u32(uint32_t v) {
  return dpp_u32<kDppWaveShr1, 0xF>(v);
}

}  // namespace amdalias
