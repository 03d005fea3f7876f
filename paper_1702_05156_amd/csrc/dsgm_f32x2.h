// dsgm_f32x2.h -- compensated single-precision arithmetic (internal).
//
// A value is the unevaluated sum hi + lo of two floats with |lo| <= ulp(hi)/2
// (a "double-float", about 48 significant bits).  Every operation below is
// built from the classic error-free transformations, each of which returns a
// rounded result together with its exact rounding error:
//
//   two_sum(a, b)       s + e = a + b exactly, s = fl(a + b)    (Knuth; 6 ops)
//   fast_two_sum(a, b)  the same when |a| >= |b|               (Dekker; 3 ops)
//   two_prod(a, b)      p + e = a * b exactly, e = fma(a, b, -p)   (2 ops)
//
// and the products and sums of pairs follow Dekker's double-length routines
// (the cross terms of a product accumulated by fused multiply-adds, the low
// parts of a sum added to the two-sum's error before one renormalisation).
// The relative error of each operation is a few units of 2^-48, against 2^-53
// for binary64: the DSGM update (means and variances blended with weights in
// [0, 1], a contraction) stays within about 1e-13 of its FP64 evaluation.
//
// The library is compiled without floating-point contraction, so the compiler
// keeps every rounding written here; the fused multiply-adds are explicit.
#pragma once

#include <hip/hip_runtime.h>

namespace dsgm {

struct alignas(8) f32x2 {
  float hi, lo;

  f32x2() = default;
  __host__ __device__ constexpr f32x2(float h, float l) : hi(h), lo(l) {}
  // the nearest pair to a double: hi = fl32(v), lo = fl32(v - hi); v - hi is
  // exact in FP64 and hi + lo is exact in FP64 as well (at most 53 bits)
  __host__ __device__ explicit f32x2(double v) : hi(float(v)), lo(float(v - double(float(v)))) {}
  __host__ __device__ explicit f32x2(float v) : hi(v), lo(0.f) {}
  __host__ __device__ explicit f32x2(int v) : f32x2(double(v)) {}
  // one rounding of hi + lo to FP32 (hi itself for a normalised pair)
  __host__ __device__ explicit operator float() const { return hi + lo; }
  // exact for a normalised pair
  __host__ __device__ explicit operator double() const { return double(hi) + double(lo); }
};

namespace x2 {

__device__ __forceinline__ f32x2 fast_two_sum(float a, float b) {
  const float s = a + b;
  return f32x2(s, b - (s - a));
}

__device__ __forceinline__ f32x2 two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return f32x2(s, (a - (s - bb)) + (b - bb));
}

// a + b
__device__ __forceinline__ f32x2 add(f32x2 a, f32x2 b) {
  const f32x2 s = two_sum(a.hi, b.hi);
  return fast_two_sum(s.hi, s.lo + (a.lo + b.lo));
}

// a - b
__device__ __forceinline__ f32x2 sub(f32x2 a, f32x2 b) { return add(a, f32x2(-b.hi, -b.lo)); }

// x - m for a float x
__device__ __forceinline__ f32x2 sub(float x, f32x2 m) {
  const f32x2 s = two_sum(x, -m.hi);
  return fast_two_sum(s.hi, s.lo - m.lo);
}

// a * b
__device__ __forceinline__ f32x2 mul(f32x2 a, f32x2 b) {
  const float p = a.hi * b.hi;
  float e = __builtin_fmaf(a.hi, b.hi, -p);
  e = __builtin_fmaf(a.hi, b.lo, e);
  e = __builtin_fmaf(a.lo, b.hi, e);
  return fast_two_sum(p, e);
}

// a * b for a float b
__device__ __forceinline__ f32x2 mul(f32x2 a, float b) {
  const float p = a.hi * b;
  float e = __builtin_fmaf(a.hi, b, -p);
  e = __builtin_fmaf(a.lo, b, e);
  return fast_two_sum(p, e);
}

// a * a
__device__ __forceinline__ f32x2 sqr(f32x2 a) {
  const float p = a.hi * a.hi;
  float e = __builtin_fmaf(a.hi, a.hi, -p);
  e = __builtin_fmaf(a.hi + a.hi, a.lo, e);
  return fast_two_sum(p, e);
}

// comparisons of normalised pairs: lexicographic on (hi, lo)
__device__ __forceinline__ bool lt(f32x2 a, f32x2 b) {
  return (a.hi < b.hi) | ((a.hi == b.hi) & (a.lo < b.lo));
}
__device__ __forceinline__ bool le(f32x2 a, f32x2 b) {
  return (a.hi < b.hi) | ((a.hi == b.hi) & (a.lo <= b.lo));
}

__device__ __forceinline__ f32x2 sel(bool c, f32x2 a, f32x2 b) {
  return f32x2(c ? a.hi : b.hi, c ? a.lo : b.lo);
}

}  // namespace x2

// operators for the generic parts of the kernels (the adjoint sweep)
__device__ __forceinline__ f32x2 operator+(f32x2 a, f32x2 b) { return x2::add(a, b); }
__device__ __forceinline__ f32x2 operator-(f32x2 a, f32x2 b) { return x2::sub(a, b); }
__device__ __forceinline__ f32x2 operator*(f32x2 a, f32x2 b) { return x2::mul(a, b); }

template <typename T>
struct is_f32x2 {
  static constexpr bool value = false;
};
template <>
struct is_f32x2<f32x2> {
  static constexpr bool value = true;
};

}  // namespace dsgm
