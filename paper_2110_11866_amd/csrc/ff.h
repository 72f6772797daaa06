// Float-float ("double-float") numbers for the compensated scan: a value is the unevaluated
// sum h + l of two float32 numbers with |l| <= ulp(h) / 2. Sums and products are formed with
// error-free transformations: Knuth's TwoSum (the exact rounding error of a float32 addition)
// and the fused multiply-add form of Dekker's TwoProduct (the exact rounding error of a float32
// product), then renormalised with Dekker's Fast2Sum. Every operation is float32 arithmetic;
// the precision is about 2^-44 relative, enough that the scan's rounding stays below the input
// quantisation of 16-bit signals. Contraction is switched off inside each operation: fusing a
// product into a following sum would destroy the exact error terms.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace mk {
namespace {

struct ff {
  float h, l;

  ff() = default;
  __device__ constexpr ff(float x) : h(x), l(0.0f) {}
  __device__ constexpr ff(float hi, float lo) : h(hi), l(lo) {}
  // small integer constants (0, 1)
  template <typename I, typename std::enable_if<std::is_integral<I>::value, int>::type = 0>
  __device__ constexpr ff(I x) : h((float)x), l(0.0f) {}
  // from a float64 value (a carry): the float32 nearest to it and the float32 nearest to the rest
  __device__ explicit ff(double x) : h((float)x), l((float)(x - (double)(float)x)) {}
  __device__ explicit operator double() const { return (double)h + (double)l; }
  __device__ explicit operator float() const { return h + l; }

  // s + e = a + b exactly (Knuth)
  static __device__ __forceinline__ ff two_sum(float a, float b) {
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return ff(s, e);
  }
  // s + e = a + b exactly when |a| >= |b| or a == 0 (Dekker)
  static __device__ __forceinline__ ff fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
    const float s = a + b;
    const float e = b - (s - a);
    return ff(s, e);
  }

  friend __device__ __forceinline__ ff operator-(ff a) { return ff(-a.h, -a.l); }
  // sum with both parts' errors carried (the accurate float-float addition)
  friend __device__ __forceinline__ ff operator+(ff a, ff b) {
#pragma clang fp contract(off)
    ff s = two_sum(a.h, b.h);
    const ff t = two_sum(a.l, b.l);
    s = fast_two_sum(s.h, s.l + t.h);
    return fast_two_sum(s.h, s.l + t.l);
  }
  friend __device__ __forceinline__ ff operator-(ff a, ff b) { return a + (-b); }
  // product: the exact product of the high parts (p + e), the cross terms added to e
  friend __device__ __forceinline__ ff operator*(ff a, ff b) {
#pragma clang fp contract(off)
    const float p = a.h * b.h;
    float e = __builtin_fmaf(a.h, b.h, -p);
    e = __builtin_fmaf(a.h, b.l, e);
    e = __builtin_fmaf(a.l, b.h, e);
    return fast_two_sum(p, e);
  }
  friend __device__ __forceinline__ ff fma(ff a, ff b, ff c) { return a * b + c; }
};

}  // namespace
}  // namespace mk
