// rounding.hpp -- FP64 directed rounding on gfx950 (CDNA4).
//
// Outward rounding of every bound (Sec. 3.2, eq 25-27) is obtained by running
// the whole kernel with the FP64 rounding field of the wave's MODE register set
// to "toward -infinity" (set_fp64_round_down(), called once at kernel entry).
// Every FP64 arithmetic operation of the interval path is then ONE hardware
// instruction issued through inline assembly, so that the compiler neither
// folds nor reorders it under a round-to-nearest assumption:
//
//   rd(x)       = the instruction itself;
//   ru(a op b)  = -rd(-(a op b)), i.e. the same instruction with negated
//                 source modifiers, which costs nothing.
//
// Upper bounds are therefore carried NEGATED throughout the device code
// (see interval.hpp): an interval [lo, hi] is stored as (lo, nhi = -hi), and
// every bound of every operation is a single round-down instruction.
//
// The FP32 rounding field is left at round-to-nearest-even, so the
// single-precision preconditioner (ordinary compiler-generated float code) is
// unaffected.  FP64 denormals stay enabled (the MODE denormal bits are not
// touched).  No compiler-generated FP64 add/sub/mul/fma/div may appear in code
// that runs after set_fp64_round_down(); conversions float<->double, compares,
// min/max and sign manipulation are rounding-independent (float->double is
// exact; double->float uses the FP32 field).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibb {

// MODE register, FP_ROUND field bits [3:2] (FP64/FP16 rounding): 2 = toward -inf.
__device__ __forceinline__ void set_fp64_round_down() {
  asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2" ::: "memory");
}

// The FP64/FP16 rounding field of the wave's MODE register (2 = toward
// -infinity).  The search kernels read it back when their waves finish: a
// value other than 2 means some code or event changed the mode under the
// kernel, and the search reports an error instead of a possibly wrong list.
__device__ __forceinline__ unsigned fp64_round_field() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_MODE, 2, 2)" : "=s"(v));
  return v;
}

// ---- one rounded instruction each; R(x) = x rounded toward -infinity ----
__device__ __forceinline__ double radd(double a, double b) {  // R(a + b)
  double r;
  asm("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double rsub(double a, double b) {  // R(a - b)
  double r;
  asm("v_add_f64 %0, %1, -%2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double rmul(double a, double b) {  // R(a * b)
  double r;
  asm("v_mul_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double rmul_neg(double a, double b) {  // R(-(a * b))
  double r;
  asm("v_mul_f64 %0, -%1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double rmul_abs(double a, double b) {  // R(|a| * b)
  double r;
  asm("v_mul_f64 %0, |%1|, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double rfma(double a, double b, double c) {  // R(a*b + c)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ double rfma_na(double a, double b, double c) {  // R(-a*b + c)
  double r;
  asm("v_fma_f64 %0, -%1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Minimum / maximum of two non-NaN doubles: the instructions the compiler
// would choose, written out so that it adds no canonicalising copies of
// operands produced by the asm statements above.
__device__ __forceinline__ double dmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double dmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

__device__ __forceinline__ double bits_to_f64(uint64_t u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ uint64_t f64_to_bits(double d) { return (uint64_t)__double_as_longlong(d); }

// 2^k as a double for k in [-1074, 1023].
__device__ __forceinline__ double pow2(int k) {
  if (k >= -1022) return bits_to_f64((uint64_t)(k + 1023) << 52);
  return bits_to_f64(1ull << (k + 1074));
}

// Split |x| (finite, non-zero) into m in [1,2) and an exponent e: |x| = m 2^e.
__device__ __forceinline__ double frexp12(double x, int& e) {
  uint64_t u = f64_to_bits(x) & 0x7fffffffffffffffull;
  int E = (int)(u >> 52);
  int adj = 0;
  if (E == 0) {  // subnormal: scale by 2^64 (exact), then read the exponent
    u = f64_to_bits(rmul(bits_to_f64(u), bits_to_f64(0x43f0000000000000ull)));
    E = (int)(u >> 52);
    adj = 64;
  }
  e = E - 1023 - adj;
  return bits_to_f64((u & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
}

// Neighbours of a positive normal double.
__device__ __forceinline__ double next_up_pos(double q) { return bits_to_f64(f64_to_bits(q) + 1); }
__device__ __forceinline__ double next_dn_pos(double q) { return bits_to_f64(f64_to_bits(q) - 1); }

// For ma, mb in [1,2): the largest double q with q <= ma/mb (up = false), or
// the smallest with q >= ma/mb (up = true).  The residual ma - q*mb is formed
// with one fused multiply-add; its sign is exact for q within a few units in
// the last place of ma/mb, which the Newton refinement guarantees.
__device__ __forceinline__ double quot12(double ma, double mb, bool up) {
  double y = __builtin_amdgcn_rcp(mb);
  double e = rfma_na(mb, y, 1.0);
  y = rfma(y, e, y);
  e = rfma_na(mb, y, 1.0);
  y = rfma(y, e, y);
  double q = rmul(ma, y);
  double r = rfma_na(q, mb, ma);
  q = rfma(r, y, q);
  // q*mb <= ma  <=>  ma - q*mb >= 0
  for (int it = 0; it < 4; ++it) {
    double rq = rfma_na(q, mb, ma);
    if (!up) {
      if (rq < 0.0) { q = next_dn_pos(q); continue; }
      double q1 = next_up_pos(q);
      if (rfma_na(q1, mb, ma) >= 0.0) { q = q1; continue; }
    } else {
      if (rq > 0.0) { q = next_up_pos(q); continue; }
      double q1 = next_dn_pos(q);
      if (rfma_na(q1, mb, ma) <= 0.0) { q = q1; continue; }
    }
    break;
  }
  return q;
}

// t * 2^e for t > 0 (itself a directed rounding of the exact value in the
// same direction), e in [-2200, 2200], rounded down (up = false) or up: the
// first scaling stays in the normal range and is exact, the second rounds once.
__device__ __forceinline__ double scale2(double t, int e, bool up) {
  int e1 = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
  double s = rmul(t, pow2(e1));
  int e2 = e - e1;
  if (e2 == 0) return s;
  e2 = e2 < -1074 ? -1074 : (e2 > 1023 ? 1023 : e2);
  return up ? -rmul_neg(s, pow2(e2)) : rmul(s, pow2(e2));
}

// Correctly rounded quotients of finite a and non-zero finite b.
__device__ __forceinline__ double rd_div(double a, double b) {
  if (a == 0.0) {
    bool negz = (f64_to_bits(a) ^ f64_to_bits(b)) >> 63;
    return negz ? -0.0 : 0.0;
  }
  bool neg = ((f64_to_bits(a) ^ f64_to_bits(b)) >> 63) != 0;
  int ea, eb;
  double ma = frexp12(a, ea), mb = frexp12(b, eb);
  // positive quotient: round the magnitude down; negative: round it up, negate
  double q = quot12(ma, mb, neg);
  double r = scale2(q, ea - eb, neg);
  return neg ? -r : r;
}
__device__ __forceinline__ double ru_div(double a, double b) { return -rd_div(-a, b); }

}  // namespace ibb
