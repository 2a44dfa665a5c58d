// interval.hpp -- FP64 interval arithmetic with outward rounding (Sec. 2.2
// eq 3-10, Sec. 3.2 eq 25-27) for kernels running with the FP64 rounding mode
// set toward -infinity (rounding.hpp).
//
// An interval [lo, hi] is held as (lo, nhi) with nhi = -hi, so that the upper
// bound of every operation, ru(.) = -rd(-.), is again a single round-down
// instruction.  Each function below states the bound it computes; R(x) is x
// rounded toward -infinity.
#pragma once
#include "rounding.hpp"

namespace ibb {

struct iv {
  double lo;   // lower bound
  double nhi;  // negated upper bound
};

__device__ __forceinline__ iv make_iv(double lo, double hi) { return {lo, -hi}; }
__device__ __forceinline__ iv point_iv(double x) { return {x, -x}; }
__device__ __forceinline__ double hi_of(iv x) { return -x.nhi; }
__device__ __forceinline__ bool has_zero(iv x) { return x.lo <= 0.0 && x.nhi <= 0.0; }
__device__ __forceinline__ bool is_zero(iv x) { return x.lo == 0.0 && x.nhi == 0.0; }

// eq (25): [a,b] + [c,d] = [R(a+c), -R(-b-d)]
__device__ __forceinline__ iv iadd(iv x, iv y) { return {radd(x.lo, y.lo), radd(x.nhi, y.nhi)}; }

// eq (26): [a,b] - [c,d] = [R(a-d), -R(c-b)]
__device__ __forceinline__ iv isub(iv x, iv y) { return {radd(x.lo, y.nhi), radd(x.nhi, y.lo)}; }

// eq (27): lower bound = min of the round-down products, upper bound = max of
// the round-up products, for the four endpoint pairs.
__device__ __forceinline__ iv imul(iv x, iv y) {
  double l1 = rmul(x.lo, y.lo);        // R(a c)
  double l2 = rmul_neg(x.lo, y.nhi);   // R(a d)
  double l3 = rmul_neg(x.nhi, y.lo);   // R(b c)
  double l4 = rmul(x.nhi, y.nhi);      // R(b d)
  double u1 = rmul_neg(x.lo, y.lo);    // R(-a c)
  double u2 = rmul(x.lo, y.nhi);       // R(-a d)
  double u3 = rmul(x.nhi, y.lo);       // R(-b c)
  double u4 = rmul_neg(x.nhi, y.nhi);  // R(-b d)
  return {fmin(fmin(l1, l2), fmin(l3, l4)), fmin(fmin(u1, u2), fmin(u3, u4))};
}

// Point times interval (the four products reduce to two by the sign of y).
__device__ __forceinline__ iv pmul(double y, iv x) {
  bool pos = !(y < 0.0);
  double a = pos ? x.lo : x.nhi;
  double b = pos ? x.nhi : x.lo;
  return {rmul_abs(y, a), rmul_abs(y, b)};
}

// t <- R(t u), p-1 times, starting from s (left-to-right chained bound).
__device__ __forceinline__ double chain(double s, double u, int p) {
  double t = s;
  for (int i = 1; i < p; ++i) t = rmul(t, u);
  return t;
}

// Power X^p, p >= 1.  Odd powers are monotone: each endpoint e maps to the
// chain e * |e| * ... .  Even powers are taken over |X|: [mn^p, m^p] with
// m = max |endpoint| and mn = min |endpoint| (0 when X straddles 0).
__device__ __forceinline__ iv ipow(iv x, int p) {
  if (p == 1) return x;
  if (p & 1) return {chain(x.lo, fabs(x.lo), p), chain(x.nhi, fabs(x.nhi), p)};
  double al = fabs(x.lo), ah = fabs(x.nhi);
  double m = fmax(al, ah);
  double mn = (x.lo >= 0.0 || x.nhi >= 0.0) ? fmin(al, ah) : 0.0;
  return {chain(mn, mn, p), chain(-m, m, p)};
}

// Midpoint (eq 2.5): R(R(a + b) * 0.5), which lies in [a, b].
__device__ __forceinline__ double imid(iv x) { return rmul(rsub(x.lo, x.nhi), 0.5); }

// Width rounded up: -R(a - b).
__device__ __forceinline__ double iwidth(iv x) { return -radd(x.lo, x.nhi); }

}  // namespace ibb
