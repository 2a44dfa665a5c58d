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
  return {dmin(dmin(l1, l2), dmin(l3, l4)), dmin(dmin(u1, u2), dmin(u3, u4))};
}

// Point times interval (the four products reduce to two by the sign of y).
__device__ __forceinline__ iv pmul(double y, iv x) {
  bool pos = !(y < 0.0);
  double a = pos ? x.lo : x.nhi;
  double b = pos ? x.nhi : x.lo;
  return {rmul_abs(y, a), rmul_abs(y, b)};
}

// Power X^p, p >= 1, each bound a left-to-right chain t <- R(t u) of p-1
// products.  Odd powers are monotone: each endpoint e maps to the chain
// e * |e| * ... (p = 1 is the empty chain).  Even powers are taken over |X|:
// [mn^p, m^p] with m = max |endpoint| and mn = min |endpoint| (0 when X
// straddles 0).  The two cases differ only in the chains' starting values,
// so lanes with different exponents do not branch.
__device__ __forceinline__ iv ipow(iv x, int p) {
  const double al = fabs(x.lo), ah = fabs(x.nhi);
  const bool odd = (p & 1) != 0;
  const double m = dmax(al, ah);
  const double mn = (x.lo >= 0.0 || x.nhi >= 0.0) ? dmin(al, ah) : 0.0;
  double a = odd ? x.lo : mn, b = odd ? x.nhi : -m;
  const double ua = odd ? al : mn, ub = odd ? ah : m;
  for (int i = 1; i < p; ++i) {
    a = rmul(a, ua);
    b = rmul(b, ub);
  }
  return {a, b};
}

// Midpoint (eq 2.5): R(R(a + b) * 0.5), which lies in [a, b].
__device__ __forceinline__ double imid(iv x) { return rmul(rsub(x.lo, x.nhi), 0.5); }

// Width rounded up: -R(a - b).
__device__ __forceinline__ double iwidth(iv x) { return -radd(x.lo, x.nhi); }

}  // namespace ibb
