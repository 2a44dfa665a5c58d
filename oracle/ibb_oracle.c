/*
 * ibb_oracle.c -- plain, slow CPU oracle for interval branch-and-bound with the
 * Hansen-Sengupta contraction (Lin & Chen, arXiv 1802.00330).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It shares no code with the GPU library.
 *
 * Every floating-point operation that the method rounds is written as ONE C
 * operation executed after an explicit fesetround() to the direction it needs
 * (round-down for lower bounds, round-up for upper bounds, nearest for the
 * single-precision preconditioner).  Compile with
 *     gcc -O2 -frounding-math -ffp-contract=off -fno-fast-math
 * so that no operation is contracted, folded or moved across a mode switch.
 *
 * Pinned by the CPU tests: primitives against exact rationals, the evaluator
 * against closed forms and exact point values, the preconditioner against exact
 * inverses, the contraction against linear systems with known solutions, the
 * solver against planted, closed-form and brute-force roots.
 *
 * Paper sections followed (see each function):
 *   Sec. 2.2 eq (3)-(10)   interval set, midpoint, + - x /, extended division
 *   Sec. 3.2 eq (25)-(27)  outward (directed) rounding of + - x
 *   Sec. 2.2 Def. 1-2      interval evaluation, the feasibility (exclusion) test
 *   Sec. 2.3 eq (13)-(22)  preconditioned Hansen-Sengupta Gauss-Seidel step
 *   Alg. 3, Alg. 4         HS on one box; interval matrix products
 *   Alg. 1, Alg. 2         branch-and-bound driver, bisection
 */
#include <fenv.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_N 16

/* status codes (same numbering as the public API's) */
#define OR_OK 0
#define OR_ERR_INVALID_ARG (-1)
#define OR_ERR_BUDGET (-2)
#define OR_ERR_OUTPUT_CAPACITY (-3)
#define OR_ERR_NO_MEMORY (-5)
#define OR_ERR_UNSUPPORTED (-7)

#define OR_SPLIT_WIDEST 0
#define OR_SPLIT_ALL 1

/* Every exported entry point leaves the caller's rounding mode as it found
 * it: the interval operations below switch the mode per bound, and a caller
 * (for example an interpreter evaluating its own floating-point expressions
 * afterwards) must not inherit a directed mode. */
static void restore_mode(const int* m) { fesetround(*m); }
#define KEEP_CALLER_MODE const int keep_mode_ __attribute__((cleanup(restore_mode))) = fegetround()

/* ------------------------------------------------------------------------- */
/* Directed rounding of a single operation: eq (25)-(27).                      */
/* The operands are read, the mode is set, the operation is performed and the  */
/* result stored through volatile objects, so the operation cannot be moved    */
/* outside the window in which the mode is in force.                           */
/* ------------------------------------------------------------------------- */
#define ROUNDED_OP(name, mode, expr)                                  \
  double name(double a, double b) {                                   \
    volatile double x = a, y = b;                                     \
    volatile double r;                                                \
    const int caller = fegetround();                                  \
    fesetround(mode);                                                 \
    r = expr;                                                         \
    fesetround(caller);                                               \
    return r;                                                         \
  }

ROUNDED_OP(oracle_rd_add, FE_DOWNWARD, x + y)
ROUNDED_OP(oracle_ru_add, FE_UPWARD, x + y)
ROUNDED_OP(oracle_rd_sub, FE_DOWNWARD, x - y)
ROUNDED_OP(oracle_ru_sub, FE_UPWARD, x - y)
ROUNDED_OP(oracle_rd_mul, FE_DOWNWARD, x * y)
ROUNDED_OP(oracle_ru_mul, FE_UPWARD, x * y)
ROUNDED_OP(oracle_rd_div, FE_DOWNWARD, x / y)
ROUNDED_OP(oracle_ru_div, FE_UPWARD, x / y)

#define rd_add oracle_rd_add
#define ru_add oracle_ru_add
#define rd_sub oracle_rd_sub
#define ru_sub oracle_ru_sub
#define rd_mul oracle_rd_mul
#define ru_mul oracle_ru_mul
#define rd_div oracle_rd_div
#define ru_div oracle_ru_div

static double min2(double a, double b) { return b < a ? b : a; }
static double max2(double a, double b) { return b > a ? b : a; }
static double min4(double a, double b, double c, double d) { return min2(min2(a, b), min2(c, d)); }
static double max4(double a, double b, double c, double d) { return max2(max2(a, b), max2(c, d)); }

/* An interval [lo, hi] with lo <= hi: eq (3). */
typedef struct {
  double lo, hi;
} ival;

static ival iv(double lo, double hi) {
  ival r = {lo, hi};
  return r;
}

/* Each interval operation below computes its lower bound with the rounding
 * mode set downward and its upper bound with the mode set upward; operands
 * and results pass through volatile objects so that no operation leaves the
 * window of the mode it was written for. */

/* eq (25): [a,b] + [c,d] = [rd(a+c), ru(b+d)] */
static ival i_add(ival x, ival y) {
  volatile double a = x.lo, b = x.hi, c = y.lo, d = y.hi;
  volatile double lo, hi;
  fesetround(FE_DOWNWARD);
  lo = a + c;
  fesetround(FE_UPWARD);
  hi = b + d;
  return iv(lo, hi);
}

/* eq (26): [a,b] - [c,d] = [rd(a-d), ru(b-c)] */
static ival i_sub(ival x, ival y) {
  volatile double a = x.lo, b = x.hi, c = y.lo, d = y.hi;
  volatile double lo, hi;
  fesetround(FE_DOWNWARD);
  lo = a - d;
  fesetround(FE_UPWARD);
  hi = b - c;
  return iv(lo, hi);
}

/* eq (27): lower bound = smallest of the four round-down products,
 * upper bound = largest of the four round-up products. */
static ival i_mul(ival x, ival y) {
  volatile double a = x.lo, b = x.hi, c = y.lo, d = y.hi;
  volatile double p1, p2, p3, p4, q1, q2, q3, q4;
  fesetround(FE_DOWNWARD);
  p1 = a * c;
  p2 = a * d;
  p3 = b * c;
  p4 = b * d;
  fesetround(FE_UPWARD);
  q1 = a * c;
  q2 = a * d;
  q3 = b * c;
  q4 = b * d;
  return iv(min4(p1, p2, p3, p4), max4(q1, q2, q3, q4));
}

void oracle_i_mul(double a, double b, double c, double d, double* out) {
  KEEP_CALLER_MODE;
  ival r = i_mul(iv(a, b), iv(c, d));
  out[0] = r.lo;
  out[1] = r.hi;
}

/* v^p for v >= 0 bounded from below / above by p-1 successive directed
 * products t <- t*v, evaluated left to right. */
static double pow_down_nonneg(double v, int p) {
  double t = v;
  for (int i = 1; i < p; ++i) t = rd_mul(t, v);
  return t;
}
static double pow_up_nonneg(double v, int p) {
  double t = v;
  for (int i = 1; i < p; ++i) t = ru_mul(t, v);
  return t;
}
/* Signed versions for odd p: v^p = -(-v)^p when v < 0. */
static double pow_down(double v, int p) { return v >= 0 ? pow_down_nonneg(v, p) : -pow_up_nonneg(-v, p); }
static double pow_up(double v, int p) { return v >= 0 ? pow_up_nonneg(v, p) : -pow_down_nonneg(-v, p); }

/* Power X^p of an interval (p >= 1).  Odd powers are monotone; even powers are
 * evaluated on |X| so that [-1,2]^2 = [0,4] rather than the product [-2,4]. */
static ival i_pow(ival x, int p) {
  if (p == 1) return x;
  if (p % 2 == 1) return iv(pow_down(x.lo, p), pow_up(x.hi, p));
  if (x.lo >= 0) return iv(pow_down_nonneg(x.lo, p), pow_up_nonneg(x.hi, p));
  if (x.hi <= 0) return iv(pow_down_nonneg(-x.hi, p), pow_up_nonneg(-x.lo, p));
  return iv(0.0, pow_up_nonneg(max2(-x.lo, x.hi), p));
}

void oracle_i_pow(double a, double b, int p, double* out) {
  KEEP_CALLER_MODE;
  ival r = i_pow(iv(a, b), p);
  out[0] = r.lo;
  out[1] = r.hi;
}

/* Midpoint, eq (2.5): (a+b)/2, both operations rounded down.  Lies in [a,b]. */
static double i_mid(ival x) { return rd_mul(rd_add(x.lo, x.hi), 0.5); }

/* Width of a coordinate, rounded up: hi - lo. */
static double i_width(ival x) { return ru_sub(x.hi, x.lo); }

/* Extended division x / y, eq (10), with the case conditions read as strict
 * sign conditions and the degenerate divisor [0,0] added:
 *   0 not in y          -> ordinary quotient (four directed quotients);
 *   0 in x, 0 in y      -> the whole line;
 *   y = [0,0], 0 not in x -> empty;
 *   x < 0:  y=[0,d]: (-inf, b/d];  y=[c,0]: [b/c, +inf);  c<0<d: both pieces
 *   x > 0:  y=[0,d]: [a/d, +inf);  y=[c,0]: (-inf, a/c];  c<0<d: both pieces
 * Returns the number of pieces (0, 1 or 2) written to out[0..1]. */
static int i_div_ext(ival x, ival y, ival out[2]) {
  double a = x.lo, b = x.hi, c = y.lo, d = y.hi;
  if (c > 0 || d < 0) {
    double lo = min4(rd_div(a, c), rd_div(a, d), rd_div(b, c), rd_div(b, d));
    double hi = max4(ru_div(a, c), ru_div(a, d), ru_div(b, c), ru_div(b, d));
    out[0] = iv(lo, hi);
    return 1;
  }
  if (a <= 0 && b >= 0) {
    out[0] = iv(-INFINITY, INFINITY);
    return 1;
  }
  if (c == 0 && d == 0) return 0;
  if (b < 0) {
    if (c == 0) { out[0] = iv(-INFINITY, ru_div(b, d)); return 1; }
    if (d == 0) { out[0] = iv(rd_div(b, c), INFINITY); return 1; }
    out[0] = iv(-INFINITY, ru_div(b, d));
    out[1] = iv(rd_div(b, c), INFINITY);
    return 2;
  }
  /* a > 0 */
  if (c == 0) { out[0] = iv(rd_div(a, d), INFINITY); return 1; }
  if (d == 0) { out[0] = iv(-INFINITY, ru_div(a, c)); return 1; }
  out[0] = iv(-INFINITY, ru_div(a, c));
  out[1] = iv(rd_div(a, d), INFINITY);
  return 2;
}

int oracle_i_div_ext(double a, double b, double c, double d, double* out) {
  KEEP_CALLER_MODE;
  ival p[2];
  int k = i_div_ext(iv(a, b), iv(c, d), p);
  for (int i = 0; i < k; ++i) {
    out[2 * i] = p[i].lo;
    out[2 * i + 1] = p[i].hi;
  }
  return k;
}

/* ------------------------------------------------------------------------- */
/* The polynomial system: sparse monomials, Sec. 2.1.                          */
/* ------------------------------------------------------------------------- */
typedef struct {
  int n;
  const int32_t* term_off; /* [n+1] */
  const uint8_t* expo;     /* [T*n] */
  const double* coef;      /* [T]   */
} osys;

/* Interval value of the monomial  coefficient * prod_k X_k^e_k  (Def. 1):
 * the factors are multiplied for k ascending, the coefficient last. */
static ival monomial(ival coefficient, const int* e, int n, const ival* X) {
  int have = 0;
  ival t = iv(0, 0);
  for (int k = 0; k < n; ++k) {
    if (e[k] == 0) continue;
    ival f = i_pow(X[k], e[k]);
    t = have ? i_mul(t, f) : f;
    have = 1;
  }
  if (!have) return coefficient;
  return i_mul(coefficient, t);
}

/* F_i(X): the terms of equation i summed in stored order (Def. 1). */
static ival eval_f(const osys* s, int i, const ival* X) {
  int e[OR_MAX_N];
  ival sum = iv(0, 0);
  for (int t = s->term_off[i]; t < s->term_off[i + 1]; ++t) {
    for (int k = 0; k < s->n; ++k) e[k] = s->expo[(size_t)t * s->n + k];
    ival v = monomial(iv(s->coef[t], s->coef[t]), e, s->n, X);
    sum = (t == s->term_off[i]) ? v : i_add(sum, v);
  }
  return sum;
}

/* J_ik(X) = d f_i / d x_k over X (Alg. 3, first step).  For each term of
 * equation i with e_k >= 1, in stored order: the coefficient e_k * c enclosed
 * as [rd(e_k c), ru(e_k c)], times the monomial with e_k lowered by one.
 * [0,0] when no term of f_i depends on x_k. */
static ival eval_df(const osys* s, int i, int k, const ival* X) {
  int e[OR_MAX_N];
  int have = 0;
  ival sum = iv(0, 0);
  for (int t = s->term_off[i]; t < s->term_off[i + 1]; ++t) {
    int ek = s->expo[(size_t)t * s->n + k];
    if (ek == 0) continue;
    for (int m = 0; m < s->n; ++m) e[m] = s->expo[(size_t)t * s->n + m];
    e[k] = ek - 1;
    double c = s->coef[t];
    ival cf = iv(rd_mul((double)ek, c), ru_mul((double)ek, c));
    ival v = monomial(cf, e, s->n, X);
    sum = have ? i_add(sum, v) : v;
    have = 1;
  }
  return sum;
}

static osys make_sys(int n, const int32_t* term_off, const uint8_t* expo, const double* coef) {
  osys s = {n, term_off, expo, coef};
  return s;
}

void oracle_eval_F(int n, const int32_t* term_off, const uint8_t* expo, const double* coef,
                   const double* lo, const double* hi, double* out_lo, double* out_hi) {
  KEEP_CALLER_MODE;
  osys s = make_sys(n, term_off, expo, coef);
  ival X[OR_MAX_N];
  for (int k = 0; k < n; ++k) X[k] = iv(lo[k], hi[k]);
  for (int i = 0; i < n; ++i) {
    ival f = eval_f(&s, i, X);
    out_lo[i] = f.lo;
    out_hi[i] = f.hi;
  }
}

void oracle_eval_J(int n, const int32_t* term_off, const uint8_t* expo, const double* coef,
                   const double* lo, const double* hi, double* out_lo, double* out_hi) {
  KEEP_CALLER_MODE;
  osys s = make_sys(n, term_off, expo, coef);
  ival X[OR_MAX_N];
  for (int k = 0; k < n; ++k) X[k] = iv(lo[k], hi[k]);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      ival v = eval_df(&s, i, k, X);
      out_lo[i * n + k] = v.lo;
      out_hi[i * n + k] = v.hi;
    }
}

/* ------------------------------------------------------------------------- */
/* Approximate inverse of mid J(X) in single precision (Sec. 2.3: "B", an      */
/* approximate inverse of J_c; Alg. 3 second step).  LU with partial pivoting, */
/* then one forward and one back substitution per column of the identity.     */
/* All single-precision operations round to nearest; no fused multiply-add.    */
/* Returns 0 and Y on success, 1 if the inverse is unusable (a zero pivot or   */
/* any non-finite value), in which case the contraction is skipped.            */
/* ------------------------------------------------------------------------- */
int oracle_fp32_inverse(int n, const float* Min, float* Y) {
  KEEP_CALLER_MODE;
  float M[OR_MAX_N][OR_MAX_N];
  int perm[OR_MAX_N];
  fesetround(FE_TONEAREST);
  for (int i = 0; i < n; ++i) {
    perm[i] = i;
    for (int j = 0; j < n; ++j) {
      M[i][j] = Min[i * n + j];
      if (!isfinite(M[i][j])) return 1;
    }
  }
  for (int k = 0; k < n; ++k) {
    /* pivot: the first row, from k down, of largest magnitude in column k */
    int p = k;
    float best = fabsf(M[k][k]);
    for (int i = k + 1; i < n; ++i)
      if (fabsf(M[i][k]) > best) {
        best = fabsf(M[i][k]);
        p = i;
      }
    if (M[p][k] == 0.0f) return 1;
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        float t = M[k][j];
        M[k][j] = M[p][j];
        M[p][j] = t;
      }
      int t = perm[k];
      perm[k] = perm[p];
      perm[p] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      float l = M[i][k] / M[k][k];
      M[i][k] = l;
      for (int j = k + 1; j < n; ++j) {
        float prod = l * M[k][j];
        M[i][j] = M[i][j] - prod;
      }
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (!isfinite(M[i][j])) return 1;
  for (int c = 0; c < n; ++c) {
    float z[OR_MAX_N], x[OR_MAX_N];
    /* L z = P e_c, j ascending */
    for (int i = 0; i < n; ++i) {
      float t = (perm[i] == c) ? 1.0f : 0.0f;
      for (int j = 0; j < i; ++j) {
        float prod = M[i][j] * z[j];
        t = t - prod;
      }
      z[i] = t;
    }
    /* U x = z, i descending; the subtractions for j descending from n-1 */
    for (int i = n - 1; i >= 0; --i) {
      float t = z[i];
      for (int j = n - 1; j > i; --j) {
        float prod = M[i][j] * x[j];
        t = t - prod;
      }
      x[i] = t / M[i][i];
    }
    for (int i = 0; i < n; ++i) {
      if (!isfinite(x[i])) return 1;
      Y[i * n + c] = x[i];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Hansen-Sengupta step on one box: eq (13)-(22), Alg. 3, Alg. 4.              */
/* ------------------------------------------------------------------------- */
/* Optional trace of one contraction step (same layout as the device
 * diagnostic dump), written when non-null.  Test infrastructure only. */
static double* g_trace = NULL;
static int tr_J(int n) { (void)n; return 0; }
static int tr_F(int n) { return 2 * n * n; }
static int tr_M(int n) { return 2 * n * n + 2 * n; }
static int tr_Y(int n) { return 3 * n * n + 2 * n; }
static int tr_g(int n) { return 4 * n * n + 2 * n; }
static int tr_P(int n) { return 4 * n * n + 4 * n; }
static int tr_N(int n) { return 6 * n * n + 4 * n; }
static int tr_X(int n) { return 6 * n * n + 6 * n; }
static int tr_flags(int n) { return 6 * n * n + 8 * n; }

#define HS_EMPTY 0   /* the box holds no root */
#define HS_SKIPPED 1 /* preconditioner unusable: box unchanged, nothing proven */
#define HS_DONE 2    /* contracted box X' (possibly equal to X) */

/* Y (a point, exactly representable) times an interval. */
static ival pmul(double y, ival x) { return i_mul(iv(y, y), x); }

#define OR_CONTRACT_HS 0
#define OR_CONTRACT_KRAWCZYK 1

static int hs_step(const osys* s, const ival* X, ival* Xn, int* unique, int contractor) {
  const int n = s->n;
  double xc[OR_MAX_N];
  ival Xc[OR_MAX_N], Fc[OR_MAX_N], D[OR_MAX_N];
  ival J[OR_MAX_N][OR_MAX_N], P[OR_MAX_N][OR_MAX_N], g[OR_MAX_N];
  float Mf[OR_MAX_N * OR_MAX_N], Yf[OR_MAX_N * OR_MAX_N];

  /* expansion point x = mid X, eq (2.5) */
  for (int k = 0; k < n; ++k) {
    xc[k] = i_mid(X[k]);
    Xc[k] = iv(xc[k], xc[k]);
  }
  /* J(X) and F(x) over the degenerate box [x, x] */
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) J[i][k] = eval_df(s, i, k, X);
  for (int i = 0; i < n; ++i) Fc[i] = eval_f(s, i, Xc);
  if (g_trace) {
    for (int i = 0; i < n; ++i) {
      for (int k = 0; k < n; ++k) {
        g_trace[tr_J(n) + (i * n + k) * 2] = J[i][k].lo;
        g_trace[tr_J(n) + (i * n + k) * 2 + 1] = J[i][k].hi;
      }
      g_trace[tr_F(n) + 2 * i] = Fc[i].lo;
      g_trace[tr_F(n) + 2 * i + 1] = Fc[i].hi;
    }
  }

  /* B ~ inverse of mid J(X), single precision (narrowing rounds to nearest) */
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double m = i_mid(J[i][k]);
      fesetround(FE_TONEAREST);
      Mf[i * n + k] = (float)m;
    }
  if (g_trace)
    for (int i = 0; i < n * n; ++i) g_trace[tr_M(n) + i] = (double)Mf[i];
  if (oracle_fp32_inverse(n, Mf, Yf) != 0) {
    if (g_trace) g_trace[tr_flags(n)] = 1.0;
    return HS_SKIPPED;
  }
  if (g_trace)
    for (int i = 0; i < n * n; ++i) g_trace[tr_Y(n) + i] = (double)Yf[i];

  /* g = B F(x) and P = B J(X) by interval matrix products (Alg. 4): the sum
   * over k ascending, starting from the first term.  Terms whose point or
   * interval factor is exactly zero contribute exactly zero and are omitted. */
  for (int i = 0; i < n; ++i) {
    int have = 0;
    ival acc = iv(0, 0);
    for (int k = 0; k < n; ++k) {
      double y = (double)Yf[i * n + k];
      if (y == 0 || (Fc[k].lo == 0 && Fc[k].hi == 0)) continue;
      ival t = pmul(y, Fc[k]);
      acc = have ? i_add(acc, t) : t;
      have = 1;
    }
    g[i] = acc;
    for (int j = 0; j < n; ++j) {
      have = 0;
      acc = iv(0, 0);
      for (int k = 0; k < n; ++k) {
        double y = (double)Yf[i * n + k];
        if (y == 0 || (J[k][j].lo == 0 && J[k][j].hi == 0)) continue;
        ival t = pmul(y, J[k][j]);
        acc = have ? i_add(acc, t) : t;
        have = 1;
      }
      P[i][j] = acc;
    }
  }

  if (g_trace)
    for (int i = 0; i < n; ++i) {
      g_trace[tr_g(n) + 2 * i] = g[i].lo;
      g_trace[tr_g(n) + 2 * i + 1] = g[i].hi;
      for (int j = 0; j < n; ++j) {
        g_trace[tr_P(n) + (i * n + j) * 2] = P[i][j].lo;
        g_trace[tr_P(n) + (i * n + j) * 2 + 1] = P[i][j].hi;
      }
    }
  /* X - x, eq (19) */
  for (int k = 0; k < n; ++k) D[k] = i_sub(X[k], Xc[k]);

  if (contractor == OR_CONTRACT_KRAWCZYK) {
    /* Krawczyk operator, eq (15): K(X) = x - B f(x) + [I - B J(X)](X - x), with
     * B f(x) = g and B J(X) = P as above; every component uses X (no update as
     * the components are obtained).  The sum over j ascending starts from its
     * first term; K_i = (x_i - g_i) + sum.  Eq (16): X' = X meets K(X); an
     * empty meet means no root; K(X) inside the interior of X proves one. */
    int uniq = 1;
    for (int i = 0; i < n; ++i) {
      ival sum = iv(0, 0);
      for (int j = 0; j < n; ++j) {
        ival m = (j == i) ? i_sub(iv(1.0, 1.0), P[i][j]) : iv(-P[i][j].hi, -P[i][j].lo);
        ival t = i_mul(m, D[j]);
        sum = j ? i_add(sum, t) : t;
      }
      ival K = i_add(i_sub(Xc[i], g[i]), sum);
      if (g_trace) {
        g_trace[tr_N(n) + 2 * i] = K.lo;
        g_trace[tr_N(n) + 2 * i + 1] = K.hi;
      }
      double a = max2(K.lo, X[i].lo), b = min2(K.hi, X[i].hi);
      if (a > b) {
        if (g_trace) g_trace[tr_flags(n) + 1] = 1.0;
        return HS_EMPTY;
      }
      uniq = uniq && X[i].lo < K.lo && K.hi < X[i].hi;
      Xn[i] = iv(a, b);
      if (g_trace) {
        g_trace[tr_X(n) + 2 * i] = a;
        g_trace[tr_X(n) + 2 * i + 1] = b;
      }
    }
    *unique = uniq;
    if (g_trace) {
      g_trace[tr_flags(n) + 2] = uniq ? 1.0 : 0.0;
      g_trace[tr_flags(n) + 3] = 1.0;
    }
    return HS_DONE;
  }

  /* Gauss-Seidel sweep, eq (21)-(22):
   *   Y_i = x_i - (P_ii)^{-1} [ g_i + sum_{j<i} P_ij (X'_j - x_j) + sum_{j>i} P_ij (X_j - x_j) ]
   * The bracket is evaluated as written: the two sums are formed separately
   * (each over j ascending, from its first term) and then added to g_i left
   * to right; an empty sum is omitted. */
  int uniq = 1;
  ival Dn[OR_MAX_N];
  for (int i = 0; i < n; ++i) {
    ival N = g[i];
    int have = 0;
    ival lower = iv(0, 0);
    for (int j = 0; j < i; ++j) {
      ival t = i_mul(P[i][j], Dn[j]);
      lower = have ? i_add(lower, t) : t;
      have = 1;
    }
    if (have) N = i_add(N, lower);
    have = 0;
    ival upper = iv(0, 0);
    for (int j = i + 1; j < n; ++j) {
      ival t = i_mul(P[i][j], D[j]);
      upper = have ? i_add(upper, t) : t;
      have = 1;
    }
    if (have) N = i_add(N, upper);

    if (g_trace) {
      g_trace[tr_N(n) + 2 * i] = N.lo;
      g_trace[tr_N(n) + 2 * i + 1] = N.hi;
    }
    ival Q[2];
    int nq = i_div_ext(N, P[i][i], Q);
    /* Y_i = x_i - Q, piece by piece; X'_i = hull of (piece intersect X_i) */
    int any = 0;
    double nlo = 0, nhi = 0;
    int inside = (nq == 1 && isfinite(Q[0].lo) && isfinite(Q[0].hi));
    for (int q = 0; q < nq; ++q) {
      ival Yi = i_sub(Xc[i], Q[q]);
      double ylo = Yi.lo, yhi = Yi.hi;
      if (nq == 1) inside = inside && (X[i].lo < ylo) && (yhi < X[i].hi);
      double a = max2(ylo, X[i].lo), b = min2(yhi, X[i].hi);
      if (a > b) continue;
      if (!any) {
        nlo = a;
        nhi = b;
        any = 1;
      } else {
        nlo = min2(nlo, a);
        nhi = max2(nhi, b);
      }
    }
    if (!any) {
      if (g_trace) g_trace[tr_flags(n) + 1] = 1.0;
      return HS_EMPTY;
    }
    uniq = uniq && inside;
    Xn[i] = iv(nlo, nhi);
    if (g_trace) {
      g_trace[tr_X(n) + 2 * i] = nlo;
      g_trace[tr_X(n) + 2 * i + 1] = nhi;
    }
    Dn[i] = i_sub(Xn[i], Xc[i]);
  }
  *unique = uniq;
  if (g_trace) {
    g_trace[tr_flags(n) + 2] = uniq ? 1.0 : 0.0;
    g_trace[tr_flags(n) + 3] = 1.0;
  }
  return HS_DONE;
}

/* The exclusion test (Def. 2) on m boxes (row-major [m][n] bounds): keep[b] = 1
 * when every F_i holds 0 over box b, else 0.  Used to count the boxes kept by
 * the rounds of the paper's worked examples. */
void oracle_exclusion_keep(int n, const int32_t* term_off, const uint8_t* expo, const double* coef, int64_t m,
                           const double* lo, const double* hi, uint8_t* keep) {
  KEEP_CALLER_MODE;
  osys s = make_sys(n, term_off, expo, coef);
  for (int64_t b = 0; b < m; ++b) {
    ival X[OR_MAX_N];
    for (int k = 0; k < n; ++k) X[k] = iv(lo[b * n + k], hi[b * n + k]);
    int kept = 1;
    for (int i = 0; i < n && kept; ++i) {
      ival f = eval_f(&s, i, X);
      if (f.lo > 0 || f.hi < 0) kept = 0;
    }
    keep[b] = (uint8_t)kept;
  }
}

/* One contraction step with its intermediates written to `trace`
 * (6n^2 + 8n + 4 doubles, layout of tr_* above). */
int oracle_hs_trace(int n, const int32_t* term_off, const uint8_t* expo, const double* coef,
                    const double* lo, const double* hi, double* trace, int contractor) {
  KEEP_CALLER_MODE;
  osys s = make_sys(n, term_off, expo, coef);
  ival X[OR_MAX_N], Xn[OR_MAX_N];
  for (int k = 0; k < n; ++k) X[k] = iv(lo[k], hi[k]);
  memset(trace, 0, sizeof(double) * (size_t)(6 * n * n + 8 * n + 4));
  int u = 0;
  g_trace = trace;
  int st = hs_step(&s, X, Xn, &u, contractor);
  g_trace = NULL;
  return st;
}

int oracle_hs(int n, const int32_t* term_off, const uint8_t* expo, const double* coef,
              const double* lo, const double* hi, double* out_lo, double* out_hi, int* unique, int contractor) {
  KEEP_CALLER_MODE;
  osys s = make_sys(n, term_off, expo, coef);
  ival X[OR_MAX_N], Xn[OR_MAX_N];
  for (int k = 0; k < n; ++k) X[k] = iv(lo[k], hi[k]);
  int u = 0;
  int st = hs_step(&s, X, Xn, &u, contractor);
  if (st == HS_DONE)
    for (int k = 0; k < n; ++k) {
      out_lo[k] = Xn[k].lo;
      out_hi[k] = Xn[k].hi;
    }
  *unique = u;
  return st;
}

/* ------------------------------------------------------------------------- */
/* Branch and bound driver: Alg. 1 and Alg. 2.                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
  double tol;
  int64_t max_boxes;
  int32_t split_mode;
  int32_t max_recontract;
  double recontract_ratio;
  double hs_max_width;
  int32_t contractor; /* OR_CONTRACT_HS or OR_CONTRACT_KRAWCZYK */
  int32_t inclusion;  /* 0 natural extension; 1 also the mean-value form */
} oparams;

typedef struct {
  int64_t processed, excluded_eval, excluded_hs, hs_skipped, recontracted, bisected,
      emitted_unique, emitted_undecided;
} ostats;

typedef struct {
  ival X[OR_MAX_N];
  int proven;
  int rc;
} obox;

typedef struct {
  obox* a;
  size_t len, cap, head; /* head: FIFO read position */
} ostack;

static int push(ostack* st, const obox* b) {
  if (st->len == st->cap) {
    size_t nc = st->cap ? 2 * st->cap : 256;
    obox* na = (obox*)realloc(st->a, nc * sizeof(obox));
    if (!na) return -1;
    st->a = na;
    st->cap = nc;
  }
  st->a[st->len++] = *b;
  return 0;
}

typedef struct {
  ival X[OR_MAX_N];
  uint8_t tag;
} oemit;

typedef struct {
  oemit* a;
  size_t len, cap;
} olist;

static int emit(olist* l, const ival* X, int n, int tag) {
  if (l->len == l->cap) {
    size_t nc = l->cap ? 2 * l->cap : 64;
    oemit* na = (oemit*)realloc(l->a, nc * sizeof(oemit));
    if (!na) return -1;
    l->a = na;
    l->cap = nc;
  }
  oemit* e = &l->a[l->len++];
  memset(e, 0, sizeof(*e));
  for (int k = 0; k < n; ++k) e->X[k] = X[k];
  e->tag = (uint8_t)tag;
  return 0;
}

static double box_width(const ival* X, int n) {
  double w = 0;
  for (int k = 0; k < n; ++k) w = max2(w, i_width(X[k]));
  return w;
}

static int g_sort_n; /* dimension used by the qsort comparator */

static int cmp_emit(const void* pa, const void* pb) {
  const oemit* a = (const oemit*)pa;
  const oemit* b = (const oemit*)pb;
  for (int k = 0; k < g_sort_n; ++k) {
    if (a->X[k].lo < b->X[k].lo) return -1;
    if (a->X[k].lo > b->X[k].lo) return 1;
  }
  for (int k = 0; k < g_sort_n; ++k) {
    if (a->X[k].hi < b->X[k].hi) return -1;
    if (a->X[k].hi > b->X[k].hi) return 1;
  }
  return (int)a->tag - (int)b->tag;
}

static double canon_zero(double v) { return v == 0 ? 0.0 : v; }

/* splitmix64, only for the randomised processing order used by the
 * order-independence test */
static uint64_t mix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static int valid_input(int n, const int32_t* term_off, const uint8_t* expo, const double* coef,
                       const double* lo, const double* hi, const oparams* p) {
  if (n < 1 || n > OR_MAX_N) return 0;
  if (term_off[0] != 0) return 0;
  for (int i = 0; i < n; ++i)
    if (term_off[i + 1] <= term_off[i]) return 0;
  const double big = 0x1p40;
  for (int t = 0; t < term_off[n]; ++t) {
    if (!isfinite(coef[t]) || fabs(coef[t]) > big) return 0;
    int deg = 0;
    for (int k = 0; k < n; ++k) deg += expo[(size_t)t * n + k];
    if (deg > 8) return 0;
  }
  for (int k = 0; k < n; ++k)
    if (!isfinite(lo[k]) || !isfinite(hi[k]) || lo[k] > hi[k] || fabs(lo[k]) > big || fabs(hi[k]) > big)
      return 0;
  if (!(p->tol > 0) || !isfinite(p->tol)) return 0;
  if (p->max_boxes < 1) return 0;
  if (p->split_mode != OR_SPLIT_WIDEST && p->split_mode != OR_SPLIT_ALL) return 0;
  if (p->max_recontract < 1) return 0;
  if (!(p->recontract_ratio >= 0) || !(p->recontract_ratio <= 1)) return 0;
  if (isnan(p->hs_max_width)) return 0;
  if (p->contractor != OR_CONTRACT_HS && p->contractor != OR_CONTRACT_KRAWCZYK) return 0;
  if (p->inclusion != 0 && p->inclusion != 1) return 0;
  return 1;
}

/* Optional record of the proof chains of a solve (test infrastructure): for
 * every stepped box that is proven or becomes proven, its box and the
 * contracted box, 4n doubles (lo, hi, lo', hi').  Set by oracle_set_chain. */
static double* g_chain = NULL;
static int64_t g_chain_cap = 0, g_chain_len = 0;

void oracle_set_chain(double* buf, int64_t cap) {
  g_chain = buf;
  g_chain_cap = cap;
  g_chain_len = 0;
}

int64_t oracle_chain_len(void) { return g_chain_len; }

static void chain_record(const ival* X, const ival* Xn, int n) {
  if (!g_chain || g_chain_len >= g_chain_cap) return;
  double* d = g_chain + (size_t)g_chain_len * 4 * n;
  for (int k = 0; k < n; ++k) {
    d[k] = X[k].lo;
    d[n + k] = X[k].hi;
    d[2 * n + k] = Xn[k].lo;
    d[3 * n + k] = Xn[k].hi;
  }
  g_chain_len++;
}

/* One box through steps S1-S7 of the search (Alg. 1 with the contraction of
 * Alg. 3 and the bisection of Alg. 2): counters in S, children pushed on st,
 * boxes of width <= tol appended to out. */
static int step_box(const osys* s, const oparams* p, const obox* b, ostack* st, olist* out, ostats* S) {
  const int n = s->n;
  /* Exclusion test (Def. 2): X holds no root if some F_i(X) excludes 0. */
  if (!b->proven) {
    int excluded = 0;
    for (int i = 0; i < n && !excluded; ++i) {
      ival f = eval_f(s, i, b->X);
      if (f.lo > 0 || f.hi < 0) excluded = 1;
    }
    if (excluded) {
      S->excluded_eval++;
      return OR_OK;
    }
    /* Mean-value form (a centred inclusion, Sec. 2.2): by the mean value
     * theorem f_i(X) lies in F_i(x) + sum_k J_ik(X) (X_k - x_k), x = mid X;
     * evaluated as written, the sum over k ascending added to F_i(x) term by
     * term.  The box holds no root if some component excludes 0. */
    if (p->inclusion == 1) {
      ival Xc[OR_MAX_N], D[OR_MAX_N];
      for (int k = 0; k < n; ++k) {
        double m = i_mid(b->X[k]);
        Xc[k] = iv(m, m);
        D[k] = i_sub(b->X[k], Xc[k]);
      }
      for (int i = 0; i < n && !excluded; ++i) {
        ival acc = eval_f(s, i, Xc);
        for (int k = 0; k < n; ++k) acc = i_add(acc, i_mul(eval_df(s, i, k, b->X), D[k]));
        if (acc.lo > 0 || acc.hi < 0) excluded = 1;
      }
      if (excluded) {
        S->excluded_eval++;
        return OR_OK;
      }
    }
  }

  /* Contraction (Alg. 3), unless the box is wider than hs_max_width. */
  double w = box_width(b->X, n);
  ival Xn[OR_MAX_N];
  int u = 0;
  int hs = HS_SKIPPED;
  if (!(w > p->hs_max_width)) hs = hs_step(s, b->X, Xn, &u, p->contractor);
  if (hs == HS_EMPTY) {
    S->excluded_hs++;
    return OR_OK;
  }
  if (hs == HS_SKIPPED) {
    S->hs_skipped++;
    for (int k = 0; k < n; ++k) Xn[k] = b->X[k];
    u = 0;
  }
  int proven = b->proven || u;
  if (proven) chain_record(b->X, Xn, n);
  double wn = box_width(Xn, n);

  if (wn <= p->tol) {
    if (emit(out, Xn, n, proven ? 1 : 0)) return OR_ERR_NO_MEMORY;
    if (proven) S->emitted_unique++; else S->emitted_undecided++;
    return OR_OK;
  }
  if (proven) {
    if (wn < w && b->rc + 1 < p->max_recontract) {
      obox c;
      memset(&c, 0, sizeof c);
      for (int k = 0; k < n; ++k) c.X[k] = Xn[k];
      c.proven = 1;
      c.rc = b->rc + 1;
      if (push(st, &c)) return OR_ERR_NO_MEMORY;
      S->recontracted++;
    } else {
      if (emit(out, Xn, n, 1)) return OR_ERR_NO_MEMORY;
      S->emitted_unique++;
    }
    return OR_OK;
  }
  if (wn <= rd_mul(p->recontract_ratio, w) && b->rc + 1 < p->max_recontract) {
    obox c;
    memset(&c, 0, sizeof c);
    for (int k = 0; k < n; ++k) c.X[k] = Xn[k];
    c.proven = 0;
    c.rc = b->rc + 1;
    if (push(st, &c)) return OR_ERR_NO_MEMORY;
    S->recontracted++;
    return OR_OK;
  }

  /* Bisection (Alg. 2 splits every coordinate at its midpoint; the default
   * mode splits only the widest coordinate, first index on ties). */
  if (p->split_mode == OR_SPLIT_WIDEST) {
    int kk = 0;
    double best = i_width(Xn[0]);
    for (int k = 1; k < n; ++k) {
      double wk = i_width(Xn[k]);
      if (wk > best) {
        best = wk;
        kk = k;
      }
    }
    double m = i_mid(Xn[kk]);
    if (!(m > Xn[kk].lo && m < Xn[kk].hi)) {
      if (emit(out, Xn, n, 0)) return OR_ERR_NO_MEMORY;
      S->emitted_undecided++;
      return OR_OK;
    }
    obox c;
    memset(&c, 0, sizeof c);
    for (int k = 0; k < n; ++k) c.X[k] = Xn[k];
    c.X[kk] = iv(Xn[kk].lo, m);
    if (push(st, &c)) return OR_ERR_NO_MEMORY;
    c.X[kk] = iv(m, Xn[kk].hi);
    if (push(st, &c)) return OR_ERR_NO_MEMORY;
    S->bisected++;
  } else {
    int split[OR_MAX_N], ns = 0;
    double mids[OR_MAX_N];
    for (int k = 0; k < n; ++k) {
      double m = i_mid(Xn[k]);
      if (m > Xn[k].lo && m < Xn[k].hi) {
        split[ns++] = k;
        mids[k] = m;
      }
    }
    if (ns == 0) {
      if (emit(out, Xn, n, 0)) return OR_ERR_NO_MEMORY;
      S->emitted_undecided++;
      return OR_OK;
    }
    for (uint32_t bits = 0; bits < (1u << ns); ++bits) {
      obox c;
      memset(&c, 0, sizeof c);
      for (int k = 0; k < n; ++k) c.X[k] = Xn[k];
      for (int q = 0; q < ns; ++q) {
        int k = split[q];
        c.X[k] = ((bits >> q) & 1) ? iv(mids[k], Xn[k].hi) : iv(Xn[k].lo, mids[k]);
      }
      if (push(st, &c)) return OR_ERR_NO_MEMORY;
    }
    S->bisected++;
  }
  return OR_OK;
}

/* Solve: returns a status; on success the sorted boxes and tags.
 * order: 0 = last in first out, 1 = first in first out, 2 = random (seeded).
 * stats_out: 8 int64 counters (see ostats). */
int oracle_solve(int n, const int32_t* term_off, const uint8_t* expo, const double* coef,
                 const double* lo, const double* hi, double tol, int64_t max_boxes,
                 int32_t split_mode, int32_t max_recontract, double recontract_ratio,
                 double hs_max_width, double* out_lo, double* out_hi, uint8_t* out_tag,
                 int64_t cap, int64_t* n_out, int64_t* stats_out, int order, uint64_t seed, int32_t contractor,
                 int32_t inclusion) {
  KEEP_CALLER_MODE;
  oparams p = {tol, max_boxes, split_mode, max_recontract, recontract_ratio, hs_max_width, contractor, inclusion};
  ostats S;
  memset(&S, 0, sizeof S);
  *n_out = 0;
  if (!valid_input(n, term_off, expo, coef, lo, hi, &p)) return OR_ERR_INVALID_ARG;
  osys s = make_sys(n, term_off, expo, coef);

  ostack st = {0};
  olist out = {0};
  obox root;
  memset(&root, 0, sizeof root);
  for (int k = 0; k < n; ++k) root.X[k] = iv(lo[k], hi[k]);
  if (push(&st, &root)) return OR_ERR_NO_MEMORY;

  int status = OR_OK;
  uint64_t rng = seed;
  while (st.len > st.head) {
    obox b;
    if (order == 1) {
      b = st.a[st.head++];
    } else if (order == 2) {
      size_t live = st.len - st.head;
      size_t j = st.head + (size_t)(mix64(&rng) % live);
      b = st.a[j];
      st.a[j] = st.a[st.len - 1];
      st.len--;
    } else {
      b = st.a[--st.len];
    }
    if (order == 1 && st.head > 4096 && st.head * 2 > st.len) { /* compact the FIFO */
      memmove(st.a, st.a + st.head, (st.len - st.head) * sizeof(obox));
      st.len -= st.head;
      st.head = 0;
    }

    S.processed++;
    if (S.processed > p.max_boxes) {
      status = OR_ERR_BUDGET;
      break;
    }

    status = step_box(&s, &p, &b, &st, &out, &S);
    if (status != OR_OK) break;
  }

  if (stats_out) {
    int64_t v[8] = {S.processed, S.excluded_eval, S.excluded_hs, S.hs_skipped, S.recontracted,
                    S.bisected, S.emitted_unique, S.emitted_undecided};
    memcpy(stats_out, v, sizeof v);
  }
  if (status == OR_OK) {
    for (size_t e = 0; e < out.len; ++e)
      for (int k = 0; k < n; ++k) {
        out.a[e].X[k].lo = canon_zero(out.a[e].X[k].lo);
        out.a[e].X[k].hi = canon_zero(out.a[e].X[k].hi);
      }
    g_sort_n = n;
    qsort(out.a, out.len, sizeof(oemit), cmp_emit);
    *n_out = (int64_t)out.len;
    if ((int64_t)out.len > cap) {
      status = OR_ERR_OUTPUT_CAPACITY;
    } else {
      for (size_t e = 0; e < out.len; ++e) {
        for (int k = 0; k < n; ++k) {
          out_lo[e * n + k] = out.a[e].X[k].lo;
          out_hi[e * n + k] = out.a[e].X[k].hi;
        }
        out_tag[e] = out.a[e].tag;
      }
    }
  }
  free(st.a);
  free(out.a);
  return status;
}

/* One round of the search on a caller-given list of boxes (the boxes of one
 * round set of Alg. 1, each through step_box): the children in the order they
 * are pushed, the boxes of width <= tol in the order they are emitted, neither
 * sorted nor made canonical.  rec per box: bit 0 proven, bits 8-15 the
 * recontraction count; the same record is written for each child.  No budget
 * applies.  n_child and n_emit receive the counts also when they exceed the
 * capacities (then OR_ERR_OUTPUT_CAPACITY is returned and nothing is copied). */
int oracle_round(int n, const int32_t* term_off, const uint8_t* expo, const double* coef, int64_t count,
                 const double* lo, const double* hi, const uint32_t* rec, double tol, int32_t split_mode,
                 int32_t max_recontract, double recontract_ratio, double hs_max_width, double* child_lo,
                 double* child_hi, uint32_t* child_rec, int64_t child_cap, int64_t* n_child, double* emit_lo,
                 double* emit_hi, uint8_t* emit_tag, int64_t emit_cap, int64_t* n_emit, int64_t* stats_out,
                 int32_t contractor, int32_t inclusion) {
  KEEP_CALLER_MODE;
  oparams p = {tol, 1, split_mode, max_recontract, recontract_ratio, hs_max_width, contractor, inclusion};
  ostats S;
  memset(&S, 0, sizeof S);
  *n_child = 0;
  *n_emit = 0;
  if (count < 0) return OR_ERR_INVALID_ARG;
  for (int64_t b = 0; b < count; ++b)
    if (!valid_input(n, term_off, expo, coef, lo + b * n, hi + b * n, &p)) return OR_ERR_INVALID_ARG;
  if (count == 0) {
    /* no box to check: validate the system and parameters on a zero box */
    double z[OR_MAX_N] = {0};
    if (!valid_input(n, term_off, expo, coef, z, z, &p)) return OR_ERR_INVALID_ARG;
  }
  osys s = make_sys(n, term_off, expo, coef);
  ostack st = {0};
  olist out = {0};
  int status = OR_OK;
  for (int64_t b = 0; b < count && status == OR_OK; ++b) {
    obox x;
    memset(&x, 0, sizeof x);
    for (int k = 0; k < n; ++k) x.X[k] = iv(lo[b * n + k], hi[b * n + k]);
    x.proven = (int)(rec[b] & 1u);
    x.rc = (int)((rec[b] >> 8) & 0xFFu);
    S.processed++;
    status = step_box(&s, &p, &x, &st, &out, &S);
  }
  if (stats_out) {
    int64_t v[8] = {S.processed, S.excluded_eval, S.excluded_hs, S.hs_skipped, S.recontracted,
                    S.bisected, S.emitted_unique, S.emitted_undecided};
    memcpy(stats_out, v, sizeof v);
  }
  if (status == OR_OK) {
    *n_child = (int64_t)st.len;
    *n_emit = (int64_t)out.len;
    if ((int64_t)st.len > child_cap || (int64_t)out.len > emit_cap) {
      status = OR_ERR_OUTPUT_CAPACITY;
    } else {
      for (size_t c = 0; c < st.len; ++c) {
        for (int k = 0; k < n; ++k) {
          child_lo[c * n + k] = st.a[c].X[k].lo;
          child_hi[c * n + k] = st.a[c].X[k].hi;
        }
        child_rec[c] = (uint32_t)(st.a[c].proven ? 1u : 0u) | ((uint32_t)st.a[c].rc << 8);
      }
      for (size_t e = 0; e < out.len; ++e) {
        for (int k = 0; k < n; ++k) {
          emit_lo[e * n + k] = out.a[e].X[k].lo;
          emit_hi[e * n + k] = out.a[e].X[k].hi;
        }
        emit_tag[e] = out.a[e].tag;
      }
    }
  }
  free(st.a);
  free(out.a);
  return status;
}
