// backtrack.cpp -- the backtracking merge of Alg. 5 (Sec. 3.4) on the host:
// output boxes become cells of the all-coordinate bisection grid of the
// initial box, then every cell of round k is mapped to the round k-1 cell it
// was split from (index j -> j / 2 per coordinate) and duplicates are removed,
// round after round down to the initial box.
//
// Cell j of round k in a coordinate with initial range [a, b] covers
// [B_j, B_{j+1}], B_j = a + j (b - a) / 2^k.  Every comparison of a double
// with a grid line is exact: x >= B_j  <=>  2^k x - 2^k a - j b + j a >= 0, a
// sum of six doubles (two scaled exactly by 2^k, two exact products of j and
// a double split by fused multiply-adds) whose sign is taken from an exact
// floating-point expansion.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ibb.h"

namespace {

// a + b = s + e exactly (round to nearest, no overflow).
inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bv = s - a;
  const double av = s - bv;
  e = (a - av) + (b - bv);
}

// Sign (-1, 0, 1) of the exact sum of m doubles: the terms are accumulated
// into a nonoverlapping expansion (each term is added to every component in
// turn, keeping the rounding errors), whose largest nonzero component has the
// sign of the sum.
int exact_sign(const double* t, int m) {
  double e[16];
  int k = 0;
  for (int i = 0; i < m; ++i) {
    double q = t[i];
    for (int j = 0; j < k; ++j) {
      double s, err;
      two_sum(q, e[j], s, err);
      e[j] = err;
      q = s;
    }
    e[k++] = q;
  }
  for (int j = k - 1; j >= 0; --j)
    if (e[j] != 0.0) return e[j] > 0.0 ? 1 : -1;
  return 0;
}

// Sign of x - B_j on the round-`level` grid of [a, b].
int cmp_line(double x, double a, double b, int level, int64_t j) {
  const double sc = std::ldexp(1.0, level);
  const double jd = (double)j;  // exact: j < 2^53
  const double pb = jd * b, pa = jd * a;
  const double t[6] = {sc * x, -(sc * a), -pb, -std::fma(jd, b, -pb), pa, std::fma(jd, a, -pa)};
  return exact_sign(t, 6);
}

// The j with B_j <= x < B_{j+1}, clamped to [0, 2^level - 1].
int64_t cell_index(double x, double a, double b, int level) {
  const int64_t m = (int64_t)1 << level;
  double est = std::floor((x - a) / (b - a) * std::ldexp(1.0, level));
  int64_t j = est < 0 ? 0 : (est >= (double)m ? m - 1 : (int64_t)est);
  while (j > 0 && cmp_line(x, a, b, level, j) < 0) --j;
  while (j + 1 < m && cmp_line(x, a, b, level, j + 1) >= 0) ++j;
  return j;
}

bool usable(double v) {
  const double a = std::fabs(v);
  return std::isfinite(v) && a <= std::ldexp(1.0, 40) && (a == 0.0 || a >= std::ldexp(1.0, -500));
}

}  // namespace

extern "C" int ibb_backtrack(int32_t n, const double* x0_lo, const double* x0_hi, int64_t m, const double* lo,
                             const double* hi, int32_t level, int64_t* counts, int32_t out_level,
                             int64_t* out_cells, int64_t cap, int64_t* n_out) {
  if (n < 1 || n > IBB_MAX_N || m < 0 || level < 0 || level > IBB_BACKTRACK_MAX_LEVEL || out_level < 0 ||
      out_level > level || !x0_lo || !x0_hi || !counts || !n_out || cap < 0 || (cap > 0 && !out_cells) ||
      (m > 0 && (!lo || !hi)))
    return IBB_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    if (!usable(x0_lo[i]) || !usable(x0_hi[i]) || !(x0_lo[i] < x0_hi[i])) return IBB_ERR_INVALID_ARG;
  for (int64_t b = 0; b < m; ++b)
    for (int i = 0; i < n; ++i) {
      const double l = lo[b * n + i], h = hi[b * n + i];
      if (!std::isfinite(l) || !std::isfinite(h) || l > h || l < x0_lo[i] || h > x0_hi[i])
        return IBB_ERR_INVALID_ARG;
    }
  try {
    // round-`level` cells met by each box: per coordinate a range of indices
    std::vector<int64_t> cells;  // n indices per cell
    std::vector<int64_t> j0((size_t)n), j1((size_t)n), cur((size_t)n);
    for (int64_t b = 0; b < m; ++b) {
      int64_t total = 1;
      for (int i = 0; i < n; ++i) {
        const double l = lo[b * n + i], h = hi[b * n + i], a = x0_lo[i], c = x0_hi[i];
        j0[i] = cell_index(l, a, c, level);
        j1[i] = j0[i];
        if (l < h) {
          j1[i] = cell_index(h, a, c, level);
          // an upper end on a grid line touches the next cell only in a face
          if (j1[i] > j0[i] && cmp_line(h, a, c, level, j1[i]) == 0) --j1[i];
        }
        total *= j1[i] - j0[i] + 1;
        if (total > IBB_BACKTRACK_MAX_CELLS) return IBB_ERR_UNSUPPORTED;
      }
      if ((int64_t)(cells.size() / n) + total > IBB_BACKTRACK_MAX_CELLS) return IBB_ERR_UNSUPPORTED;
      std::copy(j0.begin(), j0.end(), cur.begin());
      for (;;) {
        cells.insert(cells.end(), cur.begin(), cur.end());
        int i = n - 1;
        while (i >= 0 && cur[i] == j1[i]) {
          cur[i] = j0[i];
          --i;
        }
        if (i < 0) break;
        ++cur[i];
      }
    }
    // sort and deduplicate the cells of a round; count them
    std::vector<int64_t> order, tmp;
    auto dedupe = [&]() {
      const int64_t c = (int64_t)(cells.size() / n);
      order.resize((size_t)c);
      for (int64_t k = 0; k < c; ++k) order[k] = k;
      std::sort(order.begin(), order.end(), [&](int64_t p, int64_t q) {
        return std::lexicographical_compare(cells.begin() + p * n, cells.begin() + (p + 1) * n,
                                            cells.begin() + q * n, cells.begin() + (q + 1) * n);
      });
      tmp.clear();
      for (int64_t k = 0; k < c; ++k) {
        const int64_t* x = cells.data() + order[k] * n;
        if (!tmp.empty() && std::equal(x, x + n, tmp.end() - n)) continue;
        tmp.insert(tmp.end(), x, x + n);
      }
      cells.swap(tmp);
      return (int64_t)(cells.size() / n);
    };
    *n_out = 0;
    int status = IBB_OK;
    for (int k = level; k >= 0; --k) {
      counts[k] = dedupe();
      if (k == out_level) {
        *n_out = counts[k];
        if (counts[k] > cap) status = IBB_ERR_OUTPUT_CAPACITY;
        else if (counts[k] > 0) std::memcpy(out_cells, cells.data(), sizeof(int64_t) * cells.size());
      }
      for (auto& j : cells) j >>= 1;  // Alg. 5: the parent cell of round k - 1
    }
    return status;
  } catch (const std::bad_alloc&) {
    return IBB_ERR_NO_MEMORY;
  }
}
