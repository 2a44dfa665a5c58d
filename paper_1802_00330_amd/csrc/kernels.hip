// kernels.hip -- the per-box branch-and-bound step on gfx950.
//
// One persistent cooperative launch runs the whole search tree level by level
// (Alg. 1: the round sets M_0, M_1, ...).  A level's boxes sit in a device
// frontier; waves claim tiles of boxes with one atomic, step them, and append
// children / output boxes with one atomic per wave after a ballot + prefix-sum
// compaction.  A grid barrier separates levels.
//
// Inside a wave, a box is owned by a group of G lanes (G = next power of two
// >= n): lane r owns row r -- equation r for F(X) and J(X), the row of the
// single-precision LU it holds, and, after the LU, the row of the
// preconditioner at its logical pivot position.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/ibb.h"
#include "interval.hpp"
#include "layout.hpp"

namespace ibb {

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work-queue records go between XCDs, whose L2 caches are not coherent with
// each other.  Instead of a device-scope release (an L2 write-back) per push
// and an acquire (an L2 invalidation) per claimed tile, the records are
// stored and loaded at device scope (relaxed device-scope atomic accesses,
// which are written through to, and read from, the point of coherence); a
// producer waits for its record stores to complete (s_waitcnt vmcnt(0))
// before it stores the slot's sequence word, and a consumer loads a record
// only after it has read that word.
__device__ __forceinline__ void store_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_coherent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_coherent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t ballot, int g) {
  constexpr uint64_t gm = (G >= 64) ? ~0ull : ((1ull << G) - 1ull);
  return (ballot >> (g * G)) & gm;
}

template <int G>
__device__ __forceinline__ double group_max(double x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, G));
  return x;
}

// Largest v; ties to the smallest key.  Every lane of the group gets the winner.
template <int G>
__device__ __forceinline__ void group_argmax(double& v, int& key, int& who) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    double ov = __shfl_xor(v, o, G);
    int ok = __shfl_xor(key, o, G);
    int ow = __shfl_xor(who, o, G);
    if (ov > v || (ov == v && ok < key)) {
      v = ov;
      key = ok;
      who = ow;
    }
  }
}

// Inclusive prefix sum over the 64 lanes of the wave.
__device__ __forceinline__ unsigned wave_inclusive_sum(unsigned x) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    unsigned y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// ---------------------------------------------------------------------------
// The compiled system, staged once per workgroup in LDS.
// ---------------------------------------------------------------------------
struct LTable {
  int n;
  const int* eq_off;
  const int* der_off;
  const uint32_t* jnz;
  const double* coef;
  const uint64_t* fac;
  const iv* dco;  // [R(e c), -R(-e c)]: the derivative coefficient, enclosed
  const uint64_t* dfac;
};

// All threads of the block cooperate; requires the FP64 round-down mode.
__device__ __forceinline__ LTable stage_table(const uint64_t* blob, char* lds) {
  const SysDesc* d = reinterpret_cast<const SysDesc*>(blob);
  const int n = d->n, T = d->T, TD = d->TD;
  char* p = lds;
  int* eq_off = reinterpret_cast<int*>(p);
  p += align16(sizeof(int) * (n + 1));
  int* der_off = reinterpret_cast<int*>(p);
  p += align16(sizeof(int) * (n * n + 1));
  uint32_t* jnz = reinterpret_cast<uint32_t*>(p);
  p += align16(sizeof(uint32_t) * kMaxN);
  double* coef = reinterpret_cast<double*>(p);
  p += align16(sizeof(double) * T);
  uint64_t* fac = reinterpret_cast<uint64_t*>(p);
  p += align16(sizeof(uint64_t) * T);
  iv* dco = reinterpret_cast<iv*>(p);
  p += align16(sizeof(iv) * TD);
  uint64_t* dfac = reinterpret_cast<uint64_t*>(p);

  const int* g_eq = reinterpret_cast<const int*>(blob + d->eq_off_w);
  const int* g_der = reinterpret_cast<const int*>(blob + d->der_off_w);
  const double* g_coef = reinterpret_cast<const double*>(blob + d->coef_w);
  const uint64_t* g_fac = blob + d->fac_w;
  const iv* g_dco = reinterpret_cast<const iv*>(blob + d->dco_w);
  const uint64_t* g_dfac = blob + d->dfac_w;
  for (int i = threadIdx.x; i <= n; i += blockDim.x) eq_off[i] = g_eq[i];
  for (int i = threadIdx.x; i <= n * n; i += blockDim.x) der_off[i] = g_der[i];
  for (int i = threadIdx.x; i < kMaxN; i += blockDim.x) jnz[i] = d->jnz[i];
  for (int i = threadIdx.x; i < T; i += blockDim.x) {
    coef[i] = g_coef[i];
    fac[i] = g_fac[i];
  }
  for (int i = threadIdx.x; i < TD; i += blockDim.x) {
    dco[i] = g_dco[i];
    dfac[i] = g_dfac[i];
  }
  return LTable{n, eq_off, der_off, jnz, coef, fac, dco, dfac};
}

// The same table read in place from global memory (batches of systems).
__device__ __forceinline__ LTable global_table(const uint64_t* blob) {
  const SysDesc* d = reinterpret_cast<const SysDesc*>(blob);
  return LTable{d->n,
                reinterpret_cast<const int*>(blob + d->eq_off_w),
                reinterpret_cast<const int*>(blob + d->der_off_w),
                d->jnz,
                reinterpret_cast<const double*>(blob + d->coef_w),
                blob + d->fac_w,
                reinterpret_cast<const iv*>(blob + d->dco_w),
                blob + d->dfac_w};
}

// Encloses every derivative coefficient e_k * c once per system:
// [R(e c), -R(-e c)], written into the blob's dco region.
__global__ void prep_kernel(uint64_t* blobs, const long long* blob_off, int B) {
  set_fp64_round_down();
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    uint64_t* blob = blobs + (blob_off ? blob_off[b] : 0);
    const SysDesc* d = reinterpret_cast<const SysDesc*>(blob);
    const double* dcoef = reinterpret_cast<const double*>(blob + d->dcoef_w);
    const uint32_t* dmult = reinterpret_cast<const uint32_t*>(blob + d->dmult_w);
    double* dco = reinterpret_cast<double*>(blob + d->dco_w);
    for (int i = threadIdx.x; i < d->TD; i += blockDim.x) {
      const double e = (double)dmult[i];
      const double c = dcoef[i];
      dco[2 * i] = rmul(e, c);
      dco[2 * i + 1] = rmul_neg(e, c);
    }
  }
}

// ---------------------------------------------------------------------------
// Interval evaluation (Def. 1): monomials as products of powers, variables
// ascending, coefficient last; equations as sums of terms in stored order.
// ---------------------------------------------------------------------------
//
// The powers of a box's coordinates are staged in LDS before an evaluation:
// the lane owning coordinate v writes X_v^2 and (when E = 3) X_v^3, each the
// value ipow returns, so that a factor x_v^e with e <= E is one LDS read
// instead of a chain set up per term; larger exponents are evaluated by ipow
// in place.  The values are those of ipow in every case, so the evaluation is
// unchanged bit for bit.
template <int E>
struct Powers {
  const iv* p1;  // X
  const iv* p2;  // X^2
  const iv* p3;  // X^3 (E = 3)
};

template <int E>
__device__ __forceinline__ iv factor_power(const Powers<E>& P, uint64_t f) {
  const int v = (int)(f & 0xF), e = (int)((f >> 4) & 0xF);
  if (E == 1) return ipow(P.p1[v], e);
  const iv* src = (e == 2) ? P.p2 : ((E == 3 && e == 3) ? P.p3 : P.p1);
  iv x = src[v];
  if (e > E) x = ipow(x, e);
  return x;
}

// The owner lane of coordinate r stages its powers (called by lanes r < n of
// the groups that evaluate; followed by a wave-level LDS sync).  E = 1 stages
// nothing: every factor is evaluated in place.
template <int E>
__device__ __forceinline__ void stage_powers(const Powers<E>& P, int r) {
  if (E == 1) return;
  const iv x = P.p1[r];
  const_cast<iv*>(P.p2)[r] = ipow(x, 2);
  if (E == 3) const_cast<iv*>(P.p3)[r] = ipow(x, 3);
}

template <int E>
__device__ __forceinline__ iv eval_monomial(uint64_t f, const Powers<E>& P) {
  iv m = factor_power<E>(P, f);
  f >>= 8;
  while (f & 0xF0) {
    m = imul(m, factor_power<E>(P, f));
    f >>= 8;
  }
  return m;
}

template <int E>
__device__ __forceinline__ iv eval_equation(const LTable& t, int i, const Powers<E>& P) {
  const int a = t.eq_off[i], b = t.eq_off[i + 1];
  iv acc{0.0, 0.0};
  for (int q = a; q < b; ++q) {
    const uint64_t f = t.fac[q];
    const double c = t.coef[q];
    iv v = f ? pmul(c, eval_monomial<E>(f, P)) : point_iv(c);
    acc = (q == a) ? v : iadd(acc, v);
  }
  return acc;
}

// Row i of J(X) into J(g, i, 0..n-1) (Alg. 3, first step): d f_i / d x_k is
// the sum of the derivative terms of entry (i, k) in stored order, the first
// term's value being the start of the sum, and [0, 0] without terms.  The
// derivative terms of the row are walked in one loop (columns ascending), so
// the lanes of a wave, whose rows have different numbers of terms per column
// but similar totals, run one loop of about the same length instead of n
// loops of different lengths.
template <int E, typename JV>
__device__ __forceinline__ void eval_jacobian_row(const LTable& t, int i, const Powers<E>& P, const JV& J, int g) {
  const int n = t.n;
  const int* off = t.der_off + i * n;
  const int q1 = off[n];
  int k = 0;
  int kend = off[1];
  iv acc{0.0, -0.0};
  bool have = false;
  for (int q = off[0]; q < q1; ++q) {
    while (q >= kend) {  // column k is complete (or has no terms)
      J(g, i, k) = acc;
      acc = iv{0.0, -0.0};
      have = false;
      ++k;
      kend = off[k + 1];
    }
    const uint64_t f = t.dfac[q];
    const iv c = t.dco[q];
    const iv v = f ? imul(c, eval_monomial<E>(f, P)) : c;
    acc = have ? iadd(acc, v) : v;
    have = true;
  }
  for (; k < n; ++k) {
    J(g, i, k) = acc;
    acc = iv{0.0, -0.0};
  }
}

// ---------------------------------------------------------------------------
// Per-wave scratch in LDS for the W = 64/G boxes of a tile.  Each box's rows
// are padded by one element so that the boxes of a wave (and, in the
// Jacobian, the rows of a box) start on different LDS banks.
// ---------------------------------------------------------------------------
template <int G>
struct Scratch {
  static constexpr int W = 64 / G;
  iv X[W][G + 1];      // current box
  iv Xn[W][G + 1];     // contracted box
  iv D[W][G + 1];      // X - mid X, then X' - mid X as the sweep advances
  iv Fc[W][G + 1];     // F at the expansion point
  iv Xc[W][G + 1];     // expansion point as degenerate intervals
  float row[W][G + 1]; // broadcast buffer of the single-precision solver
};

// A wave's LDS region: its eight tree counters (64 bytes), then Scratch<G>,
// then the Jacobian of its W boxes.
constexpr size_t kWaveHeader = 64;

// The interval Jacobian of the W boxes follows the Scratch block: box g, row
// r, column k at g * (jn * rs + 1) + r * rs + k, with jn = n for one system
// and the largest n among the members for batches of systems of different
// sizes (the area shrinks with jn, which raises the number of resident
// waves; every access has r, k < n <= jn), and a row stride rs of jn or
// jn + 1 (padding spreads the rows of a box over the LDS banks; the host drops
// it when it would cost resident waves).
template <int G>
__host__ __device__ constexpr size_t wave_scratch_bytes(int jn, int rs) {
  return kWaveHeader + ((sizeof(Scratch<G>) + 15) / 16) * 16 + (size_t)(64 / G) * (jn * rs + 1) * sizeof(iv);
}



struct JView {
  iv* p;
  int gs, rs;  // box and row strides
  __device__ __forceinline__ iv& operator()(int g, int r, int k) const { return p[g * gs + r * rs + k]; }
};

// Narrowing of the midpoint of J to single precision, round to nearest.  The
// conversion instruction takes its rounding from the FP32 field of MODE,
// which the kernels leave at round-to-nearest-even.
__device__ __forceinline__ float narrow_rn(double x) { return (float)x; }

// The eight tree counters of a wave, kept in the wave's LDS scratch rather
// than in registers (the search kernels are register-bound): added to by the
// wave's first active lane, flushed to the control block when the wave ends.
struct StepCounters {
  unsigned long long* s;
  __device__ __forceinline__ void add(int k, unsigned long long v) const {
    if (v && __lane_id() == __ffsll((long long)__ballot(1)) - 1) atomicAdd(&s[k], v);
  }
  __device__ __forceinline__ void clear() const {
    if (__lane_id() < 8) s[__lane_id()] = 0ull;
    wave_lds_sync();
  }
  __device__ __forceinline__ void flush(unsigned long long* stats) const {
    wave_lds_sync();
    if (__lane_id() < 8) {
      const unsigned long long v = s[__lane_id()];
      if (v) atomicAdd(&stats[__lane_id()], v);
    }
  }
};

enum : int { kProcessed = 0, kExclEval, kExclHs, kHsSkipped, kRecontract, kBisected, kEmitU, kEmitUnd };

// Extended division N / P (eq 10) followed by Y = x - Q, the intersection
// with X_i and the hull of the pieces (eq 21-22).  Returns false when the
// intersection is empty.  `inside` reports Y strictly inside X_i with Q one
// bounded interval (the uniqueness condition of Alg. 3).
__device__ __forceinline__ bool gs_component(iv N, iv P, double xc, iv Xi, iv& Xn, bool& inside) {
  const double na = N.lo, nb = -N.nhi;
  const double pc = P.lo, pd = -P.nhi;
  const double INF = __builtin_huge_val();
  int npieces = 1;
  double q0l = 0.0, q0h = 0.0, q1l = 0.0, q1h = 0.0;
  bool bounded = false;
  if (pc > 0.0 || pd < 0.0) {
    // ordinary quotient: the extreme endpoint quotients, chosen by sign class
    double ln, ld, hn, hd;
    if (pc > 0.0) {
      if (na >= 0.0) { ln = na; ld = pd; hn = nb; hd = pc; }
      else if (nb <= 0.0) { ln = na; ld = pc; hn = nb; hd = pd; }
      else { ln = na; ld = pc; hn = nb; hd = pc; }
    } else {
      if (na >= 0.0) { ln = nb; ld = pd; hn = na; hd = pc; }
      else if (nb <= 0.0) { ln = nb; ld = pc; hn = na; hd = pd; }
      else { ln = nb; ld = pd; hn = na; hd = pd; }
    }
    q0l = rd_div(ln, ld);
    q0h = ru_div(hn, hd);
    bounded = isfinite(q0l) && isfinite(q0h);
  } else if (na <= 0.0 && nb >= 0.0) {
    q0l = -INF;
    q0h = INF;
  } else if (pc == 0.0 && pd == 0.0) {
    npieces = 0;
  } else if (nb < 0.0) {
    if (pc == 0.0) { q0l = -INF; q0h = ru_div(nb, pd); }
    else if (pd == 0.0) { q0l = rd_div(nb, pc); q0h = INF; }
    else { npieces = 2; q0l = -INF; q0h = ru_div(nb, pd); q1l = rd_div(nb, pc); q1h = INF; }
  } else {
    if (pc == 0.0) { q0l = rd_div(na, pd); q0h = INF; }
    else if (pd == 0.0) { q0l = -INF; q0h = ru_div(na, pc); }
    else { npieces = 2; q0l = -INF; q0h = ru_div(na, pc); q1l = rd_div(na, pd); q1h = INF; }
  }
  bool any = false;
  double lo = 0.0, nhi = 0.0;
  inside = (npieces == 1) && bounded;
  for (int q = 0; q < npieces; ++q) {
    const double ql = q ? q1l : q0l, qh = q ? q1h : q0h;
    const iv Yq = isub(point_iv(xc), make_iv(ql, qh));
    if (npieces == 1) inside = inside && (Xi.lo < Yq.lo) && (Yq.nhi > Xi.nhi);
    const double il = fmax(Yq.lo, Xi.lo), inh = fmax(Yq.nhi, Xi.nhi);
    if (!(il > -inh)) {
      if (!any) {
        lo = il;
        nhi = inh;
        any = true;
      } else {
        lo = fmin(lo, il);
        nhi = fmin(nhi, inh);
      }
    }
  }
  Xn = iv{lo, nhi};
  return any;
}

// One tile: boxes [base, base + W) of the current level (those < cnt).
// Adds v (counted at group leaders) to arr[system]: one atomic per wave when
// all groups of the wave work on the same system, else one per group.
__device__ __forceinline__ void sys_add(unsigned long long* arr, uint32_t sysid, unsigned v, bool leader) {
  const uint32_t s0 = __shfl(sysid, 0, 64);
  const bool same = __ballot(leader && sysid != s0) == 0;
  if (same) {
    const unsigned tot = __shfl(wave_inclusive_sum(leader ? v : 0u), 63, 64);
    if (__lane_id() == 0 && tot) atomicAdd(&arr[s0], (unsigned long long)(long long)(int)tot);
  } else if (leader && v) {
    atomicAdd(&arr[sysid], (unsigned long long)(long long)(int)v);
  }
}

// Work-queue mode: waits (bounded) until ring slot `at` is free for item t.
// A ring that stays full means the live boxes outgrew it: the search stops
// with IBB_ERR_QUEUE_OVERFLOW and the host retries with a larger ring.
__device__ __forceinline__ bool ring_slot_free(const SolveArgs& a, unsigned long long t, size_t at) {
  if (__hip_atomic_load(&a.qseq[at], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == t) return true;
  const long long t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    if (__hip_atomic_load(&a.qseq[at], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == t) return true;
    if (__hip_atomic_load(&a.ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > a.timeout_ticks / 64) {
      atomicCAS(&a.ctrl->status, 0, -4);
      return false;
    }
  }
}

// Per-wave state of a work-queue search, kept in registers: the deepest level
// seen, a run of boxes of one depth not yet added to the depth counts, and the
// wave's share of `pending` not yet applied (never positive, so the global
// count never falls below the boxes still to step).
struct QueueLocal {
  unsigned depth_max = 0;
  unsigned run_depth = 0;
  unsigned long long run_count = 0;
  long long pend = 0;
};

// Work-queue bookkeeping once a wave has read its groups' boxes: the slots are
// freed for the items one ring length later, and the boxes are counted by depth.
__device__ __forceinline__ void queue_after_load(const SolveArgs& a, long long idx, bool valid, uint32_t meta, int r,
                                                 QueueLocal* ql) {
  const int lane = __lane_id();
  const unsigned long long qmask = (unsigned long long)a.front_cap - 1ull;
  // the slot is read once this wave's loads of it have returned (a
  // workgroup-scope fence does not wait for them): free it for the item one
  // ring length later
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  if (valid && r == 0)
    __hip_atomic_store(&a.qseq[(unsigned long long)idx & qmask], (unsigned long long)idx + qmask + 1ull,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // boxes per depth (the round sizes of Alg. 1): runs of one depth are
  // counted in registers and added when the depth changes
  const unsigned depth = meta >> 16;
  const bool lead = valid && r == 0;
  const uint64_t vm = __ballot(lead);
  if (vm) {
    const unsigned d0 = __shfl(depth, __ffsll((long long)vm) - 1, 64);
    const bool same = __ballot(lead && depth == d0) == vm;
    const unsigned long long nv = (unsigned long long)__popcll(vm);
    if (same && (d0 == ql->run_depth || ql->run_count == 0)) {
      ql->run_depth = d0;
      ql->run_count += nv;
    } else if (same) {
      if (lane == 0 && ql->run_depth < (unsigned)a.level_cap)
        atomicAdd(reinterpret_cast<unsigned long long*>(&a.level_sizes[ql->run_depth]), ql->run_count);
      ql->run_depth = d0;
      ql->run_count = nv;
    } else if (lead && depth < (unsigned)a.level_cap) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.level_sizes[depth]), 1ull);
    }
    if (d0 + 1 > ql->depth_max) ql->depth_max = d0 + 1;
    if (!same) {
      unsigned dm = lead ? depth + 1 : 0u;
      for (int o = 32; o > 0; o >>= 1) dm = max(dm, (unsigned)__shfl_xor((int)dm, o, 64));
      if (dm > ql->depth_max) ql->depth_max = dm;
    }
  }
}

// A wave's staging ring of boxes that passed the exclusion test: 2W records
// (box rows (lo, -hi) and the box record) in device memory, indexed by
// monotone counters held by the wave.
struct Stage {
  double* box;     // [2W][G][2]
  uint32_t* meta;  // [2W]
  unsigned long long head = 0, tail = 0;
};

// Level mode (QUEUE = false): boxes [base, base + W) of level `level` in
// front[cur], children appended to front[cur ^ 1].  Work-queue mode: each
// group's box is in ring slot qslot (valid when qvalid), children are
// reserved at the ring's tail and published through qseq.  STAGED: the
// boxes are the next (at most W) records of the wave's staging ring, which
// passed the exclusion test and were counted when they were screened.  VAR:
// the step also supports the Krawczyk contractor and the mean-value test
// (chosen per system at run time); without it, only Hansen-Sengupta and the
// natural extension are compiled in.
template <int G, bool MULTI, bool QUEUE = false, bool STAGED = false, bool VAR = true>
__device__ __forceinline__ void step_tile(const SolveArgs& a, const LTable& Tl, Scratch<G>& S, const JView J,
                          long long base,
                          long long cnt, int cur, int level, unsigned long long* next_count,
                          const StepCounters& sc, long long qslot = 0, bool qvalid = false,
                          QueueLocal* ql = nullptr, Stage* stg = nullptr) {
  const int lane = __lane_id();
  const int g = lane / G;
  const int r = lane % G;
  const unsigned long long qmask = (unsigned long long)a.front_cap - 1ull;
  const long long idx = QUEUE ? qslot : base + g;
  bool valid = STAGED ? (stg->head + (unsigned long long)g < stg->tail) : (QUEUE ? qvalid : idx < cnt);
  // the group's system: its table, size and parameters
  LTable T = Tl;
  uint32_t sysid = 0;
  double p_hsw = a.hs_max_width;
  // split mode (bits 0-1), contractor (bit 2), inclusion (bit 3), most
  // consecutive re-contractions (bits 8-15): one register per group in batches
  int p_mode = a.split_mode | (a.contractor << 2) | (a.inclusion << 3) | (a.max_rc << 8);
  unsigned long long room = 0;  // batches: nodes the system may add at the next level
  if (MULTI) {
    if (valid) sysid = a.sys[cur][idx];
    // serving: a system the host failed (its boxes outgrew the device pool)
    if (valid && a.evict && a.evict[sysid]) valid = false;
    T = global_table(a.blobs + a.blob_off[sysid]);
    const SysParams sp = a.sp[sysid];
    p_hsw = sp.hs_max_width;
    p_mode = sp.split_mode | (sp.contractor << 2) | (sp.inclusion << 3) | (sp.max_rc << 8);
    if (valid) {
      // the budget is on the system's tree nodes, checked level by level
      const unsigned long long total =
          a.cum_sys[(size_t)((level + 1) & 1) * a.B + sysid] + a.count_sys[(size_t)(level % 3) * a.B + sysid];
      if (total > (unsigned long long)sp.max_boxes) {
        if (r == 0) atomicCAS(&a.status_sys[sysid], 0, -2);
        valid = false;
      } else {
        room = (unsigned long long)sp.max_boxes - total;
        if (r == 0) {
          a.cum_sys[(size_t)(level & 1) * a.B + sysid] = total;
          a.count_sys[(size_t)((level + 2) % 3) * a.B + sysid] = 0ull;
        }
      }
    }
  }
  const int n = T.n;
  const bool row_ok = r < n;
  double* const dbg = (a.dbg && (STAGED ? g == 0 : idx == 0) && valid) ? a.dbg : nullptr;

  // ---- load the box and its record
  uint32_t meta = 0;
  if (STAGED) {
    if (valid) {
      const size_t at = (size_t)((stg->head + (unsigned long long)g) % (unsigned long long)(2 * (64 / G)));
      if (row_ok) {
        const double* src = stg->box + (at * G + r) * 2;
        S.X[g][r] = iv{src[0], src[1]};
      }
      meta = stg->meta[at];
    }
  } else if (valid) {
    const size_t at = QUEUE ? (size_t)((unsigned long long)idx & qmask) : (size_t)idx;
    const int buf = QUEUE ? 0 : cur;
    if (row_ok) {
      const double* src = a.front[buf] + (at * G + r) * 2;
      S.X[g][r] = QUEUE ? iv{load_coherent(src), load_coherent(src + 1)} : iv{src[0], src[1]};
    }
    meta = QUEUE ? load_coherent(&a.meta[buf][at]) : a.meta[buf][at];
  }
  const bool proven = meta & 1u;
  const int rc = (int)((meta >> 8) & 0xFF);
  wave_lds_sync();
  if (QUEUE && !STAGED) queue_after_load(a, idx, valid, meta, r, ql);

  // ---- exclusion test (Def. 2): some F_i(X) excludes 0
  bool excl_row = false;
  if (!STAGED) {
    // powers of X in the contracted-box and X - x rows, free until the
    // contraction (batches of up to 16 unknowns: none, which keeps their
    // register budget)
    constexpr int E = (MULTI && G == 16) ? 1 : 3;
    const Powers<E> PX{S.X[g], S.Xn[g], S.D[g]};
    if (valid && !proven && row_ok) stage_powers<E>(PX, r);
    wave_lds_sync();
    if (valid && !proven && row_ok) {
      const iv f = eval_equation<E>(T, r, PX);
      excl_row = f.lo > 0.0 || f.nhi > 0.0;
    }
    wave_lds_sync();
  }
  const bool excluded = group_bits<G>(__ballot(excl_row), g) != 0;
  const bool active = valid && !excluded;

  // ---- width of X
  const double w = group_max<G>((active && row_ok) ? iwidth(S.X[g][r]) : 0.0);
  bool do_hs = active && !(w > p_hsw);
  // the mean-value form (a centred inclusion of F) as a second exclusion
  // test, on boxes not proven to hold a root
  const bool do_mv = VAR && active && !proven && ((p_mode >> 3) & 1) != 0;
  const bool do_j = do_hs || do_mv;

  bool hs_empty = false, hs_unique = false, run = false, mv_excl = false;
  if (__ballot(do_j) != 0) {
    // H1: expansion point x = mid X, with its powers in the contracted-box
    // and X - x rows (free until the contraction and until H8)
    // (batches of up to 16 unknowns stage none, which keeps their register budget)
    constexpr int EC = (MULTI && G == 16) ? 1 : 3, EX = (MULTI && G == 16) ? 1 : 2;
    const Powers<EC> PC{S.Xc[g], S.Xn[g], S.D[g]};
    if (do_j && row_ok) {
      S.Xc[g][r] = point_iv(imid(S.X[g][r]));
      stage_powers<EC>(PC, r);
    }
    wave_lds_sync();
    // H3: F_r at the degenerate box [x, x]
    if (do_j && row_ok) S.Fc[g][r] = eval_equation<EC>(T, r, PC);
    wave_lds_sync();
    // H8: X - x; the square of X in the contracted-box row
    const Powers<EX> PX{S.X[g], S.Xn[g], nullptr};
    if (do_j && row_ok) {
      const iv x = S.X[g][r];
      S.D[g][r] = isub(x, S.Xc[g][r]);
      stage_powers<EX>(PX, r);
    }
    wave_lds_sync();
    // H2: row r of J(X)
    if (do_j && row_ok) {
      eval_jacobian_row<EX>(T, r, PX, J, g);
      if (dbg) {
        for (int k = 0; k < n; ++k) {
          dbg[dbg_off_J(n) + (r * n + k) * 2] = J(g, r, k).lo;
          dbg[dbg_off_J(n) + (r * n + k) * 2 + 1] = -J(g, r, k).nhi;
        }
        dbg[dbg_off_F(n) + 2 * r] = S.Fc[g][r].lo;
        dbg[dbg_off_F(n) + 2 * r + 1] = -S.Fc[g][r].nhi;
      }
    }
    wave_lds_sync();
    // mean-value form: F_r(x) + sum_k J_rk(X) (X_k - x_k), k ascending; the box
    // is discarded when some row excludes 0 (its natural F(X) held 0)
    if (VAR && __ballot(do_mv) != 0) {
      bool ex_row = false;
      if (do_mv && row_ok) {
        iv acc = S.Fc[g][r];
        for (int k = 0; k < n; ++k) acc = iadd(acc, imul(J(g, r, k), S.D[g][k]));
        ex_row = acc.lo > 0.0 || acc.nhi > 0.0;
      }
      mv_excl = do_mv && group_bits<G>(__ballot(ex_row), g) != 0;
      do_hs = do_hs && !mv_excl;
    }
    // H4: single-precision mid J, row r
    float M[G];
#pragma unroll
    for (int k = 0; k < G; ++k) M[k] = (do_hs && row_ok && k < n) ? narrow_rn(imid(J(g, r, k))) : 0.0f;
    if (dbg && row_ok) {
#pragma unroll
      for (int k = 0; k < G; ++k)
        if (k < n) dbg[dbg_off_M(n) + r * n + k] = (double)M[k];
    }

    // H5: LU with partial pivoting across the lanes of the group; pos is the
    // logical row this lane's data occupies after the row exchanges.
    int pos = r;
    bool bad = false, zero_pivot = false;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      if (k < n) {
        double v = (do_hs && row_ok && pos >= k) ? (double)fabsf(M[k]) : -1.0;
        int key = pos, who = r;
        group_argmax<G>(v, key, who);
        const float piv = __shfl(M[k], who, G);
        if (piv == 0.0f) zero_pivot = true;
        const int was = pos;
        if (was == k) pos = key;  // exchange logical rows k and key
        if (r == who) {
          pos = k;
#pragma unroll
          for (int j = k; j < G; ++j) S.row[g][j] = M[j];
        }
        wave_lds_sync();
        if (do_hs && row_ok && pos > k) {
          const float l = M[k] / piv;
          M[k] = l;
#pragma unroll
          for (int j = k + 1; j < G; ++j) {
            if (j < n) {
              const float prod = l * S.row[g][j];
              M[j] = M[j] - prod;
            }
          }
        }
        wave_lds_sync();
      }
    }
    if (row_ok) {
#pragma unroll
      for (int j = 0; j < G; ++j)
        if (j < n && !isfinite(M[j])) bad = true;
    }
    // Forward substitution L z = P e_c for all columns c at once: the lane at
    // logical row i holds z_i for every c; its right-hand side is e_r.
    float z[G];
#pragma unroll
    for (int c = 0; c < G; ++c) z[c] = (c == r) ? 1.0f : 0.0f;
#pragma unroll
    for (int j = 0; j < G; ++j) {
      if (j < n) {
        if (pos == j && row_ok) {
#pragma unroll
          for (int c = 0; c < G; ++c) S.row[g][c] = z[c];
        }
        wave_lds_sync();
        if (do_hs && row_ok && pos > j) {
          const float L = M[j];
#pragma unroll
          for (int c = 0; c < G; ++c) {
            if (c < n) {
              const float prod = L * S.row[g][c];
              z[c] = z[c] - prod;
            }
          }
        }
        wave_lds_sync();
      }
    }
    // Back substitution U x = z, logical rows from n-1 down: x_j = t / U_jj,
    // and every earlier row subtracts U_ij x_j as x_j becomes known.
#pragma unroll
    for (int j = G - 1; j >= 0; --j) {
      if (j < n) {
        if (pos == j && row_ok) {
          const float u = M[j];
#pragma unroll
          for (int c = 0; c < G; ++c) {
            if (c < n) z[c] = z[c] / u;
            S.row[g][c] = z[c];
          }
        }
        wave_lds_sync();
        if (do_hs && row_ok && pos < j) {
          const float U = M[j];
#pragma unroll
          for (int c = 0; c < G; ++c) {
            if (c < n) {
              const float prod = U * S.row[g][c];
              z[c] = z[c] - prod;
            }
          }
        }
        wave_lds_sync();
      }
    }
    if (row_ok) {
#pragma unroll
      for (int c = 0; c < G; ++c)
        if (c < n && !isfinite(z[c])) bad = true;
    }
    const bool skip = group_bits<G>(__ballot(bad || zero_pivot), g) != 0;
    run = do_hs && !skip;
    if (dbg && row_ok) {
#pragma unroll
      for (int c = 0; c < G; ++c)
        if (c < n) dbg[dbg_off_Y(n) + pos * n + c] = (double)z[c];
      if (r == 0) dbg[dbg_off_flags(n)] = skip ? 1.0 : 0.0;
    }

    // H6, H7: this lane holds row `pos` of Y.
    //   g_pos = sum_m Y[pos][m] F_m(x),  P[pos][j] = sum_m Y[pos][m] J[m][j],
    // m ascending from the first term; exactly-zero terms are omitted.  P is
    // formed column by column; once every lane has read column j of J, the
    // column is overwritten by column j of P (row = logical position).
    iv gv{0.0, 0.0};
    if (run && row_ok) {
      bool hg = false;
      for (int m = 0; m < n; ++m) {
        float ym = 0.0f;
#pragma unroll
        for (int c = 0; c < G; ++c)
          if (c == m) ym = z[c];
        const double y = (double)ym;
        const iv fm = S.Fc[g][m];
        if (y != 0.0 && !is_zero(fm)) {
          const iv t = pmul(y, fm);
          gv = hg ? iadd(gv, t) : t;
          hg = true;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < G; ++j) {
      iv pj{0.0, 0.0};
      if (run && row_ok && j < n) {
        bool have = false;
#pragma unroll
        for (int m = 0; m < G; ++m) {
          if (m < n && ((T.jnz[m] >> j) & 1u) && z[m] != 0.0f) {
            const iv t = pmul((double)z[m], J(g, m, j));
            pj = have ? iadd(pj, t) : t;
            have = true;
          }
        }
      }
      wave_lds_sync();
      if (run && row_ok && j < n) J(g, pos, j) = pj;
    }
    wave_lds_sync();
    if (dbg && run && row_ok) {
      dbg[dbg_off_g(n) + 2 * pos] = gv.lo;
      dbg[dbg_off_g(n) + 2 * pos + 1] = -gv.nhi;
      for (int j = 0; j < n; ++j) {
        dbg[dbg_off_P(n) + (pos * n + j) * 2] = J(g, pos, j).lo;
        dbg[dbg_off_P(n) + (pos * n + j) * 2 + 1] = -J(g, pos, j).nhi;
      }
    }
    bool my_unique = true, my_empty = false;
    if (VAR && ((p_mode >> 2) & 1)) {
      // Krawczyk (eq 15-16): K = x - g + (I - P)(X - x), every component
      // from X; X' = K meets X; K inside the interior of X proves one root.
      // The sum over j ascending starts from its first term.
      if (run && row_ok) {
        iv SK{0.0, 0.0};
        for (int j = 0; j < n; ++j) {
          const iv pj = J(g, pos, j);
          const iv m = (j == pos) ? isub(point_iv(1.0), pj) : iv{pj.nhi, pj.lo};  // 1 - P_jj or -P_ij
          const iv t = imul(m, S.D[g][j]);
          SK = j ? iadd(SK, t) : t;
        }
        const double xc = S.Xc[g][pos].lo;
        const iv K = iadd(isub(point_iv(xc), gv), SK);
        const iv Xi = S.X[g][pos];
        const double il = fmax(K.lo, Xi.lo), inh = fmax(K.nhi, Xi.nhi);
        my_empty = il > -inh;
        my_unique = !my_empty && Xi.lo < K.lo && Xi.nhi < K.nhi;
        const iv xn = my_empty ? Xi : iv{il, inh};
        if (dbg) {
          dbg[dbg_off_N(n) + 2 * pos] = K.lo;
          dbg[dbg_off_N(n) + 2 * pos + 1] = -K.nhi;
          dbg[dbg_off_X(n) + 2 * pos] = xn.lo;
          dbg[dbg_off_X(n) + 2 * pos + 1] = -xn.nhi;
        }
        S.Xn[g][pos] = xn;
      }
      wave_lds_sync();
    } else {
      // H9: Gauss-Seidel sweep (eq 21-22).  The bracket
      //   g_i + sum_{j<i} P_ij (X'_j - x_j) + sum_{j>i} P_ij (X_j - x_j)
      // is formed as (g_i + S_L) + S_U, each sum on its own, j ascending.
      iv SU{0.0, 0.0};
      bool hasU = false;
      if (run && row_ok) {
        for (int j = pos + 1; j < n; ++j) {
          const iv t = imul(J(g, pos, j), S.D[g][j]);
          SU = hasU ? iadd(SU, t) : t;
          hasU = true;
        }
      }
      iv SL{0.0, 0.0};
      bool hasL = false;
      const int nsweep = MULTI ? G : n;
      for (int i = 0; i < nsweep; ++i) {
        if (run && row_ok && pos == i) {
          iv N = gv;
          if (hasL) N = iadd(N, SL);
          if (hasU) N = iadd(N, SU);
          const double xc = S.Xc[g][i].lo;
          iv xn;
          bool inside = false;
          const bool ok = gs_component(N, J(g, i, i), xc, S.X[g][i], xn, inside);
          my_empty = !ok;
          my_unique = ok && inside;
          if (!ok) xn = S.X[g][i];
          if (dbg) {
            dbg[dbg_off_N(n) + 2 * i] = N.lo;
            dbg[dbg_off_N(n) + 2 * i + 1] = -N.nhi;
            dbg[dbg_off_X(n) + 2 * i] = xn.lo;
            dbg[dbg_off_X(n) + 2 * i + 1] = -xn.nhi;
          }
          S.Xn[g][i] = xn;
          S.D[g][i] = isub(xn, point_iv(xc));
        }
        wave_lds_sync();
        if (run && row_ok && pos > i) {
          const iv t = imul(J(g, pos, i), S.D[g][i]);
          SL = hasL ? iadd(SL, t) : t;
          hasL = true;
        }
      }
    }
    hs_empty = run && group_bits<G>(__ballot(my_empty), g) != 0;
    hs_unique = run && group_bits<G>(__ballot(row_ok && !my_unique), g) == 0;
    if (dbg && r == 0) {
      dbg[dbg_off_flags(n) + 1] = hs_empty ? 1.0 : 0.0;
      dbg[dbg_off_flags(n) + 2] = hs_unique ? 1.0 : 0.0;
      dbg[dbg_off_flags(n) + 3] = run ? 1.0 : 0.0;
    }
  }
  // boxes without a contraction keep X as X'
  if (active && !run && row_ok) S.Xn[g][r] = S.X[g][r];
  wave_lds_sync();

  // ---- decisions (S3-S7), uniform per group
  const bool alive = active && !mv_excl && !hs_empty;
  const bool prv = proven || (alive && run && hs_unique);
  double wn = (alive && row_ok) ? iwidth(S.Xn[g][r]) : -1.0;
  int kk = r, whok = r;
  group_argmax<G>(wn, kk, whok);

  const uint32_t child_depth = QUEUE ? ((meta >> 16) + 1u) << 16 : 0u;
  int n_push = 0;
  bool emit = false;
  int tag = 0;
  int kind = 0;  // 0 none, 1 same box again, 2 widest split, 3 split all
  uint32_t child_meta = 0;
  double mid_kk = 0.0;
  uint32_t split_mask = 0;
  // tolerance and re-contraction ratio, read where they are used (batches:
  // the group's system; fewer values live across the contraction)
  const double p_tol = MULTI ? a.sp[sysid].tol : a.tol;
  const double p_ratio = MULTI ? a.sp[sysid].ratio : a.ratio;
  if (alive) {
    if (wn <= p_tol) {
      emit = true;
      tag = prv ? 1 : 0;
    } else if (prv) {
      if (wn < w && rc + 1 < (p_mode >> 8)) {
        kind = 1;
        n_push = 1;
        child_meta = 1u | ((uint32_t)(rc + 1) << 8) | child_depth;
      } else {
        emit = true;
        tag = 1;
      }
    } else if (wn <= rmul(p_ratio, w) && rc + 1 < (p_mode >> 8)) {
      kind = 1;
      n_push = 1;
      child_meta = ((uint32_t)(rc + 1) << 8) | child_depth;
    } else if ((p_mode & 3) == 0) {
      const iv xk = S.Xn[g][kk];
      mid_kk = imid(xk);
      if (!(mid_kk > xk.lo && mid_kk < -xk.nhi)) {
        emit = true;
        tag = 0;
      } else {
        kind = 2;
        n_push = 2;
      }
    }
  }
  if (__ballot((p_mode & 3) != 0) != 0) {
    bool can = false;
    if (alive && row_ok && (p_mode & 3) != 0) {
      const iv xr = S.Xn[g][r];
      const double m = imid(xr);
      can = m > xr.lo && m < -xr.nhi;
    }
    split_mask = (uint32_t)group_bits<G>(__ballot(can), g);
    if (alive && !emit && kind == 0 && (p_mode & 3) != 0) {
      if (split_mask == 0) {
        emit = true;
        tag = 0;
      } else {
        kind = 3;
        n_push = 1 << __popc(split_mask);
      }
    }
  }

  // Batches: once the next level alone takes a system over its budget, the
  // system fails when that level is loaded whatever its other boxes do, so
  // the children need not be stored (a budget failure would otherwise fill
  // the frontier with boxes that are only read to be dropped).  They are
  // still counted, which keeps that check, and every counter, as it was.
  // The count read here lacks this group's children and perhaps others', so
  // the test never fires for a system that stays within its budget.  Other
  // waves update the count meanwhile, so it is read once per group (by its
  // first lane) and the decision is broadcast: every lane of a group must
  // agree with the reservation its first lane makes below.
  bool store = true;
  if (MULTI && !QUEUE) {
    int drop = 0;
    if (r == 0 && n_push > 0) {
      const unsigned long long seen = __hip_atomic_load(&a.count_sys[(size_t)((level + 1) % 3) * a.B + sysid],
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (seen + (unsigned long long)n_push > room) {
        drop = 1;
        atomicCAS(&a.status_sys[sysid], 0, -2);
      }
    }
    store = __shfl(drop, g * G, 64) == 0;
  }

  // ---- counters, once per group
  const bool leader = (r == 0) && valid;
  if (MULTI) {
    unsigned long long* st = a.stats_sys;
    const uint32_t o8 = sysid * 8u;
    sys_add(st + kProcessed, o8, 1u, leader);
    sys_add(st + kExclEval, o8, (excluded || mv_excl) ? 1u : 0u, leader);
    sys_add(st + kExclHs, o8, hs_empty ? 1u : 0u, leader);
    sys_add(st + kHsSkipped, o8, (active && !mv_excl && !run) ? 1u : 0u, leader);
    sys_add(st + kRecontract, o8, kind == 1 ? 1u : 0u, leader);
    sys_add(st + kBisected, o8, (kind == 2 || kind == 3) ? 1u : 0u, leader);
    sys_add(st + kEmitU, o8, (emit && tag == 1) ? 1u : 0u, leader);
    sys_add(st + kEmitUnd, o8, (emit && tag == 0) ? 1u : 0u, leader);
    sys_add(a.count_sys + (size_t)((level + 1) % 3) * a.B, sysid, (unsigned)n_push, leader);
    if (a.pending_sys) {
      // boxes still to step: + children stored - this box (two's complement)
      sys_add(a.pending_sys, sysid, (unsigned)((store ? n_push : 0) - 1), leader);
      const bool dropped = (idx < cnt) && !valid && r == 0;  // over the budget
      sys_add(a.pending_sys, sysid, 0xFFFFFFFFu, dropped);
    }
  }
  if (!STAGED) sc.add(kProcessed, (unsigned long long)(__popcll(__ballot(leader))));
  sc.add(kExclEval, (unsigned long long)(__popcll(__ballot(leader && (excluded || mv_excl)))));
  sc.add(kExclHs, (unsigned long long)(__popcll(__ballot(leader && hs_empty))));
  sc.add(kHsSkipped, (unsigned long long)(__popcll(__ballot(leader && active && !mv_excl && !run))));
  sc.add(kRecontract, (unsigned long long)(__popcll(__ballot(leader && kind == 1))));
  sc.add(kBisected, (unsigned long long)(__popcll(__ballot(leader && (kind == 2 || kind == 3)))));
  sc.add(kEmitU, (unsigned long long)(__popcll(__ballot(leader && emit && tag == 1))));
  sc.add(kEmitUnd, (unsigned long long)(__popcll(__ballot(leader && emit && tag == 0))));

  // ---- compaction: one atomic per wave for the pushes, one for the emits
  const unsigned my_push = (r == 0 && store) ? (unsigned)n_push : 0u;
  const unsigned my_emit = (r == 0 && emit) ? 1u : 0u;
  const unsigned incl_p = wave_inclusive_sum(my_push);
  const unsigned incl_e = wave_inclusive_sum(my_emit);
  const unsigned tot_p = __shfl(incl_p, 63, 64);
  const unsigned tot_e = __shfl(incl_e, 63, 64);
  unsigned long long pbase = 0, ebase = 0;
  if (lane == 0) {
    if (tot_p) {
      pbase = atomicAdd(QUEUE ? &a.ctrl->qtail : next_count, (unsigned long long)tot_p);
      // work queue: every created box is a tree node, so the budget (more
      // than max_boxes nodes) fails exactly when the boxes created exceed it
      if (QUEUE && pbase + tot_p > (unsigned long long)a.max_boxes) atomicCAS(&a.ctrl->status, 0, -2);
    }
    if (tot_e && !(MULTI && a.slot_out_cap > 0)) ebase = atomicAdd(a.out_count, (unsigned long long)tot_e);
  }
  pbase = __shfl(pbase, 0, 64);
  ebase = __shfl(ebase, 0, 64);
  const unsigned gp = __shfl(incl_p - my_push, g * G, 64);
  const unsigned ge = __shfl(incl_e - my_emit, g * G, 64);

  unsigned long long slot_o = 0;
  if (MULTI && a.slot_out_cap > 0) {
    // per-system output regions (serving): one record per emitted box
    if (emit && r == 0) slot_o = atomicAdd(&a.slot_out_count[sysid], 1ull);
    slot_o = __shfl(slot_o, g * G, 64);
  }
  if (emit && MULTI && a.slot_out_cap > 0) {
    const unsigned long long o = slot_o;
    if (o < (unsigned long long)a.slot_out_cap) {
      const size_t rec = (size_t)sysid * a.slot_out_cap + o;
      if (row_ok) {
        const iv x = S.Xn[g][r];
        double* dst = a.out_box + (rec * a.out_stride + r) * 2;
        dst[0] = x.lo;
        dst[1] = x.nhi;
      }
      if (r == 0) a.out_tag[rec] = (uint32_t)tag;
    }
  } else if (emit) {
    const unsigned long long o = ebase + ge;
    if (o < (unsigned long long)a.out_cap) {
      if (row_ok) {
        const iv x = S.Xn[g][r];
        double* dst = a.out_box + ((size_t)o * a.out_stride + r) * 2;
        dst[0] = x.lo;
        dst[1] = x.nhi;
      }
      if (r == 0) {
        a.out_tag[o] = (uint32_t)tag;
        if (MULTI) a.out_sys[o] = sysid;
      }
    }
  }
  // children: level mode appends to the next level's buffer; work-queue mode
  // writes into the reserved ring items once their slots are free
  const unsigned long long o = pbase + gp;
  int pushed = 0;
  if (n_push && store) {
    const iv x = row_ok ? S.Xn[g][r] : iv{0.0, 0.0};
    const bool mine = (split_mask >> r) & 1u;
    const int q = __popc(split_mask & ((1u << r) - 1u));
    const double m = (kind == 3 && row_ok) ? imid(x) : 0.0;
    const int buf = QUEUE ? 0 : cur ^ 1;
    for (int c = 0; c < n_push; ++c) {
      const unsigned long long t = o + (unsigned long long)c;
      size_t at;
      if (QUEUE) {
        at = (size_t)(t & qmask);
        if (!ring_slot_free(a, t, at)) break;
      } else {
        if (t >= (unsigned long long)a.front_cap) break;
        at = (size_t)t;
      }
      if (row_ok) {
        iv y = x;
        if (kind == 2 && r == kk) y = c ? iv{mid_kk, x.nhi} : iv{x.lo, -mid_kk};
        if (kind == 3 && mine) y = ((c >> q) & 1) ? iv{m, x.nhi} : iv{x.lo, -m};
        double* dst = a.front[buf] + (at * G + r) * 2;
        if (QUEUE) {
          store_coherent(dst, y.lo);
          store_coherent(dst + 1, y.nhi);
        } else {
          dst[0] = y.lo;
          dst[1] = y.nhi;
        }
      }
      if (r == 0) {
        if (QUEUE) store_coherent(&a.meta[buf][at], kind == 1 ? child_meta : child_depth);
        else a.meta[buf][at] = kind == 1 ? child_meta : child_depth;
        if (MULTI) a.sys[buf][at] = sysid;
      }
      pushed = c + 1;
    }
  }
  if (QUEUE) {
    // publish: the boxes were stored at device scope (coherent stores, see
    // store_coherent); they are complete before the slot flags are stored
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (r == 0)
      for (int c = 0; c < pushed; ++c)
        __hip_atomic_store(&a.qseq[(o + (unsigned long long)c) & qmask], o + (unsigned long long)c + 1ull,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // boxes still to step: + children - this box, summed over the wave; a
    // positive balance is applied at once (after the children are published)
    const unsigned delta = (valid && r == 0) ? (unsigned)(n_push - 1) : 0u;
    ql->pend += (long long)(int)__shfl(wave_inclusive_sum(delta), 63, 64);
    if (ql->pend > 0) {
      if (lane == 0) atomicAdd(&a.ctrl->pending, (unsigned long long)ql->pend);
      ql->pend = 0;
    }
  }
  wave_lds_sync();
}

// Stage one of a step for one system: the boxes of a tile (level mode: boxes
// [base, base + W) of front[cur]; work-queue mode: the groups' ring items) are
// read and tested for exclusion (Def. 2); every box is counted as processed,
// excluded ones as excluded by evaluation, and the others (proven boxes skip
// the test) are appended to the wave's staging ring, to be stepped W at a time
// by step_tile<..., STAGED> so that no group of a wave idles through the
// contraction because its box was excluded.
template <int G, bool QUEUE>
__device__ __forceinline__ void screen_tile(const SolveArgs& a, const LTable& T, Scratch<G>& S, long long base,
                                            long long cnt, int cur, const StepCounters& sc, long long qslot, bool qvalid,
                                            QueueLocal* ql, Stage& stg) {
  constexpr int W = 64 / G;
  const int lane = __lane_id();
  const int g = lane / G;
  const int r = lane % G;
  const unsigned long long qmask = (unsigned long long)a.front_cap - 1ull;
  const long long idx = QUEUE ? qslot : base + g;
  const bool valid = QUEUE ? qvalid : idx < cnt;
  const int n = T.n;
  const bool row_ok = r < n;
  uint32_t meta = 0;
  if (valid) {
    const size_t at = QUEUE ? (size_t)((unsigned long long)idx & qmask) : (size_t)idx;
    const int buf = QUEUE ? 0 : cur;
    if (row_ok) {
      const double* src = a.front[buf] + (at * G + r) * 2;
      S.X[g][r] = QUEUE ? iv{load_coherent(src), load_coherent(src + 1)} : iv{src[0], src[1]};
    }
    meta = QUEUE ? load_coherent(&a.meta[buf][at]) : a.meta[buf][at];
  }
  const bool proven = meta & 1u;
  wave_lds_sync();
  if (QUEUE) queue_after_load(a, idx, valid, meta, r, ql);
  bool excl_row = false;
  // powers of X in the contracted-box and X - x rows (not in use while screening)
  const Powers<3> PX{S.X[g], S.Xn[g], S.D[g]};
  if (valid && !proven && row_ok) stage_powers<3>(PX, r);
  wave_lds_sync();
  if (valid && !proven && row_ok) {
    const iv f = eval_equation<3>(T, r, PX);
    excl_row = f.lo > 0.0 || f.nhi > 0.0;
  }
  const bool excluded = group_bits<G>(__ballot(excl_row), g) != 0;
  const bool leader = valid && r == 0;
  sc.add(kProcessed, (unsigned long long)(__popcll(__ballot(leader))));
  const unsigned n_excl = (unsigned)__popcll(__ballot(leader && excluded));
  sc.add(kExclEval, (unsigned long long)(n_excl));
  if (QUEUE) ql->pend -= (long long)n_excl;  // stepped boxes without children
  // survivors into the staging ring, in group order
  const bool keep = valid && !excluded;
  const uint64_t km = __ballot(keep && r == 0);
  if (keep) {
    const uint64_t below = (g == 0) ? 0ull : (km & ((1ull << (g * G)) - 1ull));
    const size_t at = (size_t)((stg.tail + (unsigned long long)__popcll(below)) % (unsigned long long)(2 * W));
    if (row_ok) {
      const iv x = S.X[g][r];
      double* dst = stg.box + (at * G + r) * 2;
      dst[0] = x.lo;
      dst[1] = x.nhi;
    }
    if (r == 0) stg.meta[at] = meta;
  }
  stg.tail += (unsigned long long)__popcll(km);
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Grid barrier between levels.  The boxes a level writes are read by
// workgroups on other XCDs, whose L2 caches are not coherent with this one's,
// so each workgroup writes its XCD's L2 back before it arrives and
// invalidates its caches after the release: once per workgroup (its first
// thread, after every wave's stores have left the CU), not once per wave,
// which would repeat the write-back and invalidation thousands of times per
// level.  Arrivals are counted per group of workgroups (blockIdx % 8, one
// counter line each); the last arrival of a group arrives at the global
// counter, and the last group raises every group's release flag, which the
// group's workgroups poll.  `gen` counts the barriers of the launch (the
// barrier lines are zero at launch).  Every wait is bounded: after
// timeout_ticks of the 100 MHz device clock the barrier records
// IBB_ERR_TIMEOUT and returns, and every later wait returns as soon as it
// sees a non-zero status.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void grid_barrier(const SolveArgs& a, unsigned long long& gen) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  ++gen;
  if (threadIdx.x == 0) {
    Ctrl* c = a.ctrl;
    unsigned long long* const arrive = c->sync;
    unsigned long long* const flag = c->sync + kSyncGroups * kSyncStride;
    const unsigned x = blockIdx.x % (unsigned)kSyncGroups;
    const unsigned long long groups =
        a.nblocks < kSyncGroups ? (unsigned long long)a.nblocks : (unsigned long long)kSyncGroups;
    const unsigned long long members =
        ((unsigned long long)a.nblocks - x + (unsigned long long)kSyncGroups - 1ull) / (unsigned long long)kSyncGroups;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned long long old =
        __hip_atomic_fetch_add(&arrive[x * kSyncStride], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1ull == members * gen) {
      // the group's last arrival carries the group's writes on
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      const unsigned long long g = __hip_atomic_fetch_add(&c->bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (g + 1ull == groups * gen) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        for (int y = 0; y < kSyncGroups; ++y)
          __hip_atomic_store(&flag[y * kSyncStride], gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(&flag[x * kSyncStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
      __builtin_amdgcn_s_sleep(2);
      if (__hip_atomic_load(&c->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if ((long long)(wall_clock64() - t0) > a.timeout_ticks) {
        atomicCAS(&c->status, 0, -8);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Resident waves per SIMD the register allocation aims for: three for one
// system of up to 8 unknowns (its n-sized LDS scratch lets three workgroups of
// four waves fit a CU) and for batches (scratch sized for the largest member:
// up to ten waves per CU at n = 12), two for one system of 9 to 16 unknowns
// (its table and scratch admit no more).
template <int G, bool MULTI>
struct Occupancy {
  static constexpr int waves = (MULTI || G <= 8) ? 3 : 2;
};

template <int G, bool MULTI, bool VAR>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Occupancy<G, MULTI>::waves)))
solve_kernel(SolveArgs a) {
  set_fp64_round_down();
  extern __shared__ __align__(16) char smem[];
  LTable T{};
  size_t table_bytes = 0;
  if (!MULTI) {
    const SysDesc* d = reinterpret_cast<const SysDesc*>(a.blob);
    T = stage_table(a.blob, smem);
    table_bytes = align16(table_lds_bytes(d->n, d->T, d->TD));
  }
  const int jn = MULTI ? a.jn : reinterpret_cast<const SysDesc*>(a.blob)->n;
  // the wave's number within the workgroup, as a uniform (scalar) value
  const int wave_in_block = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  char* const wave_base = smem + table_bytes + (size_t)wave_in_block * wave_scratch_bytes<G>(jn, a.jrs);
  Scratch<G>* S = reinterpret_cast<Scratch<G>*>(wave_base + kWaveHeader);
  const JView J{reinterpret_cast<iv*>(wave_base + kWaveHeader + ((sizeof(Scratch<G>) + 15) / 16) * 16),
                jn * a.jrs + 1, a.jrs};
  __syncthreads();

  constexpr int W = 64 / G;
  const StepCounters sc{reinterpret_cast<unsigned long long*>(wave_base)};
  sc.clear();
  unsigned long long processed = 0, gen = 0;
  Stage stg;
  {
    const size_t wave = (size_t)blockIdx.x * (blockDim.x / 64) + (size_t)wave_in_block;
    stg.box = a.stage_box ? a.stage_box + wave * (size_t)(2 * W * G * 2) : nullptr;
    stg.meta = a.stage_meta ? a.stage_meta + wave * (size_t)(2 * W) : nullptr;
  }
  const int lane = __lane_id();
  Ctrl* c = a.ctrl;
  const unsigned long long nwaves = (unsigned long long)a.nblocks * (blockDim.x / 64);
  const unsigned long long wave_gid =
      (unsigned long long)blockIdx.x * (blockDim.x / 64) + (unsigned long long)wave_in_block;
  for (int level = a.level0;; ++level) {
    const unsigned long long cnt =
        __hip_atomic_load(&c->count[level % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int st = __hip_atomic_load(&c->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (st != 0 || cnt == 0 || (a.max_levels > 0 && level >= a.level0 + a.max_levels)) break;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (level < a.level_cap) a.level_sizes[level] = (long long)cnt;
      c->levels = (unsigned long long)(level + 1);
      if (cnt > c->max_frontier) c->max_frontier = cnt;
    }
    // the budget is on tree nodes: it fails exactly when the tree has more
    // than max_boxes nodes, whatever the frontier capacity (batches check it
    // per system inside the step)
    if (!MULTI && processed + cnt > (unsigned long long)a.max_boxes) {
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(&c->status, 0, -2);
      break;
    }
    if (cnt > (unsigned long long)a.front_cap) {
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicCAS(&c->status, 0, -4);
      break;
    }
    processed += cnt;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      __hip_atomic_store(&c->claim[(level + 1) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&c->count[(level + 2) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int cur = level & 1;
    unsigned long long* next_count = &c->count[(level + 1) % 3];
    // batches: a wave claims `pop` consecutive tiles per atomic.  A wave's
    // first claim of a level is static (the claim numbered by its global wave
    // index); later ones come from the level's counter, counted from the
    // first claim no wave holds.  A wave without a static claim touches no
    // counter, so a narrow level costs its few busy waves, not one atomic per
    // wave of the grid.
    const int pop = (MULTI && a.tiles_per_claim > 1) ? a.tiles_per_claim : 1;
    const unsigned long long claim_w = (unsigned long long)(W * pop);
    bool first = true;
    for (;;) {
      unsigned long long base = 0;
      if (first) {
        base = wave_gid * claim_w;
        first = false;
      } else {
        if (lane == 0) base = atomicAdd(&c->claim[level % 3], claim_w);
        base = __shfl(base, 0, 64) + nwaves * claim_w;
      }
      const bool more = base < cnt;
      if (MULTI) {
        if (!more) break;
        for (int t = 0; t < pop; ++t) {
          const unsigned long long tb = base + (unsigned long long)(t * W);
          if (tb >= cnt) break;
          step_tile<G, MULTI, false, false, VAR>(a, T, *S, J, (long long)tb, (long long)cnt, cur, level, next_count,
                                                 sc);
        }
        continue;
      }
      if (more) screen_tile<G, false>(a, T, *S, (long long)base, (long long)cnt, cur, sc, 0, false, nullptr, stg);
      // step the screened boxes W at a time; at the end of the level, all of them
      for (;;) {
        const unsigned long long avail = stg.tail - stg.head;
        if (avail == 0 || (more && avail < (unsigned long long)W)) break;
        step_tile<G, false, false, true, VAR>(a, T, *S, J, 0, 0, cur, level, next_count, sc, 0, false, nullptr,
                                              &stg);
        stg.head += avail < (unsigned long long)W ? avail : (unsigned long long)W;
      }
      if (!more) break;
    }
    grid_barrier(a, gen);
  }
  // the rounding mode held to the end (see fp64_round_field)
  if (fp64_round_field() != 2u && lane == 0) atomicCAS(&c->status, 0, kStatusModeLost);
  sc.flush(c->stats);
}

// ---------------------------------------------------------------------------
// Work-queue search of one system.  The boxes of the tree live in a ring of
// front_cap slots (front[0], meta[0]); every group of G lanes holds one claimed
// ring item, waits until the item's box has been published, and the wave
// steps the groups whose boxes are there.  Nothing waits for a level to end:
// the search tree, its counters and the sorted output are those of the level
// by level search (a box's children depend on the box alone), and the boxes
// per depth are the round sizes.  pending counts boxes created and not yet
// stepped; it reaches zero exactly when the search is over.  Every wait is
// bounded (IBB_ERR_TIMEOUT, IBB_ERR_QUEUE_OVERFLOW).
// ---------------------------------------------------------------------------
template <int G, bool VAR>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Occupancy<G, false>::waves)))
queue_kernel(SolveArgs a) {
  set_fp64_round_down();
  extern __shared__ __align__(16) char smem[];
  const SysDesc* d = reinterpret_cast<const SysDesc*>(a.blob);
  const LTable T = stage_table(a.blob, smem);
  const size_t table_bytes = align16(table_lds_bytes(d->n, d->T, d->TD));
  const int jn = d->n;
  // the wave's number within the workgroup, as a uniform (scalar) value
  const int wave_in_block = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  char* const wave_base = smem + table_bytes + (size_t)wave_in_block * wave_scratch_bytes<G>(jn, a.jrs);
  Scratch<G>* S = reinterpret_cast<Scratch<G>*>(wave_base + kWaveHeader);
  const JView J{reinterpret_cast<iv*>(wave_base + kWaveHeader + ((sizeof(Scratch<G>) + 15) / 16) * 16),
                jn * a.jrs + 1, a.jrs};
  __syncthreads();

  const StepCounters sc{reinterpret_cast<unsigned long long*>(wave_base)};
  sc.clear();
  const int lane = __lane_id();
  const int g = lane / G;
  const int r = lane % G;
  Ctrl* c = a.ctrl;
  const unsigned long long qmask = (unsigned long long)a.front_cap - 1ull;
  constexpr int W = 64 / G;
  long long slot = -1;  // this group's ring item (uniform over the group)
  QueueLocal ql;
  Stage stg;
  {
    const size_t wave = (size_t)blockIdx.x * (blockDim.x / 64) + (size_t)wave_in_block;
    stg.box = a.stage_box + wave * (size_t)(2 * W * G * 2);
    stg.meta = a.stage_meta + wave * (size_t)(2 * W);
  }
  for (;;) {
    // groups without an item claim the next ones, one atomic per wave
    const uint64_t needm = __ballot(slot < 0 && r == 0);
    unsigned long long base = 0;
    if (lane == 0 && needm) base = atomicAdd(&c->qhead, (unsigned long long)__popcll(needm));
    base = __shfl(base, 0, 64);
    if (slot < 0) {
      const uint64_t below = (g == 0) ? 0ull : (needm & ((1ull << (g * G)) - 1ull));
      slot = (long long)(base + (unsigned long long)__popcll(below));
    }
    // wait until some group's box is published, or the search is over
    bool full = false;
    bool stop = false;
    bool screen = false;  // false: nothing published yet, step what the stage holds
    const long long t0 = wall_clock64();
    for (;;) {
      unsigned long long v = 0;
      if (r == 0) v = __hip_atomic_load(&a.qseq[(unsigned long long)slot & qmask], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
      full = __shfl(v, g * G, 64) == (unsigned long long)slot + 1ull;
      if (__ballot(full) != 0) {
        screen = true;
        break;
      }
      if (stg.tail > stg.head) break;
      int st = 0;
      unsigned long long pend = 1;
      if (lane == 0) {
        st = __hip_atomic_load(&c->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pend = __hip_atomic_load(&c->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (st == 0 && pend != 0 && wall_clock64() - t0 > a.timeout_ticks) {
          atomicCAS(&c->status, 0, -8);
          st = -8;
        }
      }
      st = __shfl(st, 0, 64);
      pend = __shfl(pend, 0, 64);
      if (ql.pend != 0) {
        // idle: apply the wave's share first (the global count can reach
        // zero only once every wave has applied its share)
        if (lane == 0) atomicAdd(&c->pending, (unsigned long long)ql.pend);
        ql.pend = 0;
        continue;
      }
      if (st != 0 || pend == 0) {
        stop = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (stop) break;
    if (screen) {
      // the published boxes are read after this point, with coherent loads;
      // the wave has branched on the sequence words, and the compiler may not
      // move the record loads above them
      asm volatile("" ::: "memory");
      screen_tile<G, true>(a, T, *S, 0, 0, 0, sc, slot, full, &ql, stg);
      if (full) slot = -1;
    }
    // step the screened boxes W at a time, or all of them when none was new
    for (;;) {
      const unsigned long long avail = stg.tail - stg.head;
      if (avail == 0 || (screen && avail < (unsigned long long)W)) break;
      step_tile<G, false, true, true, VAR>(a, T, *S, J, 0, 0, 0, 0, nullptr, sc, 0, false, &ql, &stg);
      stg.head += avail < (unsigned long long)W ? avail : (unsigned long long)W;
    }
  }
  // the rounding mode held to the end (see fp64_round_field)
  if (fp64_round_field() != 2u && lane == 0) atomicCAS(&c->status, 0, kStatusModeLost);
  sc.flush(c->stats);
  if (lane == 0) {
    if (ql.run_count && ql.run_depth < (unsigned)a.level_cap)
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.level_sizes[ql.run_depth]), ql.run_count);
    if (ql.depth_max) atomicMax(&c->levels, (unsigned long long)ql.depth_max);
  }
}

// Fills count 64-bit words with v (a kernel rather than a memset, so that the
// fill can be recorded into a graph and replayed).
__global__ void fill_u64_kernel(unsigned long long* p, long long count, unsigned long long v) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

// Ring of a work-queue search: every slot free for its first item, except
// slot 0, which holds the initial box (written by init_kernel); no box stepped.
__global__ void queue_init_kernel(unsigned long long* seq, long long cap, Ctrl* c, long long* level_sizes,
                                  int level_cap) {
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = i0; i < cap; i += stride) seq[i] = (i == 0) ? 1ull : (unsigned long long)i;
  for (long long i = i0; i < level_cap; i += stride) level_sizes[i] = 0;
  if (i0 == 0) {
    c->qtail = 1ull;
    c->pending = 1ull;
  }
}

// ---------------------------------------------------------------------------
// Output: canonical (-0 -> +0) boxes sorted lexicographically by
// (lo_0..lo_{n-1}, hi_0..hi_{n-1}, tag).  Each element finds its rank by
// comparing with all others (ties broken by the original index).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cmp_boxes(const double* A, uint32_t ta, const double* B, uint32_t tb, int n) {
  for (int k = 0; k < n; ++k) {
    const double a = A[2 * k], b = B[2 * k];
    if (a < b) return -1;
    if (a > b) return 1;
  }
  for (int k = 0; k < n; ++k) {  // stored as -hi
    const double a = A[2 * k + 1], b = B[2 * k + 1];
    if (a > b) return -1;
    if (a < b) return 1;
  }
  return (ta < tb) ? -1 : (ta > tb ? 1 : 0);
}

__device__ __forceinline__ double canon(double x) { return x == 0.0 ? 0.0 : x; }

__global__ void sort_kernel(const double* box, const uint32_t* tag, const Ctrl* c, int n, int G,
                            long long out_cap, double* out_lo, double* out_hi, uint8_t* out_tag) {
  const unsigned long long total = c->out_count;
  if (c->status != 0 || total > (unsigned long long)out_cap) return;
  const long long m = (long long)total;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double* A = box + (size_t)i * G * 2;
  const uint32_t ta = tag[i];
  long long rank = 0;
  for (long long j = 0; j < m; ++j) {
    const int s = cmp_boxes(box + (size_t)j * G * 2, tag[j], A, ta, n);
    if (s < 0 || (s == 0 && j < i)) ++rank;
  }
  for (int k = 0; k < n; ++k) {
    out_lo[(size_t)rank * n + k] = canon(A[2 * k]);
    out_hi[(size_t)rank * n + k] = canon(-A[2 * k + 1]);
  }
  out_tag[rank] = (uint8_t)ta;
}

// d_info: status, box count, the eight tree counters, levels, widest level.
// With depth counts (work-queue search) the widest level is their maximum.
__global__ void finalize_kernel(const Ctrl* c, long long out_cap, long long* info, const long long* depth_counts,
                                int level_cap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int st = c->status;
  if (st == 0 && c->out_count > (unsigned long long)out_cap) st = -3;
  info[0] = st;
  info[1] = (long long)c->out_count;
  for (int i = 0; i < 8; ++i) info[2 + i] = (long long)c->stats[i];
  info[10] = (long long)c->levels;
  long long widest = (long long)c->max_frontier;
  if (depth_counts) {
    const long long m = (long long)c->levels < level_cap ? (long long)c->levels : level_cap;
    for (long long i = 0; i < m; ++i) widest = depth_counts[i] > widest ? depth_counts[i] : widest;
  }
  info[11] = widest;
}

// Initial state of a solve: control block, the root box at level 0.
__global__ void init_kernel(Ctrl* c, double* front0, uint32_t* meta0, const double* lo, const double* hi,
                            int n, int G) {
  const int t = threadIdx.x;
  for (int i = t; i < (int)(sizeof(Ctrl) / 8); i += blockDim.x) reinterpret_cast<unsigned long long*>(c)[i] = 0ull;
  if (t < G) {
    front0[2 * t] = t < n ? lo[t] : 0.0;
    front0[2 * t + 1] = t < n ? -hi[t] : 0.0;
  }
  if (t == 0) meta0[0] = 0u;
  __syncthreads();
  if (t == 0) c->count[0] = 1ull;
}

// Diagnostics: the device rounding primitives on operand arrays.
__global__ void selftest_kernel(int op, long long count, const double* x, const double* y, double* out) {
  set_fp64_round_down();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double a = x[i], b = y[i];
  double r = 0.0;
  switch (op) {
    case 0: r = radd(a, b); break;
    case 1: r = -radd(-a, -b); break;
    case 2: r = rsub(a, b); break;
    case 3: r = -rsub(-a, -b); break;
    case 4: r = rmul(a, b); break;
    case 5: r = -rmul_neg(a, b); break;
    case 6: r = rd_div(a, b); break;
    case 7: r = ru_div(a, b); break;
    case 8: r = (double)narrow_rn(a); break;
    case 9: r = imid(make_iv(a, b)); break;
    case 10: {
      const float fa = (float)a, fb = (float)b;
      const float p = fa * fb;
      r = (double)p;
      break;
    }
    case 11: {
      const float fa = (float)a, fb = (float)b;
      const float q = fa / fb;
      r = (double)q;
      break;
    }
    default: r = 0.0;
  }
  out[i] = r;
}

// ---------------------------------------------------------------------------
// Batches: level 0 of a bucket of systems, and the per-system sorted output.
// ---------------------------------------------------------------------------
__global__ void batch_init_kernel(Ctrl* c, double* front0, uint32_t* meta0, uint32_t* sys0, const double* lo,
                                  const double* hi, const int* bucket, int m, int G, const int* nsys,
                                  unsigned long long* count_sys, int B) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 8); i += blockDim.x)
      reinterpret_cast<unsigned long long*>(c)[i] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) c->count[0] = (unsigned long long)m;
  }
  if (t >= m) return;
  const int s = bucket[t];
  const int n = nsys[s];
  for (int r = 0; r < G; ++r) {
    front0[((size_t)t * G + r) * 2] = r < n ? lo[(size_t)s * kMaxN + r] : 0.0;
    front0[((size_t)t * G + r) * 2 + 1] = r < n ? -hi[(size_t)s * kMaxN + r] : 0.0;
  }
  meta0[t] = 0u;
  sys0[t] = (uint32_t)s;
  count_sys[s] = 1ull;
}

// Each emitted box takes a slot in its system's segment (order within the
// segment is fixed afterwards by the rank kernel).
__global__ void seg_scatter_kernel(const uint32_t* out_sys, long long M, const long long* seg_off,
                                   unsigned long long* cursor, uint32_t* order) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const uint32_t s = out_sys[i];
  const unsigned long long k = atomicAdd(&cursor[s], 1ull);
  order[seg_off[s] + (long long)k] = (uint32_t)i;
}

__global__ void seg_rank_kernel(const double* box, const uint32_t* tag, const uint32_t* out_sys,
                                const uint32_t* order, const long long* seg_off, const int* nsys, long long M,
                                double* out_lo, double* out_hi, uint8_t* out_tag) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const uint32_t i = order[j];
  const uint32_t s = out_sys[i];
  const int n = nsys[s];
  const long long a = seg_off[s], b = seg_off[s + 1];
  const double* A = box + (size_t)i * kMaxN * 2;
  const uint32_t ta = tag[i];
  long long rank = 0;
  for (long long k = a; k < b; ++k) {
    const uint32_t e = order[k];
    const int c = cmp_boxes(box + (size_t)e * kMaxN * 2, tag[e], A, ta, n);
    if (c < 0 || (c == 0 && e < i)) ++rank;
  }
  const long long dst = a + rank;
  for (int k = 0; k < kMaxN; ++k) {
    out_lo[(size_t)dst * kMaxN + k] = k < n ? canon(A[2 * k]) : 0.0;
    out_hi[(size_t)dst * kMaxN + k] = k < n ? canon(-A[2 * k + 1]) : 0.0;
  }
  out_tag[dst] = (uint8_t)ta;
}

// Serving: installs the requests admitted in one scheduling round (one
// workgroup each): the compiled system into its slot, the slot's parameters,
// counters and level bookkeeping, and the initial box at the end of its
// bucket's current level.
__global__ void admit_kernel(const AdmitRec* recs, const uint64_t* payload, uint64_t* blobs, int slot_words,
                             SysParams* sp, int* nsys, int* status_sys, uint8_t* evict,
                             unsigned long long* stats_sys, unsigned long long* slot_count,
                             unsigned long long* cum_sys, unsigned long long* pending, unsigned long long* count_sys,
                             int S) {
  const AdmitRec& a = recs[blockIdx.x];
  const int t = threadIdx.x;
  uint64_t* dst = blobs + (size_t)a.slot * slot_words;
  for (int i = t; i < a.nwords; i += blockDim.x) dst[i] = payload[a.blob_at + i];
  if (t < 8) stats_sys[(size_t)a.slot * 8 + t] = 0ull;
  if (t < 3) count_sys[(size_t)t * S + a.slot] = (t == a.level_slot) ? 1ull : 0ull;
  if (t < 2) cum_sys[(size_t)t * S + a.slot] = 0ull;
  if (t < a.G) {
    a.front[((size_t)a.pos * a.G + t) * 2] = t < a.n ? a.lo[t] : 0.0;
    a.front[((size_t)a.pos * a.G + t) * 2 + 1] = t < a.n ? -a.hi[t] : 0.0;
  }
  if (t == 0) {
    sp[a.slot] = a.sp;
    nsys[a.slot] = a.n;
    status_sys[a.slot] = 0;
    evict[a.slot] = 0;
    slot_count[a.slot] = 0ull;
    pending[a.slot] = 1ull;
    a.meta[a.pos] = 0u;
    a.sys[a.pos] = (uint32_t)a.slot;
    if (a.set_count) a.ctrl->count[a.level_slot] = a.new_count;
  }
}

// Serving: fails the given slots with `status`; the next pass drops their boxes.
__global__ void evict_kernel(const int* slots, int count, uint8_t* evict, int* status_sys, int status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  evict[slots[i]] = 1;
  status_sys[slots[i]] = status;
}

// Sorted output of one system's region (serving).
__global__ void slot_sort_kernel(const double* box, const uint32_t* tag, const unsigned long long* slot_count,
                                 int slot, int cap, int n, double* out_lo, double* out_hi, uint8_t* out_tag) {
  const long long m = (long long)min((unsigned long long)cap, slot_count[slot]);
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const size_t base = (size_t)slot * cap;
  const double* A = box + (base + i) * kMaxN * 2;
  const uint32_t ta = tag[base + i];
  long long rank = 0;
  for (long long j = 0; j < m; ++j) {
    const int c = cmp_boxes(box + (base + j) * kMaxN * 2, tag[base + j], A, ta, n);
    if (c < 0 || (c == 0 && j < i)) ++rank;
  }
  for (int k = 0; k < n; ++k) {
    out_lo[(size_t)rank * n + k] = canon(A[2 * k]);
    out_hi[(size_t)rank * n + k] = canon(-A[2 * k + 1]);
  }
  out_tag[rank] = (uint8_t)ta;
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (called by the runtime in api.cpp).
// ---------------------------------------------------------------------------
size_t scratch_bytes(int G, int jn, int rs) {
  switch (G) {
    case 2: return wave_scratch_bytes<2>(jn, rs);
    case 4: return wave_scratch_bytes<4>(jn, rs);
    case 8: return wave_scratch_bytes<8>(jn, rs);
    default: return wave_scratch_bytes<16>(jn, rs);
  }
}

// The search kernel of a lane count: batches (multi) always support every
// contractor and inclusion; one system gets the variant-free build unless
// its parameters ask for Krawczyk or the mean-value test (var).
const void* solve_kernel_ptr(int G, bool multi, bool var) {
  if (multi) {
    switch (G) {
      case 2: return reinterpret_cast<const void*>(&solve_kernel<2, true, true>);
      case 4: return reinterpret_cast<const void*>(&solve_kernel<4, true, true>);
      case 8: return reinterpret_cast<const void*>(&solve_kernel<8, true, true>);
      default: return reinterpret_cast<const void*>(&solve_kernel<16, true, true>);
    }
  }
  if (var) {
    switch (G) {
      case 2: return reinterpret_cast<const void*>(&solve_kernel<2, false, true>);
      case 4: return reinterpret_cast<const void*>(&solve_kernel<4, false, true>);
      case 8: return reinterpret_cast<const void*>(&solve_kernel<8, false, true>);
      default: return reinterpret_cast<const void*>(&solve_kernel<16, false, true>);
    }
  }
  switch (G) {
    case 2: return reinterpret_cast<const void*>(&solve_kernel<2, false, false>);
    case 4: return reinterpret_cast<const void*>(&solve_kernel<4, false, false>);
    case 8: return reinterpret_cast<const void*>(&solve_kernel<8, false, false>);
    default: return reinterpret_cast<const void*>(&solve_kernel<16, false, false>);
  }
}

hipError_t launch_init(hipStream_t s, Ctrl* c, double* front0, uint32_t* meta0, const double* lo,
                       const double* hi, int n, int G) {
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(64), 0, s, c, front0, meta0, lo, hi, n, G);
  return hipGetLastError();
}

hipError_t launch_sort(hipStream_t s, const double* box, const uint32_t* tag, const Ctrl* c, int n, int G,
                       long long out_cap, double* out_lo, double* out_hi, uint8_t* out_tag,
                       long long grid_elems) {
  const int blocks = (int)((grid_elems + 255) / 256);
  if (blocks > 0)
    hipLaunchKernelGGL(sort_kernel, dim3(blocks), dim3(256), 0, s, box, tag, c, n, G, out_cap, out_lo,
                       out_hi, out_tag);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, const Ctrl* c, long long out_cap, long long* info,
                           const long long* depth_counts, int level_cap) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, s, c, out_cap, info, depth_counts, level_cap);
  return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, long long count, unsigned long long v) {
  if (count <= 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

const void* queue_kernel_ptr(int G, bool var) {
  if (var) {
    switch (G) {
      case 2: return reinterpret_cast<const void*>(&queue_kernel<2, true>);
      case 4: return reinterpret_cast<const void*>(&queue_kernel<4, true>);
      case 8: return reinterpret_cast<const void*>(&queue_kernel<8, true>);
      default: return reinterpret_cast<const void*>(&queue_kernel<16, true>);
    }
  }
  switch (G) {
    case 2: return reinterpret_cast<const void*>(&queue_kernel<2, false>);
    case 4: return reinterpret_cast<const void*>(&queue_kernel<4, false>);
    case 8: return reinterpret_cast<const void*>(&queue_kernel<8, false>);
    default: return reinterpret_cast<const void*>(&queue_kernel<16, false>);
  }
}

hipError_t launch_queue_init(hipStream_t s, unsigned long long* seq, long long cap, Ctrl* c, long long* level_sizes,
                             int level_cap) {
  const long long work = cap > level_cap ? cap : level_cap;
  const int blocks = (int)std::min<long long>((work + 255) / 256, 4096);
  hipLaunchKernelGGL(queue_init_kernel, dim3(blocks), dim3(256), 0, s, seq, cap, c, level_sizes, level_cap);
  return hipGetLastError();
}

hipError_t launch_selftest(hipStream_t s, int op, long long count, const double* x, const double* y,
                           double* out) {
  const int blocks = (int)((count + 255) / 256);
  if (blocks > 0) hipLaunchKernelGGL(selftest_kernel, dim3(blocks), dim3(256), 0, s, op, count, x, y, out);
  return hipGetLastError();
}

}  // namespace ibb

namespace ibb {

hipError_t launch_prep(hipStream_t s, uint64_t* blobs, const long long* blob_off, int B) {
  if (B > 0) hipLaunchKernelGGL(prep_kernel, dim3(std::min(B, 4096)), dim3(256), 0, s, blobs, blob_off, B);
  return hipGetLastError();
}

hipError_t launch_batch_init(hipStream_t s, Ctrl* c, double* front0, uint32_t* meta0, uint32_t* sys0,
                             const double* lo, const double* hi, const int* bucket, int m, int G, const int* nsys,
                             unsigned long long* count_sys, int B) {
  const int blocks = std::max(1, (m + 255) / 256);
  hipLaunchKernelGGL(batch_init_kernel, dim3(blocks), dim3(256), 0, s, c, front0, meta0, sys0, lo, hi, bucket, m,
                     G, nsys, count_sys, B);
  return hipGetLastError();
}

hipError_t launch_seg_sort(hipStream_t s, const double* box, const uint32_t* tag, const uint32_t* out_sys,
                           long long M, const long long* seg_off, unsigned long long* cursor, uint32_t* order,
                           const int* nsys, double* out_lo, double* out_hi, uint8_t* out_tag) {
  const int blocks = (int)((M + 255) / 256);
  if (blocks > 0) {
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(blocks), dim3(256), 0, s, out_sys, M, seg_off, cursor, order);
    hipLaunchKernelGGL(seg_rank_kernel, dim3(blocks), dim3(256), 0, s, box, tag, out_sys, order, seg_off, nsys, M,
                       out_lo, out_hi, out_tag);
  }
  return hipGetLastError();
}

}  // namespace ibb

namespace ibb {

hipError_t launch_admit(hipStream_t s, const AdmitRec* recs, int count, const uint64_t* payload, uint64_t* blobs,
                        int slot_words, SysParams* sp, int* nsys, int* status_sys, uint8_t* evict,
                        unsigned long long* stats_sys, unsigned long long* slot_count, unsigned long long* cum_sys,
                        unsigned long long* pending, unsigned long long* count_sys, int S) {
  if (count > 0)
    hipLaunchKernelGGL(admit_kernel, dim3(count), dim3(256), 0, s, recs, payload, blobs, slot_words, sp, nsys,
                       status_sys, evict, stats_sys, slot_count, cum_sys, pending, count_sys, S);
  return hipGetLastError();
}

hipError_t launch_evict(hipStream_t s, const int* slots, int count, uint8_t* evict, int* status_sys, int status) {
  if (count > 0)
    hipLaunchKernelGGL(evict_kernel, dim3((count + 255) / 256), dim3(256), 0, s, slots, count, evict, status_sys,
                       status);
  return hipGetLastError();
}

hipError_t launch_slot_sort(hipStream_t s, const double* box, const uint32_t* tag,
                            const unsigned long long* slot_count, int slot, int cap, int n, double* out_lo,
                            double* out_hi, uint8_t* out_tag) {
  hipLaunchKernelGGL(slot_sort_kernel, dim3((cap + 255) / 256), dim3(256), 0, s, box, tag, slot_count, slot, cap,
                     n, out_lo, out_hi, out_tag);
  return hipGetLastError();
}

}  // namespace ibb

// ---------------------------------------------------------------------------
// Workspace of the allocation-free solve (ibb_solve_noalloc): one array per
// device, held from the first use of the library on that device until the
// process ends.  Host code never uses the array's name as an address (on the
// host it names a stand-in, not device memory); it uses the address that
// hipGetSymbolAddress returns on each device, looked up once per device.
// ---------------------------------------------------------------------------
namespace ibb {

static __device__ __align__(256) unsigned char scratch[IBB_NOALLOC_WORKSPACE_BYTES];

// The device address of `scratch` on `device`, which must be the current
// device; hipSuccess or the lookup's error.
hipError_t noalloc_scratch(int device, void** ptr) {
  constexpr int kDevices = 64;
  static std::mutex mu;
  static void* addr[kDevices] = {};
  if (device < 0 || device >= kDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

}  // namespace ibb
