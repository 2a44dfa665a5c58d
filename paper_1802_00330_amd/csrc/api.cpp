// api.cpp -- host runtime behind include/ibb.h: validation, system compilation,
// device memory, launches and result collection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <array>
#include <map>
#include <tuple>
#include <new>
#include <limits>
#include <vector>

#include "../../include/ibb.h"
#include "layout.hpp"

namespace ibb {
// kernels.hip
size_t scratch_bytes(int G, int jn, int rs);
const void* solve_kernel_ptr(int G, bool multi, bool var);
hipError_t launch_prep(hipStream_t s, uint64_t* blobs, const long long* blob_off, int B);
hipError_t launch_batch_init(hipStream_t s, Ctrl* c, double* front0, uint32_t* meta0, uint32_t* sys0,
                             const double* lo, const double* hi, const int* bucket, int m, int G, const int* nsys,
                             unsigned long long* count_sys, int B);
hipError_t launch_slot_sort(hipStream_t s, const double* box, const uint32_t* tag,
                            const unsigned long long* slot_count, int slot, int cap, int n, double* out_lo,
                            double* out_hi, uint8_t* out_tag);
hipError_t launch_seg_sort(hipStream_t s, const double* box, const uint32_t* tag, const uint32_t* out_sys,
                           long long M, const long long* seg_off, unsigned long long* cursor, uint32_t* order,
                           const int* nsys, double* out_lo, double* out_hi, uint8_t* out_tag);
hipError_t launch_init(hipStream_t s, Ctrl* c, double* front0, uint32_t* meta0, const double* lo,
                       const double* hi, int n, int G);
hipError_t launch_sort(hipStream_t s, const double* box, const uint32_t* tag, const Ctrl* c, int n, int G,
                       long long out_cap, double* out_lo, double* out_hi, uint8_t* out_tag,
                       long long grid_elems);
hipError_t launch_finalize(hipStream_t s, const Ctrl* c, long long out_cap, long long* info,
                           const long long* depth_counts, int level_cap);
const void* queue_kernel_ptr(int G, bool var);
hipError_t launch_queue_init(hipStream_t s, unsigned long long* seq, long long cap, Ctrl* c, long long* level_sizes,
                             int level_cap);
hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, long long count, unsigned long long v);
hipError_t launch_selftest(hipStream_t s, int op, long long count, const double* x, const double* y,
                           double* out);
hipError_t noalloc_scratch(int device, void** ptr);
}  // namespace ibb

using namespace ibb;

namespace {

constexpr long long kLevelCap = 1 << 16;

int lanes_for(int n) {
  if (n <= 2) return 2;
  if (n <= 4) return 4;
  if (n <= 8) return 8;
  return 16;
}

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Lane-count class of a power of two 2..16: 0..3.
int lanes_class(int G) { return G == 2 ? 0 : G == 4 ? 1 : G == 8 ? 2 : 3; }

// ---------------------------------------------------------------------------
// Validation and compilation of a system into the device blob (layout.hpp).
// ---------------------------------------------------------------------------
int validate(const ibb_system* s, const double* lo, const double* hi, const ibb_params* p) {
  if (!s || !lo || !hi || !p || !s->term_off || !s->expo || !s->coef) return IBB_ERR_INVALID_ARG;
  const int n = s->n;
  if (n < 1 || n > IBB_MAX_N) return IBB_ERR_INVALID_ARG;
  if (s->term_off[0] != 0) return IBB_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    if (s->term_off[i + 1] <= s->term_off[i]) return IBB_ERR_INVALID_ARG;
  const int T = s->term_off[n];
  const double big = std::ldexp(1.0, 40);
  for (int t = 0; t < T; ++t) {
    if (!std::isfinite(s->coef[t]) || std::fabs(s->coef[t]) > big) return IBB_ERR_INVALID_ARG;
    int deg = 0;
    for (int k = 0; k < n; ++k) deg += s->expo[(size_t)t * n + k];
    if (deg > IBB_MAX_DEG) return IBB_ERR_INVALID_ARG;
  }
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || lo[k] > hi[k] || std::fabs(lo[k]) > big ||
        std::fabs(hi[k]) > big)
      return IBB_ERR_INVALID_ARG;
  if (!(p->tol > 0) || !std::isfinite(p->tol)) return IBB_ERR_INVALID_ARG;
  if (p->max_boxes < 1) return IBB_ERR_INVALID_ARG;
  if (p->split_mode != IBB_SPLIT_WIDEST && p->split_mode != IBB_SPLIT_ALL) return IBB_ERR_INVALID_ARG;
  if (p->max_recontract < 1) return IBB_ERR_INVALID_ARG;
  if (!(p->recontract_ratio >= 0) || !(p->recontract_ratio <= 1)) return IBB_ERR_INVALID_ARG;
  if (std::isnan(p->hs_max_width)) return IBB_ERR_INVALID_ARG;
  if (p->schedule != IBB_SCHEDULE_QUEUE && p->schedule != IBB_SCHEDULE_LEVELS && p->schedule != IBB_SCHEDULE_AUTO)
    return IBB_ERR_INVALID_ARG;
  if (p->contractor != IBB_CONTRACT_HS && p->contractor != IBB_CONTRACT_KRAWCZYK) return IBB_ERR_INVALID_ARG;
  if (p->inclusion != IBB_INCLUDE_NATURAL && p->inclusion != IBB_INCLUDE_MEAN_VALUE) return IBB_ERR_INVALID_ARG;
  if (p->reserved != 0) return IBB_ERR_INVALID_ARG;
  if (T > IBB_MAX_TERMS) return IBB_ERR_UNSUPPORTED;
  if (p->max_recontract > 255) return IBB_ERR_UNSUPPORTED;
  return IBB_OK;
}

uint64_t pack_factors(const uint8_t* e, int n) {
  uint64_t f = 0;
  int q = 0;
  for (int k = 0; k < n; ++k)
    if (e[k]) f |= (uint64_t)((e[k] << 4) | k) << (8 * q++);
  return f;
}

struct Compiled {
  int n = 0, G = 0, T = 0, TD = 0;
  std::vector<uint64_t> blob;
};

void compile(const ibb_system* s, Compiled& c) {
  const int n = s->n, T = s->term_off[n];
  std::vector<int32_t> eq_off(s->term_off, s->term_off + n + 1);
  std::vector<double> coef(s->coef, s->coef + T);
  std::vector<uint64_t> fac(T);
  for (int t = 0; t < T; ++t) fac[t] = pack_factors(s->expo + (size_t)t * n, n);
  std::vector<int32_t> der_off(n * n + 1, 0);
  std::vector<double> dcoef;
  std::vector<uint32_t> dmult;
  std::vector<uint64_t> dfac;
  uint32_t jnz[kMaxN] = {0};
  uint8_t e[kMaxN];
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      der_off[i * n + k] = (int32_t)dcoef.size();
      for (int t = s->term_off[i]; t < s->term_off[i + 1]; ++t) {
        const uint8_t* a = s->expo + (size_t)t * n;
        if (a[k] == 0) continue;
        std::memcpy(e, a, n);
        e[k] = (uint8_t)(a[k] - 1);
        dcoef.push_back(s->coef[t]);
        dmult.push_back(a[k]);
        dfac.push_back(pack_factors(e, n));
        jnz[i] |= 1u << k;
      }
    }
  der_off[n * n] = (int32_t)dcoef.size();
  const int TD = (int)dcoef.size();

  SysDesc d;
  std::memset(&d, 0, sizeof d);
  d.n = n;
  d.G = lanes_for(n);
  d.T = T;
  d.TD = TD;
  int w = (int)(sizeof(SysDesc) / 8);
  auto words = [](size_t bytes) { return (int)((bytes + 7) / 8); };
  d.eq_off_w = w;
  w += words(sizeof(int32_t) * (n + 1));
  d.der_off_w = w;
  w += words(sizeof(int32_t) * (n * n + 1));
  d.coef_w = w;
  w += T;
  d.fac_w = w;
  w += T;
  d.dcoef_w = w;
  w += TD;
  d.dmult_w = w;
  w += words(sizeof(uint32_t) * TD);
  d.dfac_w = w;
  w += TD;
  d.dco_w = w;
  w += 2 * TD;
  d.total_w = w;
  std::memcpy(d.jnz, jnz, sizeof jnz);

  c.n = n;
  c.G = d.G;
  c.T = T;
  c.TD = TD;
  c.blob.assign((size_t)w, 0);
  char* base = reinterpret_cast<char*>(c.blob.data());
  std::memcpy(base, &d, sizeof d);
  std::memcpy(base + 8 * (size_t)d.eq_off_w, eq_off.data(), sizeof(int32_t) * (n + 1));
  std::memcpy(base + 8 * (size_t)d.der_off_w, der_off.data(), sizeof(int32_t) * (n * n + 1));
  if (T) std::memcpy(base + 8 * (size_t)d.coef_w, coef.data(), sizeof(double) * T);
  if (T) std::memcpy(base + 8 * (size_t)d.fac_w, fac.data(), sizeof(uint64_t) * T);
  if (TD) std::memcpy(base + 8 * (size_t)d.dcoef_w, dcoef.data(), sizeof(double) * TD);
  if (TD) std::memcpy(base + 8 * (size_t)d.dmult_w, dmult.data(), sizeof(uint32_t) * TD);
  if (TD) std::memcpy(base + 8 * (size_t)d.dfac_w, dfac.data(), sizeof(uint64_t) * TD);
}

// Device workspace partition of one solve.
struct WsLayout {
  size_t ctrl, level, blob, box, front0, front1, meta0, meta1, out_box, out_tag, seq, stage_box, stage_meta, total;
};

WsLayout ws_layout(int n, size_t blob_words, long long frontier_cap, long long out_cap) {
  const int G = lanes_for(n);
  WsLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  L.ctrl = take(sizeof(Ctrl));
  L.level = take(sizeof(long long) * kLevelCap);
  L.blob = take(8 * blob_words);
  L.box = take(sizeof(double) * 2 * kMaxN);
  L.front0 = take(sizeof(double) * 2 * G * (size_t)frontier_cap);
  L.front1 = take(sizeof(double) * 2 * G * (size_t)frontier_cap);
  L.meta0 = take(sizeof(uint32_t) * (size_t)frontier_cap);
  L.meta1 = take(sizeof(uint32_t) * (size_t)frontier_cap);
  L.out_box = take(sizeof(double) * 2 * G * (size_t)out_cap);
  L.out_tag = take(sizeof(uint32_t) * (size_t)out_cap);
  L.seq = take(sizeof(unsigned long long) * (size_t)frontier_cap);
  L.stage_box = take(sizeof(double) * 2 * 128 * (size_t)kStageWaves);  // 2W * G = 128 rows per wave
  L.stage_meta = take(sizeof(uint32_t) * 64 * (size_t)kStageWaves);     // 2W <= 64 records per wave
  L.total = o;
  return L;
}

// Ring capacity of a work-queue search: the largest power of two that fits
// the level-0 frontier buffer.
long long ring_capacity(long long frontier_cap) {
  long long c = 1;
  while (c * 2 <= frontier_cap) c *= 2;
  return c;
}

// Upper bound of the system blob size for a given n (IBB_MAX_TERMS terms).
size_t max_blob_words(int n) {
  const size_t T = IBB_MAX_TERMS, TD = (size_t)IBB_MAX_TERMS * IBB_MAX_DEG;
  return sizeof(SysDesc) / 8 + (n + 2) / 2 + (n * n + 2) / 2 + 2 * T + 4 * TD + (TD + 1) / 2 + 8;
}

}  // namespace

struct ibb_ctx {
  int device = 0;
  int num_cu = 0;
  size_t max_lds_block = 0;
  size_t lds_per_cu = 0;
  long long clock_khz = 100000;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, staged = nullptr;
  hipEvent_t done = nullptr;  // end of the last single-system solve (after its d_info)
  bool staged_pending = false;
  bool timed_pending = false;  // ev0/ev1 bracket the last persistent launch
  void* ws = nullptr;  // workspace of the host-pointer entry points
  size_t ws_bytes = 0;
  double* sorted = nullptr;  // sorted outputs of ibb_solve (lo, hi, tag)
  size_t sorted_bytes = 0;
  long long* info = nullptr;
  char* pinned = nullptr;  // host staging of the inputs
  size_t pinned_bytes = 0;
  void* noalloc_ws = nullptr;  // device address of the allocation-free workspace
  std::vector<long long> last_levels;
  void* bws = nullptr;  // batch workspace
  size_t bws_bytes = 0;
  long long batch_fcap = 0;  // frontier capacity the last batch needed
  long long batch_mem = 0;   // bound on the batch workspace in bytes (0: free device memory)
  // launch configuration of each lane-count class of batch members
  ibb_batch_config batch_cfg[4] = {{2, 1, 0, 0, 0.0}, {4, 1, 0, 0, 0.0}, {8, 1, 0, 0, 0.0}, {16, 1, 0, 0, 0.0}};
  // schedule autotuner: best kernel time per (n, T, TD, split mode) and
  // schedule, and the shape / schedule of the launch ev0..ev1 last bracketed
  // per shape: the fastest time of each schedule and how many launches it timed
  struct TuneEntry {
    float ms[2] = {-1.0f, -1.0f};
    int n[2] = {0, 0};
  };
  std::map<std::tuple<int, int, int, int>, TuneEntry> tune;
  bool tune_pending = false;
  std::tuple<int, int, int, int> tune_key;
  int tune_sched = 0;
  const long long* tune_info = nullptr;  // d_info of that launch (its status)
};

namespace {

int ensure_device(void** p, size_t* cur, size_t need) {
  if (*cur >= need) return IBB_OK;
  if (*p) hipFree(*p);
  *p = nullptr;
  *cur = 0;
  if (hipMalloc(p, need) != hipSuccess) {
    *p = nullptr;
    return IBB_ERR_NO_MEMORY;
  }
  *cur = need;
  return IBB_OK;
}

int ensure_pinned(ibb_ctx* ctx, size_t need) {
  if (ctx->staged_pending) {
    hipEventSynchronize(ctx->staged);
    ctx->staged_pending = false;
  }
  if (ctx->pinned_bytes >= need) return IBB_OK;
  if (ctx->pinned) hipHostFree(ctx->pinned);
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  if (hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), need, hipHostMallocDefault) != hipSuccess) {
    ctx->pinned = nullptr;
    return IBB_ERR_NO_MEMORY;
  }
  ctx->pinned_bytes = need;
  return IBB_OK;
}

// Workgroups of a persistent launch that are resident on one CU at once.
// The occupancy query alone over-promises near the LDS limit.  Measured on
// gfx950 (a probe that launches k workgroups per CU with L bytes of LDS each
// and waits, bounded, until all are present; L swept in 256-byte steps for
// k = 2..6): all k were resident exactly while k * ceil(L / 1280) <= 128,
// i.e. the CU's 160 KiB of LDS is allocated in 128 granules of 1280 bytes
// (largest resident L: 81,920 / 53,589 / 40,960 / 32,000 / 26,794 bytes for
// k = 2..6; smallest not resident: 82,176 / 53,845 / 41,216 / 32,256 /
// 27,050).
int resident_per_cu(ibb_ctx* ctx, const void* fn, int threads, size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) return 0;
  const size_t granules = 128, granule = ctx->lds_per_cu / granules;
  if (lds > 0 && granule > 0) {
    const size_t need = (lds + granule - 1) / granule;
    per_cu = std::min<int>(per_cu, (int)(granules / need));
  }
  return per_cu;
}

// Launch geometry of a persistent kernel: waves per block, LDS, grid and the
// row stride of the Jacobian scratch.  jn is the Jacobian dimension the
// kernel sizes its scratch for (n for one system, the largest member n for a
// batch).  Every block holds its own copy of the table, so the choice is the
// (row stride, waves per block) pair with the most resident waves per CU; on
// a tie, the padded row stride and then the larger block.
struct Geometry {
  int waves = 0, blocks = 0, jrs = 0;
  size_t lds = 0;
};

int persistent_geometry(ibb_ctx* ctx, const void* fn, size_t table_bytes, int G, int jn, Geometry* out) {
  Geometry best;
  int best_per_cu = 0;
  for (int rs : {jn + 1, jn}) {
    const size_t per_wave = scratch_bytes(G, jn, rs);
    for (int waves = 4; waves >= 1; --waves) {
      const size_t lds = table_bytes + per_wave * waves;
      if (lds > ctx->max_lds_block) continue;
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return IBB_ERR_DEVICE;
      const int per_cu = resident_per_cu(ctx, fn, 64 * waves, lds);
      if (per_cu * waves > best_per_cu * best.waves) {
        best_per_cu = per_cu;
        best.waves = waves;
        best.lds = lds;
        best.jrs = rs;
      }
    }
  }
  if (best_per_cu < 1) return IBB_ERR_UNSUPPORTED;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)best.lds) != hipSuccess)
    return IBB_ERR_DEVICE;
  best.blocks = best_per_cu * ctx->num_cu;
  *out = best;
  return IBB_OK;
}

// The persistent search launch of one system over a partitioned workspace
// whose control block and level-0 frontier are already in place.
int launch_search(ibb_ctx* ctx, const Compiled& c, const ibb_params* p, char* ws, const WsLayout& L,
                  long long frontier_cap, long long out_cap, long long max_boxes, hipStream_t s, int max_levels,
                  double* d_dbg, bool queue = false) {
  const int n = c.n, G = c.G;
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  SolveArgs a;
  std::memset(&a, 0, sizeof a);
  a.blob = reinterpret_cast<const uint64_t*>(ws + L.blob);
  a.front[0] = reinterpret_cast<double*>(ws + L.front0);
  a.front[1] = reinterpret_cast<double*>(ws + L.front1);
  a.meta[0] = reinterpret_cast<uint32_t*>(ws + L.meta0);
  a.meta[1] = reinterpret_cast<uint32_t*>(ws + L.meta1);
  a.front_cap = frontier_cap;
  a.out_box = reinterpret_cast<double*>(ws + L.out_box);
  a.out_tag = reinterpret_cast<uint32_t*>(ws + L.out_tag);
  a.out_cap = out_cap;
  a.ctrl = ctrl;
  a.level_sizes = reinterpret_cast<long long*>(ws + L.level);
  a.level_cap = kLevelCap;
  a.tol = p->tol;
  a.ratio = p->recontract_ratio;
  a.hs_max_width = p->hs_max_width;
  a.max_boxes = max_boxes;
  a.split_mode = p->split_mode;
  a.max_rc = p->max_recontract;
  a.contractor = p->contractor;
  a.inclusion = p->inclusion;
  a.timeout_ticks = ctx->clock_khz * 1000LL * 20;  // 20 s per barrier wait
  a.max_levels = max_levels;
  a.dbg = d_dbg;
  a.out_count = &ctrl->out_count;
  a.out_stride = G;
  if (queue) {
    a.front_cap = ring_capacity(frontier_cap);
    a.qseq = reinterpret_cast<unsigned long long*>(ws + L.seq);
  }
  a.stage_box = reinterpret_cast<double*>(ws + L.stage_box);
  a.stage_meta = reinterpret_cast<uint32_t*>(ws + L.stage_meta);

  const bool var = p->contractor != IBB_CONTRACT_HS || p->inclusion != IBB_INCLUDE_NATURAL;
  const void* fn = queue ? queue_kernel_ptr(G, var) : solve_kernel_ptr(G, false, var);
  const size_t tbytes = (table_lds_bytes(n, c.T, c.TD) + 15) & ~size_t(15);
  Geometry geo;
  {
    const int gst = persistent_geometry(ctx, fn, tbytes, G, n, &geo);
    if (gst) return gst;
    if ((long long)geo.blocks * geo.waves > kStageWaves) return IBB_ERR_UNSUPPORTED;
  }
  a.nblocks = geo.blocks;
  a.jrs = geo.jrs;
  a.jn = n;
  void* args[] = {&a};
  ctx->tune_pending = false;  // ev0 / ev1 now bracket this launch
  hipEventRecord(ctx->ev0, s);
  if (hipLaunchCooperativeKernel(fn, dim3(geo.blocks), dim3(64 * geo.waves), args, (unsigned)geo.lds, s) !=
      hipSuccess)
    return IBB_ERR_DEVICE;
  hipEventRecord(ctx->ev1, s);
  ctx->timed_pending = true;
  return IBB_OK;
}

// Schedule of a full solve.  With IBB_SCHEDULE_AUTO, the kernel time of the
// previous single-system launch is first credited to its shape and schedule;
// a shape with fewer than kTuneSamples timed launches of a schedule gets that
// schedule (the first launch on fresh device memory is slower than the
// following ones, so one sample each can pick the slower schedule), then the
// faster of the two.
constexpr int kTuneSamples = 2;

int resolve_schedule(ibb_ctx* ctx, const Compiled& c, const ibb_params* p) {
  if (ctx->tune_pending) {
    auto it = ctx->tune.find(ctx->tune_key);
    const bool learning =
        it != ctx->tune.end() && (it->second.n[0] < kTuneSamples || it->second.n[1] < kTuneSamples);
    long long status = 0;
    if (learning) {
      hipEventSynchronize(ctx->done);
      // a launch that stopped early (capacity, budget) says nothing about speed
      if (ctx->tune_info) hipMemcpy(&status, ctx->tune_info, sizeof status, hipMemcpyDeviceToHost);
    }
    if (status == 0 && hipEventQuery(ctx->ev1) == hipSuccess) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) == hipSuccess && it != ctx->tune.end()) {
        float& slot = it->second.ms[ctx->tune_sched];
        slot = slot < 0 ? ms : std::min(slot, ms);
        ++it->second.n[ctx->tune_sched];
      }
    }
    ctx->tune_pending = false;
  }
  // shape key: size, terms, derivative terms, and the split, contractor and inclusion (their kernels differ)
  const auto key = std::make_tuple(c.n, c.T, c.TD, p->split_mode | (p->contractor << 2) | (p->inclusion << 3));
  auto it = ctx->tune.find(key);
  if (it == ctx->tune.end()) it = ctx->tune.emplace(key, ibb_ctx::TuneEntry{}).first;
  int sched = p->schedule;
  if (sched == IBB_SCHEDULE_AUTO) {
    const auto& e = it->second;
    if (e.n[0] < kTuneSamples) sched = IBB_SCHEDULE_QUEUE;
    else if (e.n[1] < kTuneSamples) sched = IBB_SCHEDULE_LEVELS;
    else sched = e.ms[1] < e.ms[0] ? IBB_SCHEDULE_LEVELS : IBB_SCHEDULE_QUEUE;
  }
  // credited when the next solve is enqueued (see above)
  ctx->tune_key = key;
  ctx->tune_sched = sched;
  return sched;
}

// Enqueue one solve into a partitioned workspace; outputs to device arrays.
int enqueue_solve(ibb_ctx* ctx, const Compiled& c, const double* lo, const double* hi,
                  const ibb_params* p, char* ws, const WsLayout& L, long long frontier_cap,
                  long long out_cap, double* d_out_lo, double* d_out_hi, uint8_t* d_out_tag,
                  long long* d_info, hipStream_t s, int max_levels = 0, double* d_dbg = nullptr) {
  const int n = c.n, G = c.G;
  // stage the host inputs: blob, lo, hi
  const size_t blob_bytes = 8 * c.blob.size();
  int st = ensure_pinned(ctx, blob_bytes + 2 * sizeof(double) * kMaxN);
  if (st) return st;
  std::memcpy(ctx->pinned, c.blob.data(), blob_bytes);
  double* plo = reinterpret_cast<double*>(ctx->pinned + blob_bytes);
  double* phi = plo + kMaxN;
  std::memcpy(plo, lo, sizeof(double) * n);
  std::memcpy(phi, hi, sizeof(double) * n);
  if (hipMemcpyAsync(ws + L.blob, ctx->pinned, blob_bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(ws + L.box, plo, 2 * sizeof(double) * kMaxN, hipMemcpyHostToDevice, s) != hipSuccess)
    return IBB_ERR_DEVICE;
  hipEventRecord(ctx->staged, s);
  ctx->staged_pending = true;

  if (launch_prep(s, reinterpret_cast<uint64_t*>(ws + L.blob), nullptr, 1) != hipSuccess) return IBB_ERR_DEVICE;
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  const double* dlo = reinterpret_cast<const double*>(ws + L.box);
  if (launch_init(s, ctrl, reinterpret_cast<double*>(ws + L.front0), reinterpret_cast<uint32_t*>(ws + L.meta0),
                  dlo, dlo + kMaxN, n, G) != hipSuccess)
    return IBB_ERR_DEVICE;

  // full solves run as a work queue; single levels (diagnostics) level by level
  const bool full_solve = max_levels == 0 && d_dbg == nullptr;
  const bool queue = full_solve && resolve_schedule(ctx, c, p) == IBB_SCHEDULE_QUEUE;
  long long* depth_counts = reinterpret_cast<long long*>(ws + L.level);
  if (queue && launch_queue_init(s, reinterpret_cast<unsigned long long*>(ws + L.seq), ring_capacity(frontier_cap),
                                 ctrl, depth_counts, kLevelCap) != hipSuccess)
    return IBB_ERR_DEVICE;
  {
    const int lst =
        launch_search(ctx, c, p, ws, L, frontier_cap, out_cap, p->max_boxes, s, max_levels, d_dbg, queue);
    if (lst) return lst;
    ctx->tune_pending = full_solve;
    ctx->tune_info = d_info;
  }
  if (launch_sort(s, reinterpret_cast<const double*>(ws + L.out_box), reinterpret_cast<const uint32_t*>(ws + L.out_tag),
                  ctrl, n, G, out_cap, d_out_lo, d_out_hi, d_out_tag, out_cap) != hipSuccess)
    return IBB_ERR_DEVICE;
  if (launch_finalize(s, ctrl, out_cap, d_info, queue ? depth_counts : nullptr, kLevelCap) != hipSuccess)
    return IBB_ERR_DEVICE;
  hipEventRecord(ctx->done, s);
  return IBB_OK;
}

void fill_stats(ibb_stats* st, const long long* info, double ms) {
  if (!st) return;
  st->processed = info[2];
  st->excluded_eval = info[3];
  st->excluded_hs = info[4];
  st->hs_skipped = info[5];
  st->recontracted = info[6];
  st->bisected = info[7];
  st->emitted_unique = info[8];
  st->emitted_undecided = info[9];
  st->levels = info[10];
  st->max_frontier = info[11];
  st->kernel_ms = ms;
}

}  // namespace


// ---------------------------------------------------------------------------
// Batches: many systems per launch.  Systems are bucketed by lanes per box
// (2, 4, 8, 16); each bucket is one persistent launch over a frontier whose
// records carry their system index; tables are read from global memory.
// ---------------------------------------------------------------------------
namespace {

struct BatchLayout {
  size_t blobs, boff, sp, nsys, lo, hi, count_sys, cum_sys, status_sys, stats_sys, bucket, ctrl, level, front0,
      front1, meta0, meta1, sys0, sys1, out_box, out_tag, out_sys, out_count, seg_off, cursor, order, s_lo, s_hi,
      s_tag, total;
};

BatchLayout batch_layout(int B, size_t blob_words, long long fcap, long long ocap) {
  BatchLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  L.blobs = take(8 * blob_words);
  L.boff = take(sizeof(long long) * B);
  L.sp = take(sizeof(SysParams) * B);
  L.nsys = take(sizeof(int) * B);
  L.lo = take(sizeof(double) * kMaxN * B);
  L.hi = take(sizeof(double) * kMaxN * B);
  L.bucket = take(sizeof(int) * B);
  L.count_sys = take(sizeof(unsigned long long) * 3 * B);  // zeroed together: count_sys .. stats_sys
  L.cum_sys = take(sizeof(unsigned long long) * 2 * B);
  L.status_sys = take(sizeof(int) * B);
  L.stats_sys = take(sizeof(unsigned long long) * 8 * B);
  L.ctrl = take(sizeof(Ctrl) * 4);
  L.level = take(sizeof(long long) * kLevelCap);
  L.front0 = take(sizeof(double) * 2 * kMaxN * (size_t)fcap);
  L.front1 = take(sizeof(double) * 2 * kMaxN * (size_t)fcap);
  L.meta0 = take(sizeof(uint32_t) * (size_t)fcap);
  L.meta1 = take(sizeof(uint32_t) * (size_t)fcap);
  L.sys0 = take(sizeof(uint32_t) * (size_t)fcap);
  L.sys1 = take(sizeof(uint32_t) * (size_t)fcap);
  L.out_box = take(sizeof(double) * 2 * kMaxN * (size_t)ocap);
  L.out_tag = take(sizeof(uint32_t) * (size_t)ocap);
  L.out_sys = take(sizeof(uint32_t) * (size_t)ocap);
  L.out_count = take(sizeof(unsigned long long));
  L.seg_off = take(sizeof(long long) * (B + 1));
  L.cursor = take(sizeof(unsigned long long) * B);
  L.order = take(sizeof(uint32_t) * (size_t)ocap);
  L.s_lo = take(sizeof(double) * kMaxN * (size_t)ocap);
  L.s_hi = take(sizeof(double) * kMaxN * (size_t)ocap);
  L.s_tag = take((size_t)ocap);
  L.total = o;
  return L;
}

}  // namespace

namespace {

// Host side of a batch: every member validated and compiled, tables packed into
// one blob, members grouped by lanes per box.
struct BatchHost {
  int B = 0;
  size_t words = 0;
  std::vector<long long> boff;
  std::vector<int> nsys;
  std::vector<SysParams> sp;
  std::vector<uint64_t> blob;
  std::vector<double> lo16, hi16;
  std::vector<int> bucket_list;
  int bucket_start[5] = {0, 0, 0, 0, 0};
  int bucket_jn[4] = {0, 0, 0, 0};  // largest member n per bucket
  int bucket_pop[4] = {1, 1, 1, 1};     // tiles per claim
  int bucket_per_cu[4] = {0, 0, 0, 0};  // resident workgroups per CU (0 = all that fit)
  bool any = false;
};

int batch_prepare(int B, const ibb_system* systems, const double* lo, const double* hi, const ibb_params* params,
                  const ibb_batch_config* cfg, int32_t* status, BatchHost& h) {
  h.B = B;
  std::vector<Compiled> comp((size_t)B);
  h.boff.assign((size_t)B, 0);
  h.nsys.assign((size_t)B, 1);
  h.sp.assign((size_t)B, SysParams{});
  std::vector<int> buckets[4];
  long long first_valid = -1;
  h.words = 0;
  for (int b = 0; b < B; ++b) {
    status[b] = validate(&systems[b], lo + (size_t)b * kMaxN, hi + (size_t)b * kMaxN, &params[b]);
    if (status[b] != IBB_OK) continue;
    try {
      compile(&systems[b], comp[b]);
    } catch (...) {
      return IBB_ERR_NO_MEMORY;
    }
    h.boff[b] = (long long)h.words;
    if (first_valid < 0) first_valid = (long long)h.words;
    h.words += comp[b].blob.size();
    h.nsys[b] = comp[b].n;
    const ibb_params& p = params[b];
    h.sp[b] = SysParams{p.tol, p.recontract_ratio, p.hs_max_width, p.max_boxes, p.split_mode, p.max_recontract,
                         p.contractor, p.inclusion};
    // the member runs with the lane count its class is configured for
    buckets[lanes_class(cfg[lanes_class(comp[b].G)].lanes)].push_back(b);
  }
  h.any = first_valid >= 0;
  if (!h.any) return IBB_OK;
  for (int b = 0; b < B; ++b)
    if (status[b] != IBB_OK) h.boff[b] = first_valid;  // never stepped; any valid table
  try {
    h.blob.assign(h.words, 0);
    h.lo16.assign((size_t)B * kMaxN, 0.0);
    h.hi16.assign((size_t)B * kMaxN, 0.0);
  } catch (...) {
    return IBB_ERR_NO_MEMORY;
  }
  for (int b = 0; b < B; ++b)
    if (status[b] == IBB_OK) std::memcpy(h.blob.data() + h.boff[b], comp[b].blob.data(), 8 * comp[b].blob.size());
  for (int b = 0; b < B; ++b)
    for (int k = 0; k < h.nsys[b]; ++k) {
      h.lo16[(size_t)b * kMaxN + k] = lo[(size_t)b * kMaxN + k];
      h.hi16[(size_t)b * kMaxN + k] = hi[(size_t)b * kMaxN + k];
    }
  h.bucket_list.clear();
  for (int q = 0; q < 4; ++q) {
    h.bucket_start[q] = (int)h.bucket_list.size();
    h.bucket_list.insert(h.bucket_list.end(), buckets[q].begin(), buckets[q].end());
    h.bucket_jn[q] = 0;
    for (int b : buckets[q]) h.bucket_jn[q] = std::max(h.bucket_jn[q], h.nsys[b]);
    h.bucket_pop[q] = cfg[q].tiles_per_claim;
    h.bucket_per_cu[q] = cfg[q].blocks_per_cu;
  }
  h.bucket_start[4] = (int)h.bucket_list.size();
  return IBB_OK;
}

// Inputs of a batch into its workspace, and the derivative coefficients.
int batch_upload(const BatchHost& h, char* w, const BatchLayout& L, hipStream_t s) {
  const int B = h.B;
  if (hipMemcpyAsync(w + L.blobs, h.blob.data(), 8 * h.words, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + L.boff, h.boff.data(), sizeof(long long) * B, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + L.sp, h.sp.data(), sizeof(SysParams) * B, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + L.nsys, h.nsys.data(), sizeof(int) * B, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + L.lo, h.lo16.data(), sizeof(double) * kMaxN * B, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + L.hi, h.hi16.data(), sizeof(double) * kMaxN * B, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + L.bucket, h.bucket_list.data(), sizeof(int) * h.bucket_list.size(), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return IBB_ERR_DEVICE;
  if (launch_prep(s, reinterpret_cast<uint64_t*>(w + L.blobs), reinterpret_cast<const long long*>(w + L.boff), B) !=
      hipSuccess)
    return IBB_ERR_DEVICE;
  return IBB_OK;
}

// The device work of one batch solve: counters cleared by fill kernels, then per
// lane-count bucket the initial boxes and one persistent launch.  Contains no
// memset and no host synchronisation, so it can be recorded into a graph.
int batch_enqueue(ibb_ctx* ctx, const BatchHost& h, char* w, const BatchLayout& L, long long fcap, long long ocap,
                  hipStream_t s) {
  const int B = h.B;
  auto D = [&](size_t off) { return w + off; };
  if (launch_fill_u64(s, reinterpret_cast<unsigned long long*>(D(L.count_sys)), (long long)((L.ctrl - L.count_sys) / 8),
                      0ull) != hipSuccess ||
      launch_fill_u64(s, reinterpret_cast<unsigned long long*>(D(L.out_count)), 1, 0ull) != hipSuccess)
    return IBB_ERR_DEVICE;
  for (int q = 0; q < 4; ++q) {
    const int m = h.bucket_start[q + 1] - h.bucket_start[q];
    if (m == 0) continue;
    const int G = 2 << q;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(D(L.ctrl)) + q;
    if (launch_batch_init(s, ctrl, reinterpret_cast<double*>(D(L.front0)), reinterpret_cast<uint32_t*>(D(L.meta0)),
                          reinterpret_cast<uint32_t*>(D(L.sys0)), reinterpret_cast<const double*>(D(L.lo)),
                          reinterpret_cast<const double*>(D(L.hi)),
                          reinterpret_cast<const int*>(D(L.bucket)) + h.bucket_start[q], m, G,
                          reinterpret_cast<const int*>(D(L.nsys)),
                          reinterpret_cast<unsigned long long*>(D(L.count_sys)), B) != hipSuccess)
      return IBB_ERR_DEVICE;
    SolveArgs a;
    std::memset(&a, 0, sizeof a);
    a.front[0] = reinterpret_cast<double*>(D(L.front0));
    a.front[1] = reinterpret_cast<double*>(D(L.front1));
    a.meta[0] = reinterpret_cast<uint32_t*>(D(L.meta0));
    a.meta[1] = reinterpret_cast<uint32_t*>(D(L.meta1));
    a.sys[0] = reinterpret_cast<uint32_t*>(D(L.sys0));
    a.sys[1] = reinterpret_cast<uint32_t*>(D(L.sys1));
    a.front_cap = fcap;
    a.out_box = reinterpret_cast<double*>(D(L.out_box));
    a.out_tag = reinterpret_cast<uint32_t*>(D(L.out_tag));
    a.out_sys = reinterpret_cast<uint32_t*>(D(L.out_sys));
    a.out_cap = ocap;
    a.out_count = reinterpret_cast<unsigned long long*>(D(L.out_count));
    a.out_stride = kMaxN;
    a.ctrl = ctrl;
    a.level_sizes = reinterpret_cast<long long*>(D(L.level));
    a.level_cap = kLevelCap;
    a.max_boxes = 1LL << 62;
    a.timeout_ticks = ctx->clock_khz * 1000LL * 20;
    a.blobs = reinterpret_cast<const uint64_t*>(D(L.blobs));
    a.blob_off = reinterpret_cast<const long long*>(D(L.boff));
    a.sp = reinterpret_cast<const SysParams*>(D(L.sp));
    a.count_sys = reinterpret_cast<unsigned long long*>(D(L.count_sys));
    a.cum_sys = reinterpret_cast<unsigned long long*>(D(L.cum_sys));
    a.status_sys = reinterpret_cast<int*>(D(L.status_sys));
    a.stats_sys = reinterpret_cast<unsigned long long*>(D(L.stats_sys));
    a.B = B;
    const void* fn = solve_kernel_ptr(G, true, true);
    Geometry geo;
    const int st = persistent_geometry(ctx, fn, 0, G, h.bucket_jn[q], &geo);
    if (st) return st;
    if (h.bucket_per_cu[q] > 0) geo.blocks = std::min(geo.blocks, h.bucket_per_cu[q] * ctx->num_cu);
    a.nblocks = geo.blocks;
    a.jrs = geo.jrs;
    a.jn = h.bucket_jn[q];
    a.tiles_per_claim = h.bucket_pop[q];
    void* args[] = {&a};
    if (hipLaunchCooperativeKernel(fn, dim3(geo.blocks), dim3(64 * geo.waves), args, (unsigned)geo.lds, s) !=
        hipSuccess)
      return IBB_ERR_DEVICE;
  }
  return IBB_OK;
}

// Results of a batch solve: statuses, counters, per-system sorted segments.
// *grow_f / *grow_o report a frontier or output overflow (the caller re-runs).
int batch_finish(const BatchHost& h, char* w, const BatchLayout& L, long long ocap, hipStream_t s, double* out_lo,
                 double* out_hi, uint8_t* out_tag, int64_t cap, int64_t* out_off, int32_t* status, ibb_stats* stats,
                 bool* grow_f, long long* grow_o, long long* widest = nullptr) {
  const int B = h.B;
  auto D = [&](size_t off) { return w + off; };
  *grow_f = false;
  *grow_o = 0;
  Ctrl ctrls[4];
  unsigned long long M = 0;
  if (hipMemcpyAsync(ctrls, D(L.ctrl), sizeof ctrls, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&M, D(L.out_count), sizeof M, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return IBB_ERR_DEVICE;
  for (int q = 0; q < 4; ++q) {
    if (widest) widest[q] = 0;
    if (h.bucket_start[q + 1] == h.bucket_start[q]) continue;
    if (ctrls[q].status == IBB_ERR_QUEUE_OVERFLOW) *grow_f = true;
    else if (ctrls[q].status != 0) return ctrls[q].status;
    if (widest) widest[q] = (long long)ctrls[q].max_frontier;
  }
  if (*grow_f) return IBB_OK;
  if ((long long)M > ocap) {
    *grow_o = (long long)M;
    return IBB_OK;
  }
  std::vector<int> sst((size_t)B);
  std::vector<unsigned long long> sstats((size_t)B * 8);
  if (hipMemcpy(sst.data(), D(L.status_sys), sizeof(int) * B, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(sstats.data(), D(L.stats_sys), sizeof(unsigned long long) * 8 * B, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return IBB_ERR_DEVICE;
  // per-system output segments (boxes of failed systems are not returned)
  std::vector<long long> seg((size_t)B + 1, 0);
  for (int b = 0; b < B; ++b) {
    if (status[b] == IBB_OK && sst[b] != 0) status[b] = sst[b];
    const long long mb = (long long)(sstats[(size_t)b * 8 + 6] + sstats[(size_t)b * 8 + 7]);
    seg[b + 1] = seg[b] + mb;
    if (stats) {
      ibb_stats& o = stats[b];
      std::memset(&o, 0, sizeof o);
      int64_t* f = &o.processed;
      for (int k = 0; k < 8; ++k) f[k] = (int64_t)sstats[(size_t)b * 8 + k];
    }
  }
  if (seg[B] != (long long)M) return IBB_ERR_DEVICE;  // counters disagree with the output list
  out_off[0] = 0;
  for (int b = 0; b < B; ++b) out_off[b + 1] = out_off[b] + (status[b] == IBB_OK ? seg[b + 1] - seg[b] : 0);
  if (hipMemcpyAsync(D(L.seg_off), seg.data(), sizeof(long long) * (B + 1), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      launch_fill_u64(s, reinterpret_cast<unsigned long long*>(D(L.cursor)), B, 0ull) != hipSuccess ||
      launch_seg_sort(s, reinterpret_cast<const double*>(D(L.out_box)), reinterpret_cast<const uint32_t*>(D(L.out_tag)),
                      reinterpret_cast<const uint32_t*>(D(L.out_sys)), (long long)M,
                      reinterpret_cast<const long long*>(D(L.seg_off)),
                      reinterpret_cast<unsigned long long*>(D(L.cursor)), reinterpret_cast<uint32_t*>(D(L.order)),
                      reinterpret_cast<const int*>(D(L.nsys)), reinterpret_cast<double*>(D(L.s_lo)),
                      reinterpret_cast<double*>(D(L.s_hi)), reinterpret_cast<uint8_t*>(D(L.s_tag))) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return IBB_ERR_DEVICE;
  if (out_off[B] > cap) return IBB_ERR_OUTPUT_CAPACITY;
  // one transfer of the sorted segments, then each successful system's
  // segment to its place in the caller's arrays
  std::vector<double> hlo((size_t)M * kMaxN), hhi((size_t)M * kMaxN);
  std::vector<uint8_t> htag((size_t)M);
  if (M > 0 &&
      (hipMemcpy(hlo.data(), D(L.s_lo), sizeof(double) * kMaxN * M, hipMemcpyDeviceToHost) != hipSuccess ||
       hipMemcpy(hhi.data(), D(L.s_hi), sizeof(double) * kMaxN * M, hipMemcpyDeviceToHost) != hipSuccess ||
       hipMemcpy(htag.data(), D(L.s_tag), (size_t)M, hipMemcpyDeviceToHost) != hipSuccess))
    return IBB_ERR_DEVICE;
  for (int b = 0; b < B; ++b) {
    if (status[b] != IBB_OK) continue;
    const long long m = seg[b + 1] - seg[b];
    if (m == 0) continue;
    const size_t src = (size_t)seg[b], dst = (size_t)out_off[b];
    std::memcpy(out_lo + dst * kMaxN, hlo.data() + src * kMaxN, sizeof(double) * kMaxN * m);
    std::memcpy(out_hi + dst * kMaxN, hhi.data() + src * kMaxN, sizeof(double) * kMaxN * m);
    std::memcpy(out_tag + dst, htag.data() + src, (size_t)m);
  }
  return IBB_OK;
}

// Frontier capacity (boxes) of a batch's first attempt.  When the autotuner has
// measured every lane-count class present (ibb_batch_tune: the widest level
// of a class's sample launch per member), the capacity is that width times
// the members of each launch, with a margin of a half, for the widest launch;
// otherwise a quarter of the members' node budgets (each at most 2^20; a
// level of a member holds at most half of its budget and the members' widest
// levels do not all coincide).  At least what an earlier batch on this context
// needed.  *measured (if not null): the unclamped estimate from measured
// widths, 0 without one.
long long batch_first_fcap(const ibb_ctx* ctx, int32_t B, const ibb_system* systems, const ibb_params* params,
                           const int32_t* status, const ibb_batch_config* cfg, long long* measured = nullptr) {
  double sum = 0.0, launch[4] = {0, 0, 0, 0};
  bool tuned = true;
  for (int b = 0; b < B; ++b) {
    if (status[b] != IBB_OK) continue;
    sum += (double)std::min<int64_t>(params[b].max_boxes, 1LL << 20);
    const int cls = lanes_class(lanes_for(systems[b].n));
    const double w = ctx->batch_cfg[cls].front_per_member;
    if (!(w > 0.0)) tuned = false;
    launch[lanes_class(cfg[cls].lanes)] += w;
  }
  long long f;
  if (measured) *measured = 0;
  if (tuned) {
    const double widest = std::max(std::max(launch[0], launch[1]), std::max(launch[2], launch[3]));
    const double est = std::min(1.5 * widest, 1e15);
    if (measured) *measured = (long long)est;
    f = std::min<long long>(1LL << 28, std::max<long long>(1LL << 16, (long long)est));
  } else {
    f = std::min<long long>(1LL << 26, std::max<long long>(1LL << 22, (long long)(sum / 4.0)));
  }
  return std::max(f, ctx->batch_fcap);
}

bool batch_args_ok(ibb_ctx* ctx, int32_t B, const ibb_system* systems, const double* lo, const double* hi,
                   const ibb_params* params) {
  return ctx && B >= 1 && systems && lo && hi && params;
}

bool batch_outputs_ok(int64_t cap, const double* out_lo, const double* out_hi, const uint8_t* out_tag,
                      const int64_t* out_off, const int32_t* status) {
  return out_off && status && cap >= 0 && (cap == 0 || (out_lo && out_hi && out_tag));
}

}  // namespace

namespace {

// Largest frontier capacity whose batch layout fits in the device memory that
// is free now plus `reusable` bytes (the workspace a larger layout replaces),
// keeping 5 % of it and 512 MiB for other allocations, and within the
// context's bound on the batch workspace when one is set; at least 2^16.
long long batch_fcap_limit(const ibb_ctx* ctx, int B, size_t words, long long ocap, size_t reusable) {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return 1LL << 16;
  double avail = ((double)free_b + (double)reusable) * 0.95 - (double)(512ull << 20);
  if (ctx->batch_mem > 0) avail = std::min(avail, (double)ctx->batch_mem);
  const double base = (double)batch_layout(B, words, 0, ocap).total;
  const double per = ((double)batch_layout(B, words, 1LL << 20, ocap).total - base) / (double)(1 << 20);
  const double f = (avail - base) / per;
  if (!(f >= (double)(1 << 16))) return 1LL << 16;
  return std::min<long long>(1LL << 28, (long long)f);
}

constexpr int kSplit = 1;  // internal: the batch's frontier does not fit, solve it in parts

// One eager batch solve under the launch configurations cfg[4]; *ms (if not
// null) receives the device time of the batch's device work.  Returns kSplit
// when the frontier the batch needs exceeds what device memory holds and the
// batch has more than one member.
int solve_batch_part(ibb_ctx* ctx, const ibb_batch_config* cfg, int32_t B, const ibb_system* systems,
                     const double* lo, const double* hi, const ibb_params* params, double* out_lo, double* out_hi,
                     uint8_t* out_tag, int64_t cap, int64_t* out_off, int32_t* status, ibb_stats* stats,
                     float* ms, long long* widest) {
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  if (ms) *ms = 0.0f;
  BatchHost h;
  int st = batch_prepare(B, systems, lo, hi, params, cfg, status, h);
  if (st) return st;
  if (!h.any) {
    for (int b = 0; b <= B; ++b) out_off[b] = 0;
    return IBB_OK;
  }
  // capacities sized for the batch up front (an overflow re-runs the whole batch)
  long long measured = 0;
  long long fcap = batch_first_fcap(ctx, B, systems, params, status, cfg, &measured);
  long long ocap = std::max<long long>(1LL << 15, 16LL * B);
  const long long fmax = batch_fcap_limit(ctx, B, h.words, ocap, ctx->bws_bytes);
  // measured widths that cannot fit: split before running (an estimate from
  // node budgets only caps the first attempt)
  if (measured > fmax && B > 1) return kSplit;
  fcap = std::min(fcap, fmax);
  hipStream_t s = ctx->stream;
  for (int attempt = 0; attempt < 10; ++attempt) {
    const BatchLayout L = batch_layout(B, h.words, fcap, ocap);
    st = ensure_device(&ctx->bws, &ctx->bws_bytes, L.total);
    if (st) return st;
    char* w = static_cast<char*>(ctx->bws);
    st = batch_upload(h, w, L, s);
    if (st) return st;
    ctx->tune_pending = false;
    hipEventRecord(ctx->ev0, s);
    st = batch_enqueue(ctx, h, w, L, fcap, ocap, s);
    if (st) return st;
    hipEventRecord(ctx->ev1, s);
    ctx->timed_pending = true;
    bool grow_f = false;
    long long grow_o = 0;
    st = batch_finish(h, w, L, ocap, s, out_lo, out_hi, out_tag, cap, out_off, status, stats, &grow_f, &grow_o,
                      widest);
    if (st) return st;
    if (grow_f) {
      if (fcap >= fmax) {
        if (B > 1) return kSplit;
        // a single member whose widest level exceeds the memory: it fails alone
        status[0] = IBB_ERR_QUEUE_OVERFLOW;
        out_off[0] = out_off[1] = 0;
        if (stats) std::memset(stats, 0, sizeof(ibb_stats));
        return IBB_OK;
      }
      fcap = std::min(fcap * 4, fmax);
      continue;
    }
    if (grow_o) {
      ocap = grow_o;
      continue;
    }
    ctx->batch_fcap = std::max(ctx->batch_fcap, fcap);
    if (ms && hipEventElapsedTime(ms, ctx->ev0, ctx->ev1) != hipSuccess) return IBB_ERR_DEVICE;
    return IBB_OK;
  }
  return IBB_ERR_NO_MEMORY;
}

// A batch solve that splits itself in halves (recursively) while its frontier
// does not fit in device memory.  Each member's result depends on the member
// alone, so the parts' results, placed back to back, are the batch's.  *ms
// and widest[] accumulate over the parts.
int solve_batch_with(ibb_ctx* ctx, const ibb_batch_config* cfg, int32_t B, const ibb_system* systems,
                     const double* lo, const double* hi, const ibb_params* params, double* out_lo, double* out_hi,
                     uint8_t* out_tag, int64_t cap, int64_t* out_off, int32_t* status, ibb_stats* stats,
                     float* ms, long long* widest = nullptr) {
  const int st = solve_batch_part(ctx, cfg, B, systems, lo, hi, params, out_lo, out_hi, out_tag, cap, out_off,
                                  status, stats, ms, widest);
  if (st != kSplit) return st;
  const int B1 = B / 2, B2 = B - B1;
  float ms1 = 0.0f, ms2 = 0.0f;
  long long w1[4] = {0, 0, 0, 0}, w2[4] = {0, 0, 0, 0};
  const int st1 = solve_batch_with(ctx, cfg, B1, systems, lo, hi, params, out_lo, out_hi, out_tag, cap, out_off,
                                   status, stats, ms ? &ms1 : nullptr, w1);
  if (st1 != IBB_OK && st1 != IBB_ERR_OUTPUT_CAPACITY) return st1;
  // the second half writes behind the first (or only sizes its output when
  // the first did not fit)
  const int64_t base = out_off[B1];
  const bool room = st1 == IBB_OK;
  std::vector<int64_t> off2((size_t)B2 + 1);
  const int st2 = solve_batch_with(
      ctx, cfg, B2, systems + B1, lo + (size_t)B1 * kMaxN, hi + (size_t)B1 * kMaxN, params + B1,
      room ? out_lo + (size_t)base * kMaxN : nullptr, room ? out_hi + (size_t)base * kMaxN : nullptr,
      room ? out_tag + base : nullptr, room ? cap - base : 0, off2.data(), status + B1, stats ? stats + B1 : nullptr,
      ms ? &ms2 : nullptr, w2);
  if (st2 != IBB_OK && st2 != IBB_ERR_OUTPUT_CAPACITY) return st2;
  for (int b = 1; b <= B2; ++b) out_off[B1 + b] = base + off2[b];
  if (ms) *ms = ms1 + ms2;
  if (widest)
    for (int q = 0; q < 4; ++q) widest[q] = w1[q] + w2[q];
  return (st1 == IBB_OK && st2 == IBB_OK) ? IBB_OK : IBB_ERR_OUTPUT_CAPACITY;
}

}  // namespace

extern "C" int ibb_solve_batch(ibb_ctx* ctx, int32_t B, const ibb_system* systems, const double* lo,
                               const double* hi, const ibb_params* params, double* out_lo, double* out_hi,
                               uint8_t* out_tag, int64_t cap, int64_t* out_off, int32_t* status,
                               ibb_stats* stats) {
  if (!batch_args_ok(ctx, B, systems, lo, hi, params) || !batch_outputs_ok(cap, out_lo, out_hi, out_tag, out_off, status))
    return IBB_ERR_INVALID_ARG;
  return solve_batch_with(ctx, ctx->batch_cfg, B, systems, lo, hi, params, out_lo, out_hi, out_tag, cap, out_off,
                          status, stats, nullptr);
}

extern "C" int ibb_batch_set_memory(ibb_ctx* ctx, int64_t bytes) {
  if (!ctx || bytes < 0) return IBB_ERR_INVALID_ARG;
  if (bytes > 0 && ctx->bws_bytes > (size_t)bytes) {
    // batch solves are synchronous: nothing runs on the workspace now
    if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
    hipFree(ctx->bws);
    ctx->bws = nullptr;
    ctx->bws_bytes = 0;
  }
  ctx->batch_mem = bytes;
  ctx->batch_fcap = 0;  // capacities learned under another bound no longer apply
  return IBB_OK;
}

extern "C" int ibb_batch_get_config(ibb_ctx* ctx, int32_t cls, ibb_batch_config* out) {
  if (!ctx || !out || cls < 0 || cls > 3) return IBB_ERR_INVALID_ARG;
  *out = ctx->batch_cfg[cls];
  return IBB_OK;
}

namespace {
bool batch_config_ok(int32_t cls, const ibb_batch_config& c) {
  const int L = c.lanes;
  return L >= (2 << cls) && L <= 16 && (L & (L - 1)) == 0 && c.tiles_per_claim >= 1 && c.tiles_per_claim <= 16 &&
         c.blocks_per_cu >= 0;
}
}  // namespace

extern "C" int ibb_batch_set_config(ibb_ctx* ctx, int32_t cls, const ibb_batch_config* cfg) {
  if (!ctx || !cfg || cls < 0 || cls > 3 || !batch_config_ok(cls, *cfg)) return IBB_ERR_INVALID_ARG;
  ctx->batch_cfg[cls] = ibb_batch_config{cfg->lanes, cfg->tiles_per_claim, cfg->blocks_per_cu, 0, 0.0};
  return IBB_OK;
}

extern "C" int ibb_batch_tune(ibb_ctx* ctx, int32_t B, const ibb_system* systems, const double* lo, const double* hi,
                              const ibb_params* params, int32_t sample) {
  if (!batch_args_ok(ctx, B, systems, lo, hi, params) || sample < 1) return IBB_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  std::vector<int> members[4];
  for (int b = 0; b < B; ++b)
    if (validate(&systems[b], lo + (size_t)b * kMaxN, hi + (size_t)b * kMaxN, &params[b]) == IBB_OK)
      members[lanes_class(lanes_for(systems[b].n))].push_back(b);
  // wider classes first: a narrower class may move its members into the
  // launch of a wider one, whose configuration is then already chosen
  for (int q = 3; q >= 0; --q) {
    if (members[q].empty()) continue;
    const int m = (int)std::min<size_t>(members[q].size(), (size_t)sample);
    std::vector<ibb_system> ss((size_t)m);
    std::vector<ibb_params> ps((size_t)m);
    std::vector<double> ls((size_t)m * kMaxN), hs((size_t)m * kMaxN);
    int jn = 0;
    for (int i = 0; i < m; ++i) {
      const int b = members[q][(size_t)i];
      ss[(size_t)i] = systems[b];
      ps[(size_t)i] = params[b];
      std::memcpy(&ls[(size_t)i * kMaxN], lo + (size_t)b * kMaxN, sizeof(double) * kMaxN);
      std::memcpy(&hs[(size_t)i * kMaxN], hi + (size_t)b * kMaxN, sizeof(double) * kMaxN);
      jn = std::max(jn, systems[b].n);
    }
    const int G = 2 << q;
    // workgroups per CU that fit the natural launch
    Geometry geo;
    int st = persistent_geometry(ctx, solve_kernel_ptr(G, true, true), 0, G, jn, &geo);
    if (st) return st;
    const int full = geo.blocks / ctx->num_cu;
    const int part = std::max(1, (2 * full + 2) / 3);
    std::vector<ibb_batch_config> cands;
    const ibb_batch_config def{G, 1, 0, 0, 0.0};
    cands.push_back(def);
    for (int pop : {1, 4})
      for (int pc : {0, part}) {
        if (pop == 1 && pc == 0) continue;
        if (pc == full) continue;
        cands.push_back(ibb_batch_config{G, pop, pc, 0, 0.0});
      }
    if (G < 16) {
      const ibb_batch_config& w = ctx->batch_cfg[q + 1];
      cands.push_back(ibb_batch_config{2 * G, w.tiles_per_claim, w.blocks_per_cu, 0, 0.0});
    }
    // results of the sample solves (discarded; compared across candidates)
    int64_t cap = std::max<int64_t>(1 << 12, 8LL * m);
    std::vector<double> olo, ohi;
    std::vector<uint8_t> otag;
    std::vector<int64_t> off((size_t)m + 1);
    std::vector<int32_t> stat((size_t)m), stat0((size_t)m);
    std::vector<ibb_stats> sts((size_t)m), sts0((size_t)m);
    std::vector<float> times(cands.size(), 0.0f);
    double front_per_member = 0.0;
    for (size_t c = 0; c <= cands.size(); ++c) {
      // run 0 warms the default launch up; runs 1.. time the candidates
      const ibb_batch_config& cand = cands[c == 0 ? 0 : c - 1];
      ibb_batch_config cfg[4] = {{2, 1, 0, 0, 0.0}, {4, 1, 0, 0, 0.0}, {8, 1, 0, 0, 0.0}, {16, 1, 0, 0, 0.0}};
      cfg[q] = cand;
      const int qe = lanes_class(cand.lanes);
      if (qe != q) cfg[qe] = ibb_batch_config{cand.lanes, cand.tiles_per_claim, cand.blocks_per_cu, 0, 0.0};
      float ms = 0.0f;
      long long widest[4] = {0, 0, 0, 0};
      for (;;) {
        olo.assign((size_t)cap * kMaxN, 0.0);
        ohi.assign((size_t)cap * kMaxN, 0.0);
        otag.assign((size_t)cap, 0);
        st = solve_batch_with(ctx, cfg, m, ss.data(), ls.data(), hs.data(), ps.data(), olo.data(), ohi.data(),
                              otag.data(), cap, off.data(), stat.data(), sts.data(), &ms, widest);
        if (st == IBB_ERR_OUTPUT_CAPACITY && off[(size_t)m] > cap) {
          cap = off[(size_t)m];
          continue;
        }
        break;
      }
      if (st) return st;
      if (c == 0) {
        stat0 = stat;
        sts0 = sts;
        // queue size: the widest level of the class's own launch, per member
        front_per_member = (double)widest[q] / (double)m;
        continue;
      }
      // every configuration must reproduce the default's statuses and counters
      for (int i = 0; i < m; ++i)
        if (stat[(size_t)i] != stat0[(size_t)i] ||
            std::memcmp(&sts[(size_t)i], &sts0[(size_t)i], sizeof(ibb_stats)) != 0)
          return IBB_ERR_DEVICE;
      times[c - 1] = ms;
    }
    size_t best = 0;
    for (size_t c = 1; c < cands.size(); ++c)
      if (times[c] < times[best]) best = c;
    if (best != 0 && times[best] > 0.97f * times[0]) best = 0;
    ibb_batch_config chosen = cands[best];
    chosen.tuned = 1;
    chosen.ms = (double)times[best];
    chosen.front_per_member = std::max(front_per_member, 1.0);
    ctx->batch_cfg[q] = chosen;
  }
  return IBB_OK;
}

// A batch prepared once and solved many times: inputs uploaded and the device
// work recorded into a graph at creation; each run replays the graph.
struct ibb_batch_plan {
  ibb_ctx* ctx = nullptr;
  BatchHost h;
  std::vector<int32_t> status0;  // validation status of each member
  long long fcap = 0, ocap = 0;
  BatchLayout L{};
  void* ws = nullptr;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void plan_release_graph(ibb_batch_plan* p) {
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

// (Re)allocate the plan's workspace for its capacities, upload, record.
int plan_build(ibb_batch_plan* p) {
  plan_release_graph(p);
  if (p->ws) hipFree(p->ws);
  p->ws = nullptr;
  p->L = batch_layout(p->h.B, p->h.words, p->fcap, p->ocap);
  if (hipMalloc(&p->ws, p->L.total) != hipSuccess) {
    p->ws = nullptr;
    return IBB_ERR_NO_MEMORY;
  }
  char* w = static_cast<char*>(p->ws);
  int st = batch_upload(p->h, w, p->L, p->stream);
  if (st) return st;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return IBB_ERR_DEVICE;
  if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return IBB_ERR_DEVICE;
  st = batch_enqueue(p->ctx, p->h, w, p->L, p->fcap, p->ocap, p->stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(p->stream, &g);
  if (st) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess || !g) return IBB_ERR_UNSUPPORTED;
  p->graph = g;
  if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    p->exec = nullptr;
    return IBB_ERR_UNSUPPORTED;
  }
  return IBB_OK;
}

}  // namespace

extern "C" int ibb_batch_plan_create(ibb_ctx* ctx, int32_t B, const ibb_system* systems, const double* lo,
                                     const double* hi, const ibb_params* params, ibb_batch_plan** out) {
  if (!out) return IBB_ERR_INVALID_ARG;
  *out = nullptr;
  if (!batch_args_ok(ctx, B, systems, lo, hi, params)) return IBB_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  ibb_batch_plan* p = new (std::nothrow) ibb_batch_plan();
  if (!p) return IBB_ERR_NO_MEMORY;
  p->ctx = ctx;
  p->status0.assign((size_t)B, 0);
  int st = batch_prepare(B, systems, lo, hi, params, ctx->batch_cfg, p->status0.data(), p->h);
  if (!st && hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
    p->stream = nullptr;
    st = IBB_ERR_DEVICE;
  }
  p->fcap = batch_first_fcap(ctx, B, systems, params, p->status0.data(), ctx->batch_cfg);
  p->ocap = std::max<long long>(1LL << 15, 16LL * B);
  if (!st && p->h.any) {
    p->fcap = std::min(p->fcap, batch_fcap_limit(ctx, B, p->h.words, p->ocap, 0));
    st = plan_build(p);
  }
  if (st) {
    ibb_batch_plan_destroy(p);
    return st;
  }
  *out = p;
  return IBB_OK;
}

extern "C" int ibb_batch_plan_run(ibb_batch_plan* p, double* out_lo, double* out_hi, uint8_t* out_tag, int64_t cap,
                                  int64_t* out_off, int32_t* status, ibb_stats* stats) {
  if (!p || !batch_outputs_ok(cap, out_lo, out_hi, out_tag, out_off, status)) return IBB_ERR_INVALID_ARG;
  const int B = p->h.B;
  for (int b = 0; b < B; ++b) status[b] = p->status0[b];
  if (!p->h.any) {
    for (int b = 0; b <= B; ++b) out_off[b] = 0;
    return IBB_OK;
  }
  if (hipSetDevice(p->ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  ibb_ctx* ctx = p->ctx;
  for (int attempt = 0; attempt < 10; ++attempt) {
    ctx->tune_pending = false;
    hipEventRecord(ctx->ev0, p->stream);
    if (hipGraphLaunch(p->exec, p->stream) != hipSuccess) return IBB_ERR_DEVICE;
    hipEventRecord(ctx->ev1, p->stream);
    ctx->timed_pending = true;
    bool grow_f = false;
    long long grow_o = 0;
    for (int b = 0; b < B; ++b) status[b] = p->status0[b];
    int st = batch_finish(p->h, static_cast<char*>(p->ws), p->L, p->ocap, p->stream, out_lo, out_hi, out_tag, cap,
                          out_off, status, stats, &grow_f, &grow_o);
    if (st) return st;
    if (!grow_f && !grow_o) return IBB_OK;
    if (grow_f) {
      // a plan is not split: a frontier beyond device memory fails the run
      const long long fmax = batch_fcap_limit(ctx, B, p->h.words, p->ocap, p->L.total);
      if (p->fcap >= fmax) return IBB_ERR_NO_MEMORY;
      p->fcap = std::min(p->fcap * 4, fmax);
    }
    if (grow_o) p->ocap = grow_o;
    st = plan_build(p);
    if (st) return st;
  }
  return IBB_ERR_NO_MEMORY;
}

extern "C" void ibb_batch_plan_destroy(ibb_batch_plan* p) {
  if (!p) return;
  if (p->stream) hipStreamSynchronize(p->stream);
  plan_release_graph(p);
  if (p->ws) hipFree(p->ws);
  if (p->stream) hipStreamDestroy(p->stream);
  delete p;
}

extern "C" {

const char* ibb_strerror(int s) {
  switch (s) {
    case IBB_OK: return "ok";
    case IBB_ERR_INVALID_ARG: return "invalid argument";
    case IBB_ERR_BUDGET: return "box budget exceeded";
    case IBB_ERR_OUTPUT_CAPACITY: return "output capacity too small";
    case IBB_ERR_QUEUE_OVERFLOW: return "frontier capacity exceeded";
    case IBB_ERR_NO_MEMORY: return "out of memory";
    case IBB_ERR_DEVICE: return "HIP runtime error";
    case IBB_ERR_UNSUPPORTED: return "unsupported by this build";
    case IBB_ERR_TIMEOUT: return "device wait timed out";
    case IBB_ERR_WORKSPACE_LIMIT: return "workspace larger than the allocation-free maximum";
    default: return "unknown status";
  }
}

void ibb_params_default(ibb_params* p) {
  if (!p) return;
  p->tol = 1e-8;
  p->max_boxes = 100000000LL;
  p->split_mode = IBB_SPLIT_WIDEST;
  p->max_recontract = 16;
  p->recontract_ratio = 0.5;
  p->hs_max_width = INFINITY;
  p->schedule = IBB_SCHEDULE_AUTO;
  p->contractor = IBB_CONTRACT_HS;
  p->inclusion = IBB_INCLUDE_NATURAL;
  p->reserved = 0;
}

int ibb_ctx_create(int device, ibb_ctx** out) {
  if (!out) return IBB_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return IBB_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return IBB_ERR_DEVICE;
  ibb_ctx* c = new (std::nothrow) ibb_ctx();
  if (!c) return IBB_ERR_NO_MEMORY;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return IBB_ERR_DEVICE;
  }
  c->num_cu = prop.multiProcessorCount;
  c->max_lds_block = prop.sharedMemPerBlock;
  c->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    c->clock_khz = khz;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&c->info), sizeof(long long) * kInfoLen) != hipSuccess) {
    ibb_ctx_destroy(c);
    return IBB_ERR_DEVICE;
  }
  // the allocation-free solve: the workspace array's address on this device,
  // and a pinned staging buffer that holds the largest system's inputs
  if (noalloc_scratch(device, &c->noalloc_ws) != hipSuccess) {
    ibb_ctx_destroy(c);
    return IBB_ERR_DEVICE;
  }
  if (ensure_pinned(c, 8 * max_blob_words(IBB_MAX_N) + 2 * sizeof(double) * kMaxN) != IBB_OK) {
    ibb_ctx_destroy(c);
    return IBB_ERR_NO_MEMORY;
  }
  *out = c;
  return IBB_OK;
}

void ibb_ctx_destroy(ibb_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  if (c->ws) hipFree(c->ws);
  if (c->bws) hipFree(c->bws);
  if (c->sorted) hipFree(c->sorted);
  if (c->info) hipFree(c->info);
  if (c->pinned) hipHostFree(c->pinned);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  if (c->staged) hipEventDestroy(c->staged);
  if (c->done) hipEventDestroy(c->done);
  if (c->stream) hipStreamDestroy(c->stream);
  delete c;
}

size_t ibb_workspace_size(int32_t n, int64_t frontier_cap, int64_t out_cap) {
  if (n < 1 || n > IBB_MAX_N || frontier_cap < 1 || out_cap < 0) return 0;
  return ws_layout(n, max_blob_words(n), frontier_cap, out_cap).total;
}

int ibb_solve_async(ibb_ctx* ctx, const ibb_system* sys, const double* lo, const double* hi,
                    const ibb_params* params, void* d_ws, size_t ws_bytes, int64_t frontier_cap,
                    int64_t out_cap, double* d_out_lo, double* d_out_hi, uint8_t* d_out_tag,
                    int64_t* d_info, void* stream) {
  if (!ctx || !d_ws || !d_info || frontier_cap < 1 || out_cap < 0) return IBB_ERR_INVALID_ARG;
  if (out_cap > 0 && (!d_out_lo || !d_out_hi || !d_out_tag)) return IBB_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return IBB_ERR_INVALID_ARG;
  int st = validate(sys, lo, hi, params);
  if (st) return st;
  if (ws_bytes < ibb_workspace_size(sys->n, frontier_cap, out_cap)) return IBB_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  Compiled c;
  try {
    compile(sys, c);
  } catch (...) {
    return IBB_ERR_NO_MEMORY;
  }
  const WsLayout L = ws_layout(c.n, max_blob_words(c.n), frontier_cap, out_cap);
  return enqueue_solve(ctx, c, lo, hi, params, static_cast<char*>(d_ws), L, frontier_cap, out_cap, d_out_lo,
                       d_out_hi, d_out_tag, reinterpret_cast<long long*>(d_info),
                       static_cast<hipStream_t>(stream));
}

// The solve of ibb_solve_async with the device's own workspace array: no
// device or pinned allocation (the pinned staging buffer was sized for the
// largest system when the context was created, so enqueue_solve reuses it).
int ibb_solve_noalloc(ibb_ctx* ctx, const ibb_system* sys, const double* lo, const double* hi,
                      const ibb_params* params, int64_t frontier_cap, int64_t out_cap, double* d_out_lo,
                      double* d_out_hi, uint8_t* d_out_tag, int64_t* d_info, void* stream) {
  if (!ctx || !ctx->noalloc_ws || !d_info || frontier_cap < 1 || out_cap < 0) return IBB_ERR_INVALID_ARG;
  if (out_cap > 0 && (!d_out_lo || !d_out_hi || !d_out_tag)) return IBB_ERR_INVALID_ARG;
  int st = validate(sys, lo, hi, params);
  if (st) return st;
  if (ibb_workspace_size(sys->n, frontier_cap, out_cap) > (size_t)IBB_NOALLOC_WORKSPACE_BYTES)
    return IBB_ERR_WORKSPACE_LIMIT;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  Compiled c;
  try {
    compile(sys, c);
  } catch (...) {
    return IBB_ERR_NO_MEMORY;
  }
  const WsLayout L = ws_layout(c.n, max_blob_words(c.n), frontier_cap, out_cap);
  return enqueue_solve(ctx, c, lo, hi, params, static_cast<char*>(ctx->noalloc_ws), L, frontier_cap, out_cap,
                       d_out_lo, d_out_hi, d_out_tag, reinterpret_cast<long long*>(d_info),
                       static_cast<hipStream_t>(stream));
}

int ibb_solve(ibb_ctx* ctx, const ibb_system* sys, const double* lo, const double* hi,
              const ibb_params* params, double* out_lo, double* out_hi, uint8_t* out_tag, int64_t cap,
              int64_t* n_out, ibb_stats* stats) {
  if (!ctx || !n_out || cap < 0 || (cap > 0 && (!out_lo || !out_hi || !out_tag))) return IBB_ERR_INVALID_ARG;
  *n_out = 0;
  int st = validate(sys, lo, hi, params);
  if (st) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  Compiled c;
  try {
    compile(sys, c);
  } catch (...) {
    return IBB_ERR_NO_MEMORY;
  }
  const int n = c.n;
  long long fcap = std::min<long long>(1LL << 22, std::max<long long>(1024, params->max_boxes + 1));
  long long ocap = 1LL << 14;
  long long info[kInfoLen];
  for (int attempt = 0; attempt < 12; ++attempt) {
    const WsLayout L = ws_layout(n, c.blob.size(), fcap, ocap);
    const size_t sorted_need = (size_t)ocap * (2 * n * sizeof(double) + 1) + 64;
    st = ensure_device(&ctx->ws, &ctx->ws_bytes, L.total);
    if (!st) st = ensure_device(reinterpret_cast<void**>(&ctx->sorted), &ctx->sorted_bytes, sorted_need);
    if (st) return st;
    double* d_lo = ctx->sorted;
    double* d_hi = d_lo + (size_t)ocap * n;
    uint8_t* d_tag = reinterpret_cast<uint8_t*>(d_hi + (size_t)ocap * n);
    st = enqueue_solve(ctx, c, lo, hi, params, static_cast<char*>(ctx->ws), L, fcap, ocap, d_lo, d_hi, d_tag,
                       ctx->info, ctx->stream);
    if (st) return st;
    if (hipMemcpyAsync(info, ctx->info, sizeof info, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
      return IBB_ERR_DEVICE;
    float ms = 0.0f;
    hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    const int status = (int)info[0];
    if (status == IBB_ERR_QUEUE_OVERFLOW) {
      fcap *= 4;
      continue;
    }
    if (status == IBB_ERR_OUTPUT_CAPACITY) {
      ocap = std::max<long long>(ocap * 2, info[1]);
      continue;
    }
    // per-level sizes for ibb_last_level_sizes
    const long long nlev = std::min<long long>(info[10], kLevelCap);
    ctx->last_levels.assign((size_t)nlev, 0);
    if (nlev > 0)
      hipMemcpy(ctx->last_levels.data(), static_cast<char*>(ctx->ws) + L.level, sizeof(long long) * nlev,
                hipMemcpyDeviceToHost);
    fill_stats(stats, info, ms);
    if (status != IBB_OK) return status;
    *n_out = info[1];
    if (info[1] > cap) return IBB_ERR_OUTPUT_CAPACITY;
    const size_t m = (size_t)info[1];
    if (m) {
      if (hipMemcpy(out_lo, d_lo, sizeof(double) * m * n, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(out_hi, d_hi, sizeof(double) * m * n, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(out_tag, d_tag, m, hipMemcpyDeviceToHost) != hipSuccess)
        return IBB_ERR_DEVICE;
    }
    return IBB_OK;
  }
  return IBB_ERR_NO_MEMORY;
}

double ibb_last_kernel_ms(ibb_ctx* ctx) {
  if (!ctx || !ctx->timed_pending) return -1.0;
  if (hipEventSynchronize(ctx->ev1) != hipSuccess) return -1.0;
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) != hipSuccess) return -1.0;
  return (double)ms;
}

int64_t ibb_last_level_sizes(ibb_ctx* ctx, int64_t* sizes, int64_t cap) {
  if (!ctx) return 0;
  const int64_t m = (int64_t)ctx->last_levels.size();
  for (int64_t i = 0; i < std::min(m, cap); ++i) sizes[i] = ctx->last_levels[(size_t)i];
  return m;
}

int ibb_debug_step(ibb_ctx* ctx, const ibb_system* sys, const double* lo, const double* hi,
                   const ibb_params* params, double* dump, int64_t dump_len) {
  if (!ctx || !dump) return IBB_ERR_INVALID_ARG;
  int st = validate(sys, lo, hi, params);
  if (st) return st;
  const int n = sys->n;
  if (dump_len < dbg_len(n)) return IBB_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  Compiled c;
  try {
    compile(sys, c);
  } catch (...) {
    return IBB_ERR_NO_MEMORY;
  }
  const long long fcap = 1 << 17, ocap = 1 << 10;
  const WsLayout L = ws_layout(n, c.blob.size(), fcap, ocap);
  const size_t sorted_need = (size_t)ocap * (2 * n * sizeof(double) + 1) + 64;
  st = ensure_device(&ctx->ws, &ctx->ws_bytes, L.total);
  if (!st) st = ensure_device(reinterpret_cast<void**>(&ctx->sorted), &ctx->sorted_bytes, sorted_need);
  if (st) return st;
  double* d_dbg = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d_dbg), sizeof(double) * dbg_len(n)) != hipSuccess) return IBB_ERR_NO_MEMORY;
  st = IBB_OK;
  if (hipMemsetAsync(d_dbg, 0, sizeof(double) * dbg_len(n), ctx->stream) != hipSuccess) st = IBB_ERR_DEVICE;
  double* d_lo = ctx->sorted;
  double* d_hi = d_lo + (size_t)ocap * n;
  uint8_t* d_tag = reinterpret_cast<uint8_t*>(d_hi + (size_t)ocap * n);
  if (!st)
    st = enqueue_solve(ctx, c, lo, hi, params, static_cast<char*>(ctx->ws), L, fcap, ocap, d_lo, d_hi, d_tag,
                       ctx->info, ctx->stream, 1, d_dbg);
  if (!st && (hipStreamSynchronize(ctx->stream) != hipSuccess ||
              hipMemcpy(dump, d_dbg, sizeof(double) * dbg_len(n), hipMemcpyDeviceToHost) != hipSuccess))
    st = IBB_ERR_DEVICE;
  hipFree(d_dbg);
  return st;
}

int ibb_round(ibb_ctx* ctx, const ibb_system* sys, const ibb_params* params, int64_t count, const double* lo,
              const double* hi, const uint32_t* rec, double* child_lo, double* child_hi, uint32_t* child_rec,
              int64_t child_cap, int64_t* n_child, double* emit_lo, double* emit_hi, uint8_t* emit_tag,
              int64_t emit_cap, int64_t* n_emit, ibb_stats* stats) {
  if (!ctx || !n_child || !n_emit || count < 0 || child_cap < 0 || emit_cap < 0) return IBB_ERR_INVALID_ARG;
  if (count > 0 && (!lo || !hi || !rec)) return IBB_ERR_INVALID_ARG;
  if (child_cap > 0 && (!child_lo || !child_hi || !child_rec)) return IBB_ERR_INVALID_ARG;
  if (emit_cap > 0 && (!emit_lo || !emit_hi || !emit_tag)) return IBB_ERR_INVALID_ARG;
  *n_child = 0;
  *n_emit = 0;
  if (!sys || sys->n < 1 || sys->n > IBB_MAX_N) return IBB_ERR_INVALID_ARG;
  const int n = sys->n;
  std::vector<double> zero(n, 0.0);
  int st = validate(sys, zero.data(), zero.data(), params);
  for (int64_t b = 0; b < count && !st; ++b) st = validate(sys, lo + b * n, hi + b * n, params);
  if (st) return st;
  for (int64_t b = 0; b < count; ++b)
    if ((rec[b] & ~0xFF01u) != 0) return IBB_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  Compiled c;
  try {
    compile(sys, c);
  } catch (...) {
    return IBB_ERR_NO_MEMORY;
  }
  const int G = c.G;
  const long long fcap = std::max<long long>({count, child_cap, 1});
  const long long ocap = std::max<long long>(emit_cap, 1);
  const WsLayout L = ws_layout(n, c.blob.size(), fcap, ocap);
  st = ensure_device(&ctx->ws, &ctx->ws_bytes, L.total);
  if (st) return st;
  char* ws = static_cast<char*>(ctx->ws);
  // level 0: the caller's boxes in the device layout (G rows of (lo, -hi))
  std::vector<double> front((size_t)std::max<long long>(count, 1) * G * 2, 0.0);
  for (int64_t b = 0; b < count; ++b)
    for (int k = 0; k < n; ++k) {
      front[((size_t)b * G + k) * 2] = lo[b * n + k];
      front[((size_t)b * G + k) * 2 + 1] = -hi[b * n + k];
    }
  Ctrl ctrl;
  std::memset(&ctrl, 0, sizeof ctrl);
  ctrl.count[0] = (unsigned long long)count;
  hipStream_t s = ctx->stream;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(ws + L.blob, c.blob.data(), 8 * c.blob.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ws + L.ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice) != hipSuccess ||
      (count > 0 &&
       (hipMemcpy(ws + L.front0, front.data(), sizeof(double) * count * G * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ws + L.meta0, rec, sizeof(uint32_t) * count, hipMemcpyHostToDevice) != hipSuccess)))
    return IBB_ERR_DEVICE;
  if (launch_prep(s, reinterpret_cast<uint64_t*>(ws + L.blob), nullptr, 1) != hipSuccess) return IBB_ERR_DEVICE;
  st = launch_search(ctx, c, params, ws, L, fcap, ocap, std::numeric_limits<long long>::max(), s, 1, nullptr);
  if (st) return st;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(&ctrl, ws + L.ctrl, sizeof ctrl, hipMemcpyDeviceToHost) != hipSuccess)
    return IBB_ERR_DEVICE;
  if (ctrl.status != 0) return ctrl.status;
  if (stats) {
    long long info[kInfoLen] = {0};
    for (int i = 0; i < 8; ++i) info[2 + i] = (long long)ctrl.stats[i];
    info[10] = (long long)ctrl.levels;
    info[11] = (long long)ctrl.max_frontier;
    float ms = 0.0f;
    hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    fill_stats(stats, info, ms);
  }
  const long long nc = (long long)ctrl.count[1], ne = (long long)ctrl.out_count;
  *n_child = nc;
  *n_emit = ne;
  if (nc > child_cap || ne > emit_cap) return IBB_ERR_OUTPUT_CAPACITY;
  std::vector<double> cb((size_t)nc * G * 2), eb((size_t)ne * G * 2);
  std::vector<uint32_t> et((size_t)ne);
  if ((nc > 0 &&
       (hipMemcpy(cb.data(), ws + L.front1, sizeof(double) * cb.size(), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(child_rec, ws + L.meta1, sizeof(uint32_t) * nc, hipMemcpyDeviceToHost) != hipSuccess)) ||
      (ne > 0 &&
       (hipMemcpy(eb.data(), ws + L.out_box, sizeof(double) * eb.size(), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(et.data(), ws + L.out_tag, sizeof(uint32_t) * ne, hipMemcpyDeviceToHost) != hipSuccess)))
    return IBB_ERR_DEVICE;
  for (long long b = 0; b < nc; ++b)
    for (int k = 0; k < n; ++k) {
      child_lo[b * n + k] = cb[((size_t)b * G + k) * 2];
      child_hi[b * n + k] = -cb[((size_t)b * G + k) * 2 + 1];
    }
  for (long long b = 0; b < ne; ++b) {
    for (int k = 0; k < n; ++k) {
      emit_lo[b * n + k] = eb[((size_t)b * G + k) * 2];
      emit_hi[b * n + k] = -eb[((size_t)b * G + k) * 2 + 1];
    }
    emit_tag[b] = (uint8_t)et[b];
  }
  return IBB_OK;
}

int ibb_selftest_ops(ibb_ctx* ctx, int32_t op, int64_t n, const double* a, const double* b, double* out) {
  if (!ctx || n < 0 || op < 0 || op > 11 || (n > 0 && (!a || !b || !out))) return IBB_ERR_INVALID_ARG;
  if (n == 0) return IBB_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  double* d = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d), sizeof(double) * 3 * (size_t)n) != hipSuccess)
    return IBB_ERR_NO_MEMORY;
  int st = IBB_OK;
  if (hipMemcpy(d, a, sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d + n, b, sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
      launch_selftest(ctx->stream, op, n, d, d + n, d + 2 * n) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess ||
      hipMemcpy(out, d + 2 * n, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess)
    st = IBB_ERR_DEVICE;
  hipFree(d);
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: continuous batching.  Admitted solves occupy device slots; their
// boxes share one frontier per size bucket.  Each scheduling round (1) waits
// for the device pass enqueued by the previous round and harvests the solves
// that ran out of boxes, (2) admits queued requests whose reservation fits
// the device pool and uploads them with one copy and one kernel, (3) makes
// room for the next levels of every bucket (growing its frontier within the
// pool, else failing the solves that outgrew their reservation the most) and
// (4) enqueues the next pass of every bucket and returns, so that the host's
// work of the next round overlaps the device's.  A solve's result does not
// depend on its neighbours.
// ---------------------------------------------------------------------------
namespace {

constexpr int kSlotWords = 8192;  // 64 KiB of compiled table per slot

struct Request {
  int64_t id = 0;
  Compiled comp;
  double lo[kMaxN] = {0}, hi[kMaxN] = {0};
  ibb_params p{};
  long long reserve_boxes = 0;  // frontier boxes reserved at admission
  size_t reserve_bytes = 0;
  int slot = -1, bucket = -1;
  int state = 0;  // 0 queued, 1 on the device, 2 done
  int status = IBB_OK;
  ibb_stats stats{};
  std::vector<double> out_lo, out_hi;
  std::vector<uint8_t> out_tag;
};

struct Bucket {
  int G = 0;
  long long cap = 0;
  Ctrl* ctrl = nullptr;
  double* front[2] = {nullptr, nullptr};
  uint32_t* meta[2] = {nullptr, nullptr};
  uint32_t* sys[2] = {nullptr, nullptr};
  void* mem = nullptr;
  size_t bytes = 0;
  int level = 0;
  unsigned long long count = 0;  // boxes at `level`
  std::vector<int> slots;        // active slots
};

// Device bytes of a bucket frontier of `cap` boxes of G lanes: two levels of
// boxes, records and system indices.
size_t bucket_bytes(int G, long long cap) { return (size_t)cap * 2 * (sizeof(double) * 2 * G + 8) + 4096; }

// Frontier boxes reserved for a request: reserve_per_solve for every 64
// bisections the tree needs at least (every coordinate halved from its width
// down to tol), at most max_boxes + 1.
long long reserve_for(const Request& r, long long per_solve) {
  long long depth = 0;
  for (int k = 0; k < r.comp.n; ++k) {
    const double w = r.hi[k] - r.lo[k];
    if (w > r.p.tol) depth += (long long)std::ceil(std::log2(w / r.p.tol));
  }
  const long long units = std::max<long long>(1, (depth + 63) / 64);
  return std::min<long long>(r.p.max_boxes + 1, per_solve * units);
}

}  // namespace

namespace ibb {
hipError_t launch_admit(hipStream_t s, const AdmitRec* recs, int count, const uint64_t* payload, uint64_t* blobs,
                        int slot_words, SysParams* sp, int* nsys, int* status_sys, uint8_t* evict,
                        unsigned long long* stats_sys, unsigned long long* slot_count, unsigned long long* cum_sys,
                        unsigned long long* pending, unsigned long long* count_sys, int S);
hipError_t launch_evict(hipStream_t s, const int* slots, int count, uint8_t* evict, int* status_sys, int status);
}  // namespace ibb

struct ibb_server {
  ibb_ctx* ctx = nullptr;
  ibb_server_config cfg{};
  void* mem = nullptr;  // per-slot device state
  uint64_t* blobs = nullptr;
  long long* boff = nullptr;
  SysParams* sp = nullptr;
  int* nsys = nullptr;
  unsigned long long *count_sys = nullptr, *cum_sys = nullptr, *stats_sys = nullptr, *slot_count = nullptr;
  unsigned long long* pending = nullptr;  // boxes of each slot still in a frontier
  int* status_sys = nullptr;
  uint8_t* evict = nullptr;  // slots whose boxes the next pass drops
  double* out_box = nullptr;
  uint32_t* out_tag = nullptr;
  double *s_lo = nullptr, *s_hi = nullptr;
  uint8_t* s_tag = nullptr;
  long long* level_sizes = nullptr;
  Bucket bk[4];
  size_t pool_used = 0;      // device bytes of the bucket frontiers
  size_t reserved = 0;       // bytes reserved by the admitted solves
  // per-round staging: admission records and compiled systems (host pinned,
  // device), and the pinned mirror of the counters read back after a pass
  char* h_stage = nullptr;
  char* d_stage = nullptr;
  size_t stage_bytes = 0;
  char* h_back = nullptr;
  size_t back_bytes = 0;
  hipEvent_t pass_done = nullptr;
  bool in_flight = false;
  std::deque<Request*> queue;
  std::map<int64_t, Request*> reqs;
  std::vector<Request*> by_slot;
  std::vector<int> free_slots;
  std::vector<int64_t> finished;  // ids harvested and not yet reported
  int64_t next_id = 0;
};

namespace {

int bucket_of(int G) { return G == 2 ? 0 : G == 4 ? 1 : G == 8 ? 2 : 3; }

int alloc_bucket(Bucket& b, int G, long long cap) {
  b.G = G;
  b.cap = cap;
  const size_t rec = sizeof(double) * 2 * G;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  const size_t c = take(sizeof(Ctrl)), f0 = take(rec * cap), f1 = take(rec * cap), m0 = take(4 * cap),
               m1 = take(4 * cap), s0 = take(4 * cap), s1 = take(4 * cap);
  if (hipMalloc(&b.mem, o) != hipSuccess) {
    b.mem = nullptr;
    return IBB_ERR_NO_MEMORY;
  }
  b.bytes = o;
  char* w = static_cast<char*>(b.mem);
  b.ctrl = reinterpret_cast<Ctrl*>(w + c);
  b.front[0] = reinterpret_cast<double*>(w + f0);
  b.front[1] = reinterpret_cast<double*>(w + f1);
  b.meta[0] = reinterpret_cast<uint32_t*>(w + m0);
  b.meta[1] = reinterpret_cast<uint32_t*>(w + m1);
  b.sys[0] = reinterpret_cast<uint32_t*>(w + s0);
  b.sys[1] = reinterpret_cast<uint32_t*>(w + s1);
  if (hipMemset(b.ctrl, 0, sizeof(Ctrl)) != hipSuccess) return IBB_ERR_DEVICE;
  return IBB_OK;
}

// Moves a bucket to a frontier of new_cap boxes, keeping the boxes of its
// current level.
int grow_bucket(Bucket& b, long long new_cap, hipStream_t s) {
  Bucket nb;
  int st = alloc_bucket(nb, b.G, new_cap);
  if (st) return st;
  const int cur = b.level & 1;
  const size_t rec = sizeof(double) * 2 * b.G;
  if (hipMemcpyAsync(nb.ctrl, b.ctrl, sizeof(Ctrl), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(nb.front[cur], b.front[cur], rec * b.count, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(nb.meta[cur], b.meta[cur], 4 * b.count, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(nb.sys[cur], b.sys[cur], 4 * b.count, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return IBB_ERR_DEVICE;
  hipFree(b.mem);
  nb.level = b.level;
  nb.count = b.count;
  nb.slots = b.slots;
  b = nb;
  return IBB_OK;
}

int ensure_stage(ibb_server* sv, size_t need) {
  if (sv->stage_bytes >= need) return IBB_OK;
  need = std::max(need, sv->stage_bytes * 2);
  if (sv->h_stage) hipHostFree(sv->h_stage);
  if (sv->d_stage) hipFree(sv->d_stage);
  sv->h_stage = sv->d_stage = nullptr;
  sv->stage_bytes = 0;
  if (hipHostMalloc(reinterpret_cast<void**>(&sv->h_stage), need, hipHostMallocDefault) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&sv->d_stage), need) != hipSuccess)
    return IBB_ERR_NO_MEMORY;
  sv->stage_bytes = need;
  return IBB_OK;
}

// Pinned mirror of what a pass brings back: the four control blocks, then
// per slot the boxes still pending, the eight counters, the status, the
// emitted boxes and the level counts.
struct Back {
  Ctrl* ctrls;
  unsigned long long* pending;
  unsigned long long* stats;
  int* status;
  unsigned long long* emitted;
  unsigned long long* count_sys;
};

Back back_view(ibb_server* sv) {
  const int S = sv->cfg.max_slots;
  char* p = sv->h_back;
  Back b;
  b.ctrls = reinterpret_cast<Ctrl*>(p);
  p += round_up(4 * sizeof(Ctrl), 256);
  b.pending = reinterpret_cast<unsigned long long*>(p);
  p += round_up(8ull * S, 256);
  b.stats = reinterpret_cast<unsigned long long*>(p);
  p += round_up(64ull * S, 256);
  b.status = reinterpret_cast<int*>(p);
  p += round_up(4ull * S, 256);
  b.emitted = reinterpret_cast<unsigned long long*>(p);
  p += round_up(8ull * S, 256);
  b.count_sys = reinterpret_cast<unsigned long long*>(p);
  return b;
}

size_t back_size(int S) {
  return round_up(4 * sizeof(Ctrl), 256) + round_up(8ull * S, 256) + round_up(64ull * S, 256) +
         round_up(4ull * S, 256) + round_up(8ull * S, 256) + round_up(24ull * S, 256);
}

// Harvest after a pass: bucket levels and counts, then every solve without
// boxes left.  Returns the number harvested or a negative status.
int harvest(ibb_server* sv) {
  hipStream_t s = sv->ctx->stream;
  const Back bk = back_view(sv);
  for (int q = 0; q < 4; ++q) {
    Bucket& b = sv->bk[q];
    if (b.count == 0) continue;
    if (bk.ctrls[q].status != 0) return bk.ctrls[q].status;
    if ((int)bk.ctrls[q].levels > b.level) b.level = (int)bk.ctrls[q].levels;
    b.count = bk.ctrls[q].count[b.level % 3];
  }
  int finished = 0;
  for (int q = 0; q < 4; ++q) {
    Bucket& b = sv->bk[q];
    for (size_t i = 0; i < b.slots.size();) {
      const int slot = b.slots[i];
      if (bk.pending[slot] != 0) {
        ++i;
        continue;
      }
      Request* r = sv->by_slot[slot];
      const int n = r->comp.n;
      r->status = bk.status[slot];
      int64_t* f = &r->stats.processed;
      for (int k = 0; k < 8; ++k) f[k] = (int64_t)bk.stats[(size_t)slot * 8 + k];
      const long long m = (long long)bk.emitted[slot];
      if (r->status == IBB_OK && m > sv->cfg.out_cap_per_solve) r->status = IBB_ERR_OUTPUT_CAPACITY;
      if (r->status == IBB_OK && m > 0) {
        r->out_lo.resize((size_t)m * n);
        r->out_hi.resize((size_t)m * n);
        r->out_tag.resize((size_t)m);
        if (launch_slot_sort(s, sv->out_box, sv->out_tag, sv->slot_count, slot, sv->cfg.out_cap_per_solve, n,
                             sv->s_lo, sv->s_hi, sv->s_tag) != hipSuccess ||
            hipMemcpyAsync(r->out_lo.data(), sv->s_lo, sizeof(double) * m * n, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipMemcpyAsync(r->out_hi.data(), sv->s_hi, sizeof(double) * m * n, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipMemcpyAsync(r->out_tag.data(), sv->s_tag, (size_t)m, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return IBB_ERR_DEVICE;
      }
      r->state = 2;
      sv->by_slot[slot] = nullptr;
      sv->free_slots.push_back(slot);
      sv->reserved -= r->reserve_bytes;
      sv->finished.push_back(r->id);
      b.slots[i] = b.slots.back();
      b.slots.pop_back();
      ++finished;
    }
  }
  return finished;
}

}  // namespace

extern "C" {

void ibb_server_config_default(ibb_server_config* c) {
  if (!c) return;
  c->max_slots = 256;
  c->frontier_cap = 1 << 20;
  c->reserve_per_solve = 1 << 14;
  c->levels_per_quantum = 8;
  c->out_cap_per_solve = 1024;
  c->pool_bytes = 8ll << 30;
}

int ibb_server_create(ibb_ctx* ctx, const ibb_server_config* cfg, ibb_server** out) {
  if (!ctx || !out) return IBB_ERR_INVALID_ARG;
  *out = nullptr;
  ibb_server_config c;
  ibb_server_config_default(&c);
  if (cfg) c = *cfg;
  if (c.max_slots < 1 || c.frontier_cap < 16 || c.reserve_per_solve < 1 || c.levels_per_quantum < 1 ||
      c.out_cap_per_solve < 1 || c.reserve_per_solve > c.frontier_cap)
    return IBB_ERR_INVALID_ARG;
  size_t initial = 0;
  for (int q = 0; q < 4; ++q) initial += bucket_bytes(2 << q, c.frontier_cap);
  if (c.pool_bytes < (long long)initial) return IBB_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  ibb_server* sv = new (std::nothrow) ibb_server();
  if (!sv) return IBB_ERR_NO_MEMORY;
  sv->ctx = ctx;
  sv->cfg = c;
  const int S = c.max_slots;
  const long long oc = c.out_cap_per_solve;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  const size_t a_blobs = take(8ull * kSlotWords * S), a_boff = take(8ull * S), a_sp = take(sizeof(SysParams) * S),
               a_n = take(4ull * S), a_cs = take(8ull * 3 * S), a_cum = take(8ull * 2 * S),
               a_st = take(8ull * 8 * S), a_sc = take(8ull * S), a_ss = take(4ull * S),
               a_ob = take(sizeof(double) * 2 * kMaxN * oc * S), a_ot = take(4ull * oc * S),
               a_slo = take(sizeof(double) * kMaxN * oc), a_shi = take(sizeof(double) * kMaxN * oc),
               a_stag = take((size_t)oc), a_lv = take(sizeof(long long) * kLevelCap), a_pd = take(8ull * S),
               a_ev = take((size_t)S);
  if (hipMalloc(&sv->mem, o) != hipSuccess) {
    delete sv;
    return IBB_ERR_NO_MEMORY;
  }
  char* w = static_cast<char*>(sv->mem);
  sv->blobs = reinterpret_cast<uint64_t*>(w + a_blobs);
  sv->boff = reinterpret_cast<long long*>(w + a_boff);
  sv->sp = reinterpret_cast<SysParams*>(w + a_sp);
  sv->nsys = reinterpret_cast<int*>(w + a_n);
  sv->count_sys = reinterpret_cast<unsigned long long*>(w + a_cs);
  sv->cum_sys = reinterpret_cast<unsigned long long*>(w + a_cum);
  sv->stats_sys = reinterpret_cast<unsigned long long*>(w + a_st);
  sv->slot_count = reinterpret_cast<unsigned long long*>(w + a_sc);
  sv->status_sys = reinterpret_cast<int*>(w + a_ss);
  sv->out_box = reinterpret_cast<double*>(w + a_ob);
  sv->out_tag = reinterpret_cast<uint32_t*>(w + a_ot);
  sv->s_lo = reinterpret_cast<double*>(w + a_slo);
  sv->s_hi = reinterpret_cast<double*>(w + a_shi);
  sv->s_tag = reinterpret_cast<uint8_t*>(w + a_stag);
  sv->level_sizes = reinterpret_cast<long long*>(w + a_lv);
  sv->pending = reinterpret_cast<unsigned long long*>(w + a_pd);
  sv->evict = reinterpret_cast<uint8_t*>(w + a_ev);
  std::vector<long long> boff((size_t)S);
  for (int i = 0; i < S; ++i) boff[i] = (long long)i * kSlotWords;
  int st = IBB_OK;
  if (hipMemset(sv->mem, 0, o) != hipSuccess ||
      hipMemcpy(sv->boff, boff.data(), 8ull * S, hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreateWithFlags(&sv->pass_done, hipEventDisableTiming) != hipSuccess)
    st = IBB_ERR_DEVICE;
  sv->back_bytes = back_size(S);
  if (!st && hipHostMalloc(reinterpret_cast<void**>(&sv->h_back), sv->back_bytes, hipHostMallocDefault) != hipSuccess)
    st = IBB_ERR_NO_MEMORY;
  for (int q = 0; q < 4 && !st; ++q) {
    st = alloc_bucket(sv->bk[q], 2 << q, c.frontier_cap);
    sv->pool_used += sv->bk[q].bytes;
  }
  if (st) {
    ibb_server_destroy(sv);
    return st;
  }
  sv->by_slot.assign((size_t)S, nullptr);
  for (int i = S - 1; i >= 0; --i) sv->free_slots.push_back(i);
  *out = sv;
  return IBB_OK;
}

void ibb_server_destroy(ibb_server* sv) {
  if (!sv) return;
  hipSetDevice(sv->ctx->device);
  hipStreamSynchronize(sv->ctx->stream);
  for (auto& b : sv->bk)
    if (b.mem) hipFree(b.mem);
  if (sv->mem) hipFree(sv->mem);
  if (sv->d_stage) hipFree(sv->d_stage);
  if (sv->h_stage) hipHostFree(sv->h_stage);
  if (sv->h_back) hipHostFree(sv->h_back);
  if (sv->pass_done) hipEventDestroy(sv->pass_done);
  for (auto& kv : sv->reqs) delete kv.second;
  delete sv;
}

int64_t ibb_server_submit(ibb_server* sv, const ibb_system* sys, const double* lo, const double* hi,
                          const ibb_params* params) {
  if (!sv) return IBB_ERR_INVALID_ARG;
  const int st = validate(sys, lo, hi, params);
  if (st) return st;
  if (params->split_mode != IBB_SPLIT_WIDEST) return IBB_ERR_UNSUPPORTED;
  Request* r = new (std::nothrow) Request();
  if (!r) return IBB_ERR_NO_MEMORY;
  try {
    compile(sys, r->comp);
  } catch (...) {
    delete r;
    return IBB_ERR_NO_MEMORY;
  }
  if (r->comp.blob.size() > (size_t)kSlotWords) {
    delete r;
    return IBB_ERR_UNSUPPORTED;
  }
  r->id = sv->next_id++;
  std::memcpy(r->lo, lo, sizeof(double) * sys->n);
  std::memcpy(r->hi, hi, sizeof(double) * sys->n);
  r->p = *params;
  r->reserve_boxes = reserve_for(*r, sv->cfg.reserve_per_solve);
  r->reserve_bytes = bucket_bytes(r->comp.G, 2 * r->reserve_boxes) - 4096;
  if ((long long)r->reserve_bytes > sv->cfg.pool_bytes) r->reserve_bytes = (size_t)sv->cfg.pool_bytes;
  sv->queue.push_back(r);
  sv->reqs[r->id] = r;
  return r->id;
}

int ibb_server_cancel(ibb_server* sv, int64_t id) {
  if (!sv) return IBB_ERR_INVALID_ARG;
  auto it = sv->reqs.find(id);
  if (it == sv->reqs.end()) return IBB_ERR_INVALID_ARG;
  Request* r = it->second;
  if (r->state != 0) return IBB_ERR_UNSUPPORTED;  // only queued requests can be cancelled
  sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), r));
  sv->reqs.erase(it);
  delete r;
  return IBB_OK;
}

int ibb_server_pending(ibb_server* sv, int64_t* queued, int64_t* active) {
  if (!sv) return IBB_ERR_INVALID_ARG;
  if (queued) *queued = (int64_t)sv->queue.size();
  if (active) *active = (int64_t)(sv->cfg.max_slots - (int)sv->free_slots.size());
  return IBB_OK;
}

int64_t ibb_server_finished(ibb_server* sv, int64_t* ids, int64_t cap) {
  if (!sv || cap < 0 || (cap > 0 && !ids)) return IBB_ERR_INVALID_ARG;
  const int64_t m = std::min<int64_t>(cap, (int64_t)sv->finished.size());
  std::copy(sv->finished.begin(), sv->finished.begin() + m, ids);
  sv->finished.erase(sv->finished.begin(), sv->finished.begin() + m);
  return m;
}

int ibb_server_step(ibb_server* sv) {
  if (!sv) return IBB_ERR_INVALID_ARG;
  ibb_ctx* ctx = sv->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return IBB_ERR_DEVICE;
  hipStream_t s = ctx->stream;
  const int S = sv->cfg.max_slots;
  // ---- (1) the pass in flight: wait for it, harvest
  int finished = 0;
  if (sv->in_flight) {
    if (hipEventSynchronize(sv->pass_done) != hipSuccess) return IBB_ERR_DEVICE;
    sv->in_flight = false;
    finished = harvest(sv);
    if (finished < 0) return finished;
  }
  const Back bk = back_view(sv);
  // ---- (2) admission: a free slot and the request's reservation within the pool
  std::vector<Request*> admitted;
  for (auto it = sv->queue.begin(); it != sv->queue.end() && !sv->free_slots.empty();) {
    Request* r = *it;
    if (sv->reserved + r->reserve_bytes > (size_t)sv->cfg.pool_bytes) {
      ++it;
      continue;
    }
    it = sv->queue.erase(it);
    r->slot = sv->free_slots.back();
    sv->free_slots.pop_back();
    r->bucket = bucket_of(r->comp.G);
    r->state = 1;
    sv->reserved += r->reserve_bytes;
    sv->bk[r->bucket].slots.push_back(r->slot);
    sv->by_slot[r->slot] = r;
    admitted.push_back(r);
  }
  // room for the admitted roots (one box each) in their buckets' levels
  long long add[4] = {0, 0, 0, 0};
  for (Request* r : admitted) ++add[r->bucket];
  // ---- (3) room for the next levels: grow within the pool, else fail the
  // solves that outgrew their reservation the most (their boxes are dropped
  // when the next pass loads them; they end with IBB_ERR_QUEUE_OVERFLOW)
  std::vector<int> evicted;
  long long live[4];
  for (int q = 0; q < 4; ++q) {
    Bucket& b = sv->bk[q];
    const unsigned long long cur = b.count + (unsigned long long)add[q];
    live[q] = (long long)cur;
    if (cur == 0) continue;
    if ((long long)cur * 2 <= b.cap && b.cap >= (long long)cur) continue;
    const long long want = std::max<long long>(b.cap * 4, (long long)cur * 2);
    long long fit = want;
    const size_t others = sv->pool_used - b.bytes;
    while (fit > b.cap && others + bucket_bytes(b.G, fit) > (size_t)sv->cfg.pool_bytes) fit = fit * 3 / 4;
    if (fit >= (long long)cur * 2 && fit > b.cap) {
      const int st = grow_bucket(b, fit, s);
      if (st) return st;
      sv->pool_used = others + b.bytes;
      continue;
    }
    // evict: boxes of this level per slot beyond the slot's reservation
    std::vector<std::pair<long long, int>> over;
    for (int slot : b.slots) {
      const Request* r = sv->by_slot[slot];
      const long long c = r->state == 1 && std::find(admitted.begin(), admitted.end(), r) == admitted.end()
                              ? (long long)bk.count_sys[(size_t)(b.level % 3) * S + slot]
                              : 1;
      over.push_back({c - r->reserve_boxes, slot});
    }
    std::sort(over.begin(), over.end(), [](auto& x, auto& y) { return x.first > y.first; });
    for (const auto& e : over) {
      if (live[q] * 2 <= b.cap) break;
      const long long c = e.first + sv->by_slot[e.second]->reserve_boxes;
      evicted.push_back(e.second);
      live[q] -= c;
    }
  }
  // ---- upload: admission records, compiled systems, evicted slots
  size_t words = 0;
  for (Request* r : admitted) words += r->comp.blob.size();
  const size_t recs_at = 0, payload_at = round_up(sizeof(AdmitRec) * admitted.size(), 256),
               evict_at = payload_at + round_up(8 * words, 256), boff_at = evict_at + round_up(4 * evicted.size(), 256),
               need = boff_at + round_up(8 * admitted.size(), 256) + 256;
  if (!admitted.empty() || !evicted.empty()) {
    int st = ensure_stage(sv, need);
    if (st) return st;
    AdmitRec* recs = reinterpret_cast<AdmitRec*>(sv->h_stage + recs_at);
    uint64_t* payload = reinterpret_cast<uint64_t*>(sv->h_stage + payload_at);
    long long* boff = reinterpret_cast<long long*>(sv->h_stage + boff_at);
    size_t w = 0;
    for (size_t k = 0; k < admitted.size(); ++k) {
      Request* r = admitted[k];
      Bucket& b = sv->bk[r->bucket];
      AdmitRec& a = recs[k];
      std::memset(&a, 0, sizeof a);
      a.slot = r->slot;
      a.n = r->comp.n;
      a.G = b.G;
      a.nwords = (int32_t)r->comp.blob.size();
      a.blob_at = (long long)w;
      std::memcpy(payload + w, r->comp.blob.data(), 8 * r->comp.blob.size());
      w += r->comp.blob.size();
      a.sp = SysParams{r->p.tol, r->p.recontract_ratio, r->p.hs_max_width, r->p.max_boxes, r->p.split_mode,
                       r->p.max_recontract, r->p.contractor, r->p.inclusion};
      const int L = b.level;
      a.front = b.front[L & 1];
      a.meta = b.meta[L & 1];
      a.sys = b.sys[L & 1];
      a.pos = (long long)b.count;
      b.count += 1;
      a.ctrl = b.ctrl;
      a.new_count = b.count;
      a.level_slot = L % 3;
      for (int i = 0; i < r->comp.n; ++i) {
        a.lo[i] = r->lo[i];
        a.hi[i] = r->hi[i];
      }
      boff[k] = (long long)r->slot * kSlotWords;
    }
    // the last admission of each bucket sets the bucket's level count
    for (size_t k = admitted.size(); k-- > 0;) {
      bool later = false;
      for (size_t j = k + 1; j < admitted.size(); ++j) later = later || admitted[j]->bucket == admitted[k]->bucket;
      recs[k].set_count = later ? 0 : 1;
    }
    int* ev = reinterpret_cast<int*>(sv->h_stage + evict_at);
    for (size_t k = 0; k < evicted.size(); ++k) ev[k] = evicted[k];
    if (hipMemcpyAsync(sv->d_stage, sv->h_stage, need, hipMemcpyHostToDevice, s) != hipSuccess) return IBB_ERR_DEVICE;
    if (!admitted.empty()) {
      if (launch_admit(s, reinterpret_cast<const AdmitRec*>(sv->d_stage + recs_at), (int)admitted.size(),
                       reinterpret_cast<const uint64_t*>(sv->d_stage + payload_at), sv->blobs, kSlotWords, sv->sp,
                       sv->nsys, sv->status_sys, sv->evict, sv->stats_sys, sv->slot_count, sv->cum_sys,
                       sv->pending, sv->count_sys, S) != hipSuccess ||
          launch_prep(s, sv->blobs, reinterpret_cast<const long long*>(sv->d_stage + boff_at), (int)admitted.size()) !=
              hipSuccess)
        return IBB_ERR_DEVICE;
    }
    if (!evicted.empty() && launch_evict(s, reinterpret_cast<const int*>(sv->d_stage + evict_at), (int)evicted.size(),
                                         sv->evict, sv->status_sys, IBB_ERR_QUEUE_OVERFLOW) != hipSuccess)
      return IBB_ERR_DEVICE;
  }
  // ---- (4) one pass of levels per bucket, then the counters back to the host
  bool any = false;
  ctx->tune_pending = false;
  hipEventRecord(ctx->ev0, s);
  for (int q = 0; q < 4; ++q) {
    Bucket& b = sv->bk[q];
    if (b.count == 0) continue;
    // at most two children per box per level (widest split): keep the frontier
    // within capacity for the whole pass
    int K = sv->cfg.levels_per_quantum;
    const double lv = (double)std::max<long long>(live[q], 1);
    while (K > 1 && lv * (double)(1ull << K) > (double)b.cap) --K;
    SolveArgs a;
    std::memset(&a, 0, sizeof a);
    a.front[0] = b.front[0];
    a.front[1] = b.front[1];
    a.meta[0] = b.meta[0];
    a.meta[1] = b.meta[1];
    a.sys[0] = b.sys[0];
    a.sys[1] = b.sys[1];
    a.front_cap = b.cap;
    a.out_box = sv->out_box;
    a.out_tag = sv->out_tag;
    a.out_stride = kMaxN;
    a.slot_out_cap = sv->cfg.out_cap_per_solve;
    a.slot_out_count = sv->slot_count;
    a.ctrl = b.ctrl;
    a.level_sizes = sv->level_sizes;
    a.level_cap = 0;
    a.max_boxes = 1LL << 62;
    a.max_levels = K;
    a.level0 = b.level;
    a.timeout_ticks = ctx->clock_khz * 1000LL * 20;
    a.blobs = sv->blobs;
    a.blob_off = sv->boff;
    a.sp = sv->sp;
    a.count_sys = sv->count_sys;
    a.cum_sys = sv->cum_sys;
    a.status_sys = sv->status_sys;
    a.stats_sys = sv->stats_sys;
    a.pending_sys = sv->pending;
    a.evict = sv->evict;
    a.B = S;
    // the Jacobian scratch fits the largest system of the bucket's active slots
    int jn = 0;
    for (int slot : b.slots) jn = std::max(jn, sv->by_slot[slot]->comp.n);
    const void* fn = solve_kernel_ptr(b.G, true, true);
    Geometry geo;
    const int st = persistent_geometry(ctx, fn, 0, b.G, jn, &geo);
    if (st) return st;
    a.nblocks = geo.blocks;
    a.jrs = geo.jrs;
    a.jn = jn;
    // the grid barrier counts arrivals from zero in every pass
    if (launch_fill_u64(s, &b.ctrl->bar, 1, 0ull) != hipSuccess ||
        launch_fill_u64(s, b.ctrl->sync, (long long)(sizeof(b.ctrl->sync) / 8), 0ull) != hipSuccess)
      return IBB_ERR_DEVICE;
    void* args[] = {&a};
    if (hipLaunchCooperativeKernel(fn, dim3(geo.blocks), dim3(64 * geo.waves), args, (unsigned)geo.lds, s) !=
        hipSuccess)
      return IBB_ERR_DEVICE;
    any = true;
  }
  hipEventRecord(ctx->ev1, s);
  ctx->timed_pending = any;
  if (any) {
    const Back back = back_view(sv);
    for (int q = 0; q < 4; ++q)
      if (hipMemcpyAsync(&back.ctrls[q], sv->bk[q].ctrl, kCtrlCounterBytes, hipMemcpyDeviceToHost, s) != hipSuccess)
        return IBB_ERR_DEVICE;
    if (hipMemcpyAsync(back.pending, sv->pending, 8ull * S, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(back.stats, sv->stats_sys, 64ull * S, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(back.status, sv->status_sys, 4ull * S, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(back.emitted, sv->slot_count, 8ull * S, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(back.count_sys, sv->count_sys, 24ull * S, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(sv->pass_done, s) != hipSuccess)
      return IBB_ERR_DEVICE;
    sv->in_flight = true;
    // with nothing waiting for admission there is no host work to overlap:
    // harvest this pass at once (its solves finish one round earlier)
    if (sv->queue.empty()) {
      if (hipEventSynchronize(sv->pass_done) != hipSuccess) return IBB_ERR_DEVICE;
      sv->in_flight = false;
      const int more = harvest(sv);
      if (more < 0) return more;
      finished += more;
    }
  }
  return finished;
}

int ibb_server_poll(ibb_server* sv, int64_t id, double* out_lo, double* out_hi, uint8_t* out_tag, int64_t cap,
                    int64_t* n_out, int32_t* status, ibb_stats* stats) {
  if (!sv || !n_out || !status) return IBB_ERR_INVALID_ARG;
  auto it = sv->reqs.find(id);
  if (it == sv->reqs.end()) return IBB_ERR_INVALID_ARG;
  Request* r = it->second;
  if (r->state != 2) return 1;  // not finished yet
  const int64_t m = (int64_t)r->out_tag.size();
  *n_out = m;
  *status = r->status;
  if (stats) *stats = r->stats;
  if (m > cap) return IBB_ERR_OUTPUT_CAPACITY;
  if (m) {
    std::memcpy(out_lo, r->out_lo.data(), sizeof(double) * r->out_lo.size());
    std::memcpy(out_hi, r->out_hi.data(), sizeof(double) * r->out_hi.size());
    std::memcpy(out_tag, r->out_tag.data(), (size_t)m);
  }
  sv->reqs.erase(it);
  delete r;
  return IBB_OK;
}

}  // extern "C"
