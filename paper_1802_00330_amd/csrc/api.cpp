// api.cpp -- host runtime behind include/ibb.h: validation, system compilation,
// device memory, launches and result collection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ibb.h"
#include "layout.hpp"

namespace ibb {
// kernels.hip
size_t scratch_bytes(int G);
const void* solve_kernel_ptr(int G);
hipError_t launch_init(hipStream_t s, Ctrl* c, double* front0, uint32_t* meta0, const double* lo,
                       const double* hi, int n, int G);
hipError_t launch_sort(hipStream_t s, const double* box, const uint32_t* tag, const Ctrl* c, int n, int G,
                       long long out_cap, double* out_lo, double* out_hi, uint8_t* out_tag,
                       long long grid_elems);
hipError_t launch_finalize(hipStream_t s, const Ctrl* c, long long out_cap, long long* info);
hipError_t launch_selftest(hipStream_t s, int op, long long count, const double* x, const double* y,
                           double* out);
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
  size_t ctrl, level, blob, box, front0, front1, meta0, meta1, out_box, out_tag, total;
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
  L.total = o;
  return L;
}

// Upper bound of the system blob size for a given n (IBB_MAX_TERMS terms).
size_t max_blob_words(int n) {
  const size_t T = IBB_MAX_TERMS, TD = (size_t)IBB_MAX_TERMS * IBB_MAX_DEG;
  return sizeof(SysDesc) / 8 + (n + 2) / 2 + (n * n + 2) / 2 + 2 * T + 2 * TD + (TD + 1) / 2 + 8;
}

}  // namespace

struct ibb_ctx {
  int device = 0;
  int num_cu = 0;
  size_t max_lds_block = 0;
  long long clock_khz = 100000;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, staged = nullptr;
  bool staged_pending = false;
  bool timed_pending = false;  // ev0/ev1 bracket the last persistent launch
  void* ws = nullptr;  // workspace of the host-pointer entry points
  size_t ws_bytes = 0;
  double* sorted = nullptr;  // sorted outputs of ibb_solve (lo, hi, tag)
  size_t sorted_bytes = 0;
  long long* info = nullptr;
  char* pinned = nullptr;  // host staging of the inputs
  size_t pinned_bytes = 0;
  std::vector<long long> last_levels;
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

// Enqueue one solve into a partitioned workspace; outputs to device arrays.
int enqueue_solve(ibb_ctx* ctx, const Compiled& c, const double* lo, const double* hi,
                  const ibb_params* p, char* ws, const WsLayout& L, long long frontier_cap,
                  long long out_cap, double* d_out_lo, double* d_out_hi, uint8_t* d_out_tag,
                  long long* d_info, hipStream_t s) {
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

  Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  const double* dlo = reinterpret_cast<const double*>(ws + L.box);
  if (launch_init(s, ctrl, reinterpret_cast<double*>(ws + L.front0), reinterpret_cast<uint32_t*>(ws + L.meta0),
                  dlo, dlo + kMaxN, n, G) != hipSuccess)
    return IBB_ERR_DEVICE;

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
  a.max_boxes = p->max_boxes;
  a.split_mode = p->split_mode;
  a.max_rc = p->max_recontract;
  a.timeout_ticks = ctx->clock_khz * 1000LL * 20;  // 20 s per barrier wait

  const void* fn = solve_kernel_ptr(G);
  const size_t tbytes = (table_lds_bytes(n, c.T, c.TD) + 15) & ~size_t(15);
  const size_t per_wave = scratch_bytes(G);
  int waves = 4;
  while (waves > 1 && tbytes + per_wave * waves > ctx->max_lds_block) --waves;
  const size_t lds = tbytes + per_wave * waves;
  if (lds > ctx->max_lds_block) return IBB_ERR_UNSUPPORTED;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return IBB_ERR_DEVICE;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * waves, lds) != hipSuccess || per_cu < 1)
    return IBB_ERR_UNSUPPORTED;
  const int blocks = per_cu * ctx->num_cu;
  a.nblocks = blocks;
  void* args[] = {&a};
  hipEventRecord(ctx->ev0, s);
  if (hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(64 * waves), args, (unsigned)lds, s) != hipSuccess)
    return IBB_ERR_DEVICE;
  hipEventRecord(ctx->ev1, s);
  ctx->timed_pending = true;
  if (launch_sort(s, a.out_box, a.out_tag, ctrl, n, G, out_cap, d_out_lo, d_out_hi, d_out_tag, out_cap) !=
      hipSuccess)
    return IBB_ERR_DEVICE;
  if (launch_finalize(s, ctrl, out_cap, d_info) != hipSuccess) return IBB_ERR_DEVICE;
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
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    c->clock_khz = khz;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&c->info), sizeof(long long) * kInfoLen) != hipSuccess) {
    ibb_ctx_destroy(c);
    return IBB_ERR_DEVICE;
  }
  *out = c;
  return IBB_OK;
}

void ibb_ctx_destroy(ibb_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  if (c->ws) hipFree(c->ws);
  if (c->sorted) hipFree(c->sorted);
  if (c->info) hipFree(c->info);
  if (c->pinned) hipHostFree(c->pinned);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  if (c->staged) hipEventDestroy(c->staged);
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
