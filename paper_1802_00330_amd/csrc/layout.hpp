// layout.hpp -- data layouts shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ibb {

constexpr int kMaxN = 16;
constexpr int kBlock = 256;  // threads per workgroup (4 waves of 64)
constexpr int kInfoLen = 16;
constexpr int kStageWaves = 256 * 32;  // waves a persistent launch may have (CUs x waves per CU)

// Compiled system, one contiguous blob of 8-byte words in device memory:
//   [0, 16)           SysDesc
//   eq_off            int32 [n+1]        terms of equation i: eq_off[i] .. eq_off[i+1]-1
//   der_off           int32 [n*n+1]      derivative terms of (i,k): der_off[i*n+k] ..
//   coef              double [T]         term coefficients
//   fac               uint64 [T]         factors, byte q = (pow << 4) | var, var ascending, 0 ends
//   dcoef             double [TD]        coefficient c of the parent term
//   dmult             uint32 [TD]        exponent e_k of the differentiated variable
//   dfac              uint64 [TD]        factors of the lowered monomial (may be 0 = constant)
// Offsets are in 8-byte words from the start of the blob.
struct SysDesc {
  int32_t n, G, T, TD;
  int32_t eq_off_w, der_off_w, coef_w, fac_w;
  int32_t dcoef_w, dmult_w, dfac_w, total_w;
  uint32_t jnz[kMaxN];  // bit k of jnz[i]: d f_i / d x_k has at least one term
  int32_t dco_w;        // [TD][2] enclosure (lo, -hi) of e_k * c, filled on the device
  int32_t pad[3];
};
static_assert(sizeof(SysDesc) == 128, "SysDesc size");

// Control block of one solve (device memory, zero-initialised by the host
// except count[0] = 1).
// Grid barrier: groups of workgroups and the u64 stride of their lines.
constexpr int kSyncGroups = 8;
constexpr int kSyncStride = 16;

// The counters that the waves of a launch update all the time (a level's
// pushes and claims; the work queue's claims, reservations and pending
// count) each have a 256-byte block of their own: device-scope atomics on one
// block are serialised at the one place where the eight XCDs meet, so
// counters sharing a block queue behind each other's updates.
constexpr int kHotU64 = 32;

struct Ctrl {
  unsigned long long count[3];   // frontier size of level L in count[L % 3]
  unsigned long long pad_count[kHotU64 - 3];
  unsigned long long claim[3];   // next unclaimed box of level L in claim[L % 3]
  unsigned long long pad_claim[kHotU64 - 3];
  // work-queue search (one system): monotone claim and reservation counters of
  // the ring (qtail = boxes created, the budget), boxes created and not yet stepped
  unsigned long long qhead;
  unsigned long long pad_qhead[kHotU64 - 1];
  unsigned long long qtail;
  unsigned long long pad_qtail[kHotU64 - 1];
  unsigned long long pending;
  unsigned long long pad_pending[kHotU64 - 1];
  unsigned long long out_count;  // emitted boxes
  unsigned long long bar;        // grid barrier: arrivals of the last of each group (monotone)
  unsigned long long stats[8];   // processed, excluded_eval, excluded_hs, hs_skipped,
                                 // recontracted, bisected, emitted_unique, emitted_undecided
  unsigned long long levels;
  unsigned long long max_frontier;
  int32_t status;
  int32_t pad[39];  // the block of the other counters ends at 256 bytes
  // grid barrier of a persistent launch (zero at launch): the arrivals of each
  // group of workgroups (blockIdx % 8) and each group's release flag, each in
  // a 128-byte line of its own
  unsigned long long sync[2 * kSyncGroups * kSyncStride];
};
static_assert(offsetof(Ctrl, claim) == 8 * kHotU64 && offsetof(Ctrl, qhead) == 16 * kHotU64 &&
                  offsetof(Ctrl, qtail) == 24 * kHotU64 && offsetof(Ctrl, pending) == 32 * kHotU64 &&
                  offsetof(Ctrl, out_count) == 40 * kHotU64,
              "hot counters of Ctrl in blocks of their own");
static_assert(offsetof(Ctrl, sync) == 48 * kHotU64 && sizeof(Ctrl) % 256 == 0, "Ctrl lines");

// Bytes of a Ctrl before its barrier lines (the counters a host reads back).
constexpr size_t kCtrlCounterBytes = offsetof(Ctrl, sync);

// Status a search kernel records when it finds the FP64 rounding mode of its
// wave changed (reported to the caller as IBB_ERR_DEVICE).
constexpr int kStatusModeLost = -6;

// Per-system search parameters of a batch (ibb_params in device form).
struct SysParams {
  double tol, ratio, hs_max_width;
  long long max_boxes;
  int split_mode, max_rc;
  int contractor, inclusion;
};

struct SolveArgs {
  const uint64_t* blob;
  double* front[2];  // boxes as (lo, -hi) pairs, [cap][G][2]
  uint32_t* meta[2]; // bit 0 proven, bits 8..15 consecutive re-contractions,
                     // bits 16..31 depth in the tree (work-queue search)
  long long front_cap;
  double* out_box;   // [out_cap][G][2]
  uint32_t* out_tag;
  long long out_cap;
  Ctrl* ctrl;
  long long* level_sizes;
  long long level_cap;
  double tol, ratio, hs_max_width;
  long long max_boxes;
  int split_mode, max_rc;
  int contractor;  // 0 Hansen-Sengupta, 1 Krawczyk
  int inclusion;   // 0 natural extension, 1 also the mean-value form
  int nblocks;
  int max_levels;           // stop after this many levels (0 = until the tree ends)
  long long timeout_ticks;  // device wall-clock ticks (100 MHz) a barrier may wait
  double* dbg;              // diagnostics: intermediates of box 0 of level 0 (or null)
  unsigned long long* out_count;  // emitted boxes (shared by the launches of a batch)
  // batches of systems (null for a single system)
  uint32_t* sys[2];               // system index of each frontier record
  const uint64_t* blobs;          // all compiled systems
  const long long* blob_off;      // [B] word offset of each system's blob
  const SysParams* sp;            // [B]
  unsigned long long* count_sys;  // [3][B] boxes of system s at level L in slot L % 3
  unsigned long long* cum_sys;    // [2][B] tree nodes of s through level L in slot L % 2
  int* status_sys;                // [B]
  unsigned long long* stats_sys;  // [B][8]
  uint32_t* out_sys;              // [out_cap] system of each emitted box
  int B;
  int out_stride;  // coordinates per output record (G for one system, kMaxN for batches)
  int level0;      // index of the first level of this launch (continuing searches)
  int jrs;         // row stride (in intervals) of the per-box Jacobian in LDS
  int jn;          // rows of the per-box Jacobian in LDS (batches: the largest n among the members)
  int tiles_per_claim;  // batches: tiles a wave claims per atomic (values below 1 act as 1)
  // work-queue search: front[0]/meta[0] form a ring of front_cap (a power of
  // two) slots; qseq[s] = t: slot free for item t, t + 1: slot holds item t
  unsigned long long* qseq;
  // one system: per wave, a ring of 2W screened boxes ([2W][G][2] doubles and
  // [2W] records), indexed by the wave's global number
  double* stage_box;
  uint32_t* stage_meta;
  int slot_out_cap;  // > 0: each system emits into its own region of this many boxes
  unsigned long long* slot_out_count;  // [B] boxes emitted per system (regions)
  unsigned long long* pending_sys;     // [B] boxes per system still to step (or null)
  const uint8_t* evict;                // [B] nonzero: the system's boxes are dropped when loaded (or null)
};

// Serving: admission record of one request, uploaded with the others of its
// scheduling round; the admission kernel installs the request in its slot and
// appends its initial box to its bucket's current level.
struct AdmitRec {
  int32_t slot, n, G, nwords;
  long long blob_at;  // word offset of the compiled system in the round's payload
  SysParams sp;
  double* front;      // the bucket's current level; the initial box goes to index pos
  uint32_t* meta;
  uint32_t* sys;
  long long pos;
  Ctrl* ctrl;         // with set_count: the bucket's count of that level becomes new_count
  unsigned long long new_count;
  int32_t level_slot, set_count;
  double lo[kMaxN], hi[kMaxN];
};

// Layout of the diagnostic dump of one step (doubles), n = system size:
//   J [n][n][2] (lo, hi) | F(x) [n][2] | single-precision mid J [n][n] |
//   Y [n][n] (row = logical position) | g [n][2] | P [n][n][2] | N [n][2] |
//   X' [n][2] | flags [4]: skipped, empty, unique, ran
__host__ __device__ inline int dbg_off_J(int) { return 0; }
__host__ __device__ inline int dbg_off_F(int n) { return 2 * n * n; }
__host__ __device__ inline int dbg_off_M(int n) { return 2 * n * n + 2 * n; }
__host__ __device__ inline int dbg_off_Y(int n) { return 3 * n * n + 2 * n; }
__host__ __device__ inline int dbg_off_g(int n) { return 4 * n * n + 2 * n; }
__host__ __device__ inline int dbg_off_P(int n) { return 4 * n * n + 4 * n; }
__host__ __device__ inline int dbg_off_N(int n) { return 6 * n * n + 4 * n; }
__host__ __device__ inline int dbg_off_X(int n) { return 6 * n * n + 6 * n; }
__host__ __device__ inline int dbg_off_flags(int n) { return 6 * n * n + 8 * n; }
__host__ __device__ inline int dbg_len(int n) { return 6 * n * n + 8 * n + 4; }

// LDS bytes of the staged system table (kernels.hip, stage_table).
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline size_t table_lds_bytes(int n, int T, int TD) {
  return align16(sizeof(int) * (n + 1)) + align16(sizeof(int) * (n * n + 1)) +
         align16(sizeof(uint32_t) * kMaxN) + align16(sizeof(double) * T) + align16(sizeof(uint64_t) * T) +
         align16(16 * (size_t)TD) + align16(sizeof(uint64_t) * TD);
}

}  // namespace ibb
