/*
 * ibb.h -- rigorous interval branch-and-bound for square polynomial systems on
 * a box, with the Hansen-Sengupta contraction, on AMD Instinct MI355X (gfx950).
 *
 * Method: Lin & Chen, "An efficient algorithm for global interval solution of
 * nonlinear algebraic equations and its GPGPU implementation" (arXiv
 * 1802.00330).  Problem statement and outputs: Sec. 3.1, Alg. 1 (input: the
 * equations, the variable ranges, the desired width; output: the boxes that may
 * hold solutions).  Per box: interval evaluation and the exclusion test
 * (Sec. 2.2, Def. 1-2; Alg. 2), the Hansen-Sengupta step (Sec. 2.3 eq 17-22;
 * Alg. 3-4) and bisection (Alg. 2).  A box whose contraction lands strictly
 * inside it holds exactly one root (Alg. 3, second output) and is tagged
 * IBB_UNIQUE.
 *
 * Conventions for every entry point:
 *  - All pointers are plain host pointers unless the name starts with d_
 *    (device memory on the context's GPU).  Inputs are borrowed for the call;
 *    for *_async calls, until the work enqueued on the stream has completed.
 *  - The library never frees memory it did not allocate.  A context owns its
 *    internal buffers; one context per host thread.
 *  - Every call returns an int status (IBB_OK or a negative IBB_ERR_*); no C++
 *    exception crosses this interface.  On error, outputs are unspecified
 *    except where stated.
 *  - Results are deterministic: each box's fate depends only on the box, so the
 *    sorted output list and the counters do not depend on scheduling.
 */
#ifndef IBB_H
#define IBB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define IBB_OK 0
#define IBB_ERR_INVALID_ARG (-1)     /* malformed system, box or parameters            */
#define IBB_ERR_BUDGET (-2)          /* the search tree has more than max_boxes nodes  */
#define IBB_ERR_OUTPUT_CAPACITY (-3) /* more boxes than `cap`; *n_out = required count */
#define IBB_ERR_QUEUE_OVERFLOW (-4)  /* a tree level exceeded the frontier capacity    */
#define IBB_ERR_NO_MEMORY (-5)       /* device or host allocation failed               */
#define IBB_ERR_DEVICE (-6)          /* a HIP runtime call failed, or a search kernel
                                        found its FP64 rounding mode changed          */
#define IBB_ERR_UNSUPPORTED (-7)     /* valid request outside this build's limits      */
#define IBB_ERR_TIMEOUT (-8)         /* a device-side wait exceeded its time limit     */
#define IBB_ERR_WORKSPACE_LIMIT (-9) /* ibb_solve_noalloc: workspace above its maximum */

/* ---- limits ---- */
#define IBB_MAX_N 16      /* equations = variables                        */
#define IBB_MAX_DEG 8     /* total degree of a term                       */
#define IBB_MAX_TERMS 4096/* terms per system                             */

/* ---- tags of output boxes ---- */
#define IBB_UNDECIDED 0   /* may hold roots (width reached or split exhausted) */
#define IBB_UNIQUE 1      /* holds exactly one root (Alg. 3, second output)    */

/* ---- bisection ---- */
#define IBB_SPLIT_WIDEST 0 /* bisect the widest coordinate (first on ties) */
#define IBB_SPLIT_ALL 1    /* bisect every coordinate: 2^n children (Alg. 2) */

/* Order in which ibb_solve / ibb_solve_async step the boxes of the tree.  The
 * tree, its counters, the status and the sorted output are the same in both.
 * IBB_SCHEDULE_QUEUE: a device work queue, each box stepped as soon as it is
 * created (no wait at the end of a round).  IBB_SCHEDULE_LEVELS: round by
 * round as in Alg. 1, all boxes of round k before any of round k + 1; with a
 * budget error the per-level sizes then cover every completed round. */
#define IBB_SCHEDULE_QUEUE 0
#define IBB_SCHEDULE_LEVELS 1
/* IBB_SCHEDULE_AUTO (default): per system shape (n, terms, derivative terms,
 * split mode, contractor, inclusion) the context times the search kernel
 * twice with each schedule (the first launch on fresh device memory runs
 * slower than later ones), then keeps the faster one.  Results do not depend
 * on the choice. */
#define IBB_SCHEDULE_AUTO 2

/* Contraction step applied to the boxes that pass the exclusion test.
 * IBB_CONTRACT_HS: the Hansen-Sengupta step (Sec. 2.3 eq 17-22; Alg. 3):
 * X'_i = X_i meets x_i - [g_i + sum_{j<i} P_ij (X'_j - x_j) + sum_{j>i}
 * P_ij (X_j - x_j)] / P_ii, component after component; unique root when
 * every Y_i lies inside the interior of X_i.  IBB_CONTRACT_KRAWCZYK: the
 * Krawczyk operator (eq 15) K(X) = x - g + (I - P)(X - x) with g = Y F(x),
 * P = Y J(X) (the same preconditioner Y), X' = X meets K(X) (eq 16); unique
 * root when K(X) lies inside the interior of X. */
#define IBB_CONTRACT_HS 0
#define IBB_CONTRACT_KRAWCZYK 1

/* Inclusion of F used by the exclusion test (Def. 2).  IBB_INCLUDE_NATURAL:
 * the natural interval extension (Def. 1).  IBB_INCLUDE_MEAN_VALUE: a box the
 * natural extension keeps (and that is not proven to hold a root) is also
 * tested with the mean-value form F_i(x) + sum_k J_ik(X) (X_k - x_k), x the
 * midpoint (one of the tighter inclusion strategies of Sec. 2.2); it is
 * discarded when some component excludes 0 (counted as excluded_eval).  The
 * box lists differ from the natural extension's. */
#define IBB_INCLUDE_NATURAL 0
#define IBB_INCLUDE_MEAN_VALUE 1

/* A square polynomial system in sparse monomial form (Sec. 2.1).
 * Equation i owns terms term_off[i] .. term_off[i+1]-1, in the order given;
 * term t is coef[t] * prod_k x_k^expo[t*n + k].  Requirements: 1 <= n <= 16,
 * every equation has >= 1 term, finite |coef| <= 2^40, total degree <= 8,
 * at most IBB_MAX_TERMS terms. */
typedef struct {
  int32_t n;
  const int32_t* term_off; /* [n+1], term_off[0] = 0, strictly increasing */
  const uint8_t* expo;     /* [T*n], T = term_off[n]                      */
  const double* coef;      /* [T]                                          */
} ibb_system;

/* Search parameters (Alg. 1 inputs plus the contraction policy). */
typedef struct {
  double tol;              /* emit a box once every coordinate is <= tol wide (> 0)     */
  int64_t max_boxes;       /* budget on the number of tree nodes processed (>= 1)       */
  int32_t split_mode;      /* IBB_SPLIT_WIDEST or IBB_SPLIT_ALL                          */
  int32_t max_recontract;  /* consecutive re-contractions before bisecting (>= 1; 16)   */
  double recontract_ratio; /* re-contract when the width shrank to <= ratio * width (0.5) */
  double hs_max_width;     /* skip the contraction on boxes wider than this (+inf)       */
  int32_t schedule;        /* IBB_SCHEDULE_AUTO (default), _QUEUE or _LEVELS             */
  int32_t contractor;      /* IBB_CONTRACT_HS (default) or IBB_CONTRACT_KRAWCZYK         */
  int32_t inclusion;       /* IBB_INCLUDE_NATURAL (default) or IBB_INCLUDE_MEAN_VALUE     */
  int32_t reserved;        /* must be 0                                                  */
} ibb_params;

/* Counters of the search tree (identical on every run and on the CPU oracle). */
typedef struct {
  int64_t processed;         /* tree nodes stepped                               */
  int64_t excluded_eval;     /* discarded by the exclusion test (Def. 2)         */
  int64_t excluded_hs;       /* discarded by an empty contraction (Alg. 3)       */
  int64_t hs_skipped;        /* contraction skipped (unusable preconditioner)   */
  int64_t recontracted;      /* re-queued after a strong contraction            */
  int64_t bisected;          /* split into children                              */
  int64_t emitted_unique;    /* output boxes tagged IBB_UNIQUE                   */
  int64_t emitted_undecided; /* output boxes tagged IBB_UNDECIDED                */
  int64_t levels;            /* depth of the tree (levels processed)             */
  int64_t max_frontier;      /* widest tree level                                */
  double kernel_ms;          /* device time of the search (host-timed calls)     */
} ibb_stats;

typedef struct ibb_ctx ibb_ctx;

/* Create a context on HIP device `device` (loads the kernels, queries the
 * device).  Returns IBB_OK and *out, or IBB_ERR_DEVICE. */
int ibb_ctx_create(int device, ibb_ctx** out);
void ibb_ctx_destroy(ibb_ctx* ctx);

/* Static description of a status code. */
const char* ibb_strerror(int status);

/* Default parameters: tol 1e-8, max_boxes 10^8, widest split, 16, 0.5, +inf. */
void ibb_params_default(ibb_params* p);

/* Solve one system on the box [lo, hi] (host arrays of n doubles).
 * Outputs (host, caller-allocated): out_lo/out_hi [cap*n] row-major boxes,
 * out_tag [cap]; *n_out = number of boxes.  The list is sorted
 * lexicographically by (lo_0..lo_{n-1}, hi_0..hi_{n-1}, tag) with -0 written
 * as +0.  If the list holds more than `cap` boxes the call returns
 * IBB_ERR_OUTPUT_CAPACITY and *n_out is the required count.  `stats` may be
 * NULL.  Synchronous; device memory comes from the context. */
int ibb_solve(ibb_ctx* ctx, const ibb_system* sys, const double* lo, const double* hi,
              const ibb_params* params, double* out_lo, double* out_hi, uint8_t* out_tag,
              int64_t cap, int64_t* n_out, ibb_stats* stats);

/* Solve B independent systems in one pass over the device (systems bucketed
 * by size, each bucket one persistent launch).  Per system b: systems[b],
 * its box lo/hi[b*IBB_MAX_N .. b*IBB_MAX_N + n_b) (host, stride IBB_MAX_N),
 * params[b].  Outputs (host): boxes of all systems back to back, system b's
 * boxes being out_off[b] .. out_off[b+1]-1 (out_off has B+1 entries), each box
 * stored with stride IBB_MAX_N in out_lo/out_hi ([cap*IBB_MAX_N]) and its tag in
 * out_tag[cap], sorted per system as in ibb_solve; status[b] is the system's
 * own status (IBB_OK, IBB_ERR_INVALID_ARG, IBB_ERR_BUDGET; a failed system
 * returns no boxes) and stats[b] its counters (levels and max_frontier are 0)
 * when stats is not NULL.  Each system's result equals ibb_solve on it alone.
 * Device memory: the frontier is sized from the autotuner's measured widths
 * (below) within the free device memory (or the bound ibb_batch_set_memory
 * sets); a batch whose frontier does not fit is solved in parts, halving the
 * member range until each part fits, with the same results; a single member
 * whose widest level alone exceeds the memory fails alone with
 * IBB_ERR_QUEUE_OVERFLOW.
 * Returns IBB_OK, IBB_ERR_OUTPUT_CAPACITY (out_off filled: out_off[B] is the
 * required capacity) or a device error. */
int ibb_solve_batch(ibb_ctx* ctx, int32_t B, const ibb_system* systems, const double* lo,
                    const double* hi, const ibb_params* params, double* out_lo, double* out_hi,
                    uint8_t* out_tag, int64_t cap, int64_t* out_off, int32_t* status,
                    ibb_stats* stats);

/* A batch prepared once and solved repeatedly (same members, same boxes):
 * ibb_batch_plan_create validates and compiles the members, uploads them into
 * device memory owned by the plan and records the device work of a batch solve
 * (counter resets by fill kernels, initial boxes, one persistent launch per
 * lane-count bucket) into a HIP graph; ibb_batch_plan_run replays the graph on
 * the plan's stream and returns results exactly as ibb_solve_batch (same
 * arguments and meaning).  A frontier or output overflow re-records the graph
 * with larger capacities.  IBB_ERR_UNSUPPORTED if the runtime cannot record
 * the launches.  The systems and boxes are copied at creation; one plan runs
 * one batch at a time.  A plan is one batch, never split: a frontier beyond
 * the free device memory (or the context's bound) fails ibb_batch_plan_run
 * with IBB_ERR_NO_MEMORY. */
typedef struct ibb_batch_plan ibb_batch_plan;
int ibb_batch_plan_create(ibb_ctx* ctx, int32_t B, const ibb_system* systems, const double* lo,
                          const double* hi, const ibb_params* params, ibb_batch_plan** plan);
int ibb_batch_plan_run(ibb_batch_plan* plan, double* out_lo, double* out_hi, uint8_t* out_tag,
                       int64_t cap, int64_t* out_off, int32_t* status, ibb_stats* stats);
void ibb_batch_plan_destroy(ibb_batch_plan* plan);

/* ---- batch launch configuration and its autotuner ----
 * Members of a batch fall into four lane-count classes by size: class 0
 * (n <= 2), 1 (n <= 4), 2 (n <= 8), 3 (n <= 16).  A context holds one launch
 * configuration per class, which ibb_solve_batch and ibb_batch_plan_create
 * apply to the members of that class (a plan keeps the configuration it was
 * created with):
 *   lanes            lanes per box: 2 << class (the default) or a larger power
 *                    of two up to 16; members then share the persistent launch
 *                    of that lane count, whose configuration (the other fields)
 *                    is the one of the class with that lane count;
 *   tiles_per_claim  tiles a wave takes per atomic claim of the level's
 *                    frontier (1 .. 16, default 1);
 *   blocks_per_cu    resident workgroups per CU of that launch (0, the
 *                    default, as many as registers and LDS allow; larger
 *                    values are clamped to that);
 *   tuned, ms        set by ibb_batch_tune: 1 and the measured device time of
 *                    the class's sample with this configuration (else 0, 0);
 *   front_per_member set by ibb_batch_tune: the widest tree level of the
 *                    class's sample launch divided by its members (0 = not
 *                    measured).  Queue sizes: when every class of a batch has
 *                    it, the batch's frontier is sized to 1.5 times the widest
 *                    launch's sum of its members' values (else a quarter of
 *                    the members' node budgets), and never below what an
 *                    earlier batch on the context needed.
 * Each box's fate depends on the box alone, so results, counters and statuses
 * are the same under every configuration (the batched analogue of the
 * autotuner's schedule choice for one system). */
typedef struct ibb_batch_config {
  int32_t lanes;
  int32_t tiles_per_claim;
  int32_t blocks_per_cu;
  int32_t tuned;
  double ms;
  double front_per_member;
} ibb_batch_config;

/* Bound, in bytes, on the device workspace of ibb_solve_batch and of plans
 * created afterwards (0, the default: the free device memory); a batch whose
 * frontier needs more is solved in parts.  Frees the context's batch
 * workspace when it exceeds the new bound.  IBB_ERR_INVALID_ARG for a null
 * context or a negative size. */
int ibb_batch_set_memory(ibb_ctx* ctx, int64_t bytes);

/* Current configuration of class cls (0..3) into *out.  IBB_ERR_INVALID_ARG
 * for a bad class or null pointer. */
int ibb_batch_get_config(ibb_ctx* ctx, int32_t cls, ibb_batch_config* out);

/* Replace the configuration of class cls (tuned, ms and front_per_member
 * are ignored and cleared).  IBB_ERR_INVALID_ARG unless lanes is a power of two with
 * 2 << cls <= lanes <= 16, 1 <= tiles_per_claim <= 16 and blocks_per_cu >= 0. */
int ibb_batch_set_config(ibb_ctx* ctx, int32_t cls, const ibb_batch_config* cfg);

/* Autotuner: for every class with valid members among the B given systems
 * (arguments as ibb_solve_batch), solves the class's first min(count, sample)
 * members as a batch under each candidate configuration -- lanes per box
 * {2 << cls, 4 << cls (up to 16)} x tiles per claim {1, 4} x workgroups per CU
 * {all that fit, two thirds of them} -- timing the device work of each with
 * HIP events, and keeps the fastest in the context (a candidate must beat the
 * default configuration by 3 % to replace it).  The solves' results are
 * discarded; every candidate must reproduce the default's counters and
 * statuses exactly, else IBB_ERR_DEVICE.  sample >= 1.  Takes the device
 * time of (candidates x sample) solves; blocks until done. */
int ibb_batch_tune(ibb_ctx* ctx, int32_t B, const ibb_system* systems, const double* lo, const double* hi,
                   const ibb_params* params, int32_t sample);

/* ---- serving: continuous batching of solves on one device ----
 * Requests are queued by ibb_server_submit (the system is copied).  Each call
 * of ibb_server_step
 *   (1) waits for the device pass the previous call enqueued and harvests the
 *       solves that ran out of boxes (their ids become available from
 *       ibb_server_finished, their results from ibb_server_poll);
 *   (2) admits queued requests, in arrival order, while a device slot is free
 *       and the request's reservation fits the device pool: a request
 *       reserves frontier boxes for itself, reserve_per_solve for every 64
 *       bisections its tree needs at least (each coordinate halved from its
 *       initial width down to tol), at most max_boxes + 1, and the bytes of
 *       two levels of that many boxes of its size bucket; the admitted
 *       requests of a call are uploaded with one copy and one kernel and join
 *       the solves already on the device;
 *   (3) makes room for the next levels of each size bucket: its frontier grows
 *       while all bucket frontiers together stay within pool_bytes; when they
 *       cannot, the solves holding the most boxes beyond their reservation
 *       are failed with IBB_ERR_QUEUE_OVERFLOW, alone (their boxes are dropped,
 *       the other solves go on);
 *   (4) enqueues one pass of `levels_per_quantum` tree levels of every bucket
 *       and, while requests wait for admission, returns without waiting for
 *       it, so that host work between calls overlaps the device's (with none
 *       waiting it harvests the pass before returning).
 * A solve keeps its boxes resident on the device until it finishes, and its
 * result is identical to ibb_solve on it alone.  Only IBB_SPLIT_WIDEST is
 * served. */
typedef struct {
  int32_t max_slots;          /* solves resident on the device at once (256)     */
  int64_t frontier_cap;       /* initial boxes per size bucket's frontier (2^20) */
  int64_t reserve_per_solve;  /* frontier boxes reserved per 64 bisections (2^14) */
  int32_t levels_per_quantum; /* tree levels per device pass (8)                 */
  int32_t out_cap_per_solve;  /* output boxes per solve (1024)                   */
  int64_t pool_bytes;         /* device bytes for all bucket frontiers (8 GiB)   */
} ibb_server_config;

typedef struct ibb_server ibb_server;

void ibb_server_config_default(ibb_server_config* cfg);
/* Allocates the server's device state on the context's GPU (cfg may be NULL).
 * IBB_ERR_INVALID_ARG if the four initial bucket frontiers exceed pool_bytes. */
int ibb_server_create(ibb_ctx* ctx, const ibb_server_config* cfg, ibb_server** out);
/* Waits for the device, frees the server and every request it holds. */
void ibb_server_destroy(ibb_server* server);
/* Queues a request; returns its id (>= 0) or a negative status. */
int64_t ibb_server_submit(ibb_server* server, const ibb_system* sys, const double* lo, const double* hi,
                          const ibb_params* params);
/* One scheduling round (see above); returns the number of requests harvested
 * in this round, or a negative status. */
int ibb_server_step(ibb_server* server);
/* Copies up to cap ids of requests harvested since the previous call (in
 * harvest order) to ids and forgets them; returns how many were copied. */
int64_t ibb_server_finished(ibb_server* server, int64_t* ids, int64_t cap);
/* Result of a finished request (then forgotten): IBB_OK with the sorted boxes
 * as in ibb_solve, *status the request's own status (IBB_OK, IBB_ERR_BUDGET,
 * IBB_ERR_OUTPUT_CAPACITY, IBB_ERR_QUEUE_OVERFLOW); returns 1 while the request
 * is queued or running. */
int ibb_server_poll(ibb_server* server, int64_t id, double* out_lo, double* out_hi, uint8_t* out_tag,
                    int64_t cap, int64_t* n_out, int32_t* status, ibb_stats* stats);
/* Removes a request that has not been admitted yet (IBB_ERR_UNSUPPORTED once
 * it is on the device). */
int ibb_server_cancel(ibb_server* server, int64_t id);
/* Requests waiting for admission and requests on the device. */
int ibb_server_pending(ibb_server* server, int64_t* queued, int64_t* active);

/* Device workspace (bytes) that ibb_solve_async needs for a system with n
 * variables, a frontier of `frontier_cap` boxes and `out_cap` output boxes.
 * The level-by-level schedule holds one tree level (at most frontier_cap
 * boxes) at a time; the work-queue schedule keeps the boxes created and not
 * yet stepped in a ring of the largest power of two <= frontier_cap slots.
 * Either overflow ends the solve with IBB_ERR_QUEUE_OVERFLOW. */
size_t ibb_workspace_size(int32_t n, int64_t frontier_cap, int64_t out_cap);

/* Enqueue a solve on `stream` (a hipStream_t, NULL = default stream) using
 * caller-provided device memory: d_ws (>= ibb_workspace_size bytes, 256-byte
 * aligned), outputs d_out_lo/d_out_hi [out_cap*n], d_out_tag [out_cap] and
 * d_info [16] int64 written when the stream reaches the end of the solve:
 *   d_info[0] status, [1] number of output boxes (may exceed out_cap, then the
 *   status is IBB_ERR_OUTPUT_CAPACITY), [2..11] the ibb_stats counters in
 *   order (processed .. max_frontier).
 * The host inputs are copied before the call returns.  Returns IBB_OK when the
 * work was enqueued; argument errors are returned directly.  With
 * IBB_SCHEDULE_AUTO, while a system shape is still being timed, the call
 * waits for the previous solve enqueued on this context to finish. */
int ibb_solve_async(ibb_ctx* ctx, const ibb_system* sys, const double* lo, const double* hi,
                    const ibb_params* params, void* d_ws, size_t ws_bytes, int64_t frontier_cap,
                    int64_t out_cap, double* d_out_lo, double* d_out_hi, uint8_t* d_out_tag,
                    int64_t* d_info, void* stream);

/* ---- allocation-free solve ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as ibb_solve_async (same arguments, outputs, d_info and results),
 * except that the workspace is not passed in: it is the library's own array
 * of IBB_NOALLOC_WORKSPACE_BYTES bytes on the context's device, a file-scope
 * device array that each GPU the library runs on holds until the process
 * ends.  The call allocates no device memory and no pinned host memory (the
 * context reserves its pinned staging buffer for the largest system when it
 * is created); the system is compiled on the host as in every entry point.
 * Returns IBB_ERR_WORKSPACE_LIMIT, with nothing enqueued, when
 * ibb_workspace_size(n, frontier_cap, out_cap) exceeds the array (for
 * example n <= 8 with out_cap 4096 allows a frontier of about 168,000 boxes,
 * n <= 16 about 85,000).  Every call on one device shares that device's
 * array, whichever context makes it: calls whose device work overlaps race
 * and their results are undefined, so order them (e.g. enqueue them on one
 * stream).  The array keeps the last call's contents; each call initialises
 * every part of it that the solve reads. */
#define IBB_NOALLOC_WORKSPACE_BYTES (64ull << 20)
int ibb_solve_noalloc(ibb_ctx* ctx, const ibb_system* sys, const double* lo, const double* hi,
                      const ibb_params* params, int64_t frontier_cap, int64_t out_cap, double* d_out_lo,
                      double* d_out_hi, uint8_t* d_out_tag, int64_t* d_info, void* stream);

/* Per-level frontier sizes of the most recent ibb_solve on this context
 * (level 0 = the initial box): copies min(count, cap) values, returns the
 * number of levels (boxes at depth k of the tree = the size of round k).  The
 * boxes kept by the exclusion test at a level are the paper's per-round
 * counts (Tables 1, 4, 7) when split_mode = IBB_SPLIT_ALL and the
 * contraction is off (hs_max_width = 0).  After a budget error the sizes are
 * complete for every finished round with IBB_SCHEDULE_LEVELS only. */
int64_t ibb_last_level_sizes(ibb_ctx* ctx, int64_t* sizes, int64_t cap);

/* Device time (ms) of the persistent search kernel of the most recent solve
 * enqueued on this context (either entry point), measured with HIP events
 * recorded on the solve's stream around the launch; waits for that event.
 * Returns -1 if no solve was enqueued. */
double ibb_last_kernel_ms(ibb_ctx* ctx);

/* One round of the search (Alg. 1: a round set of boxes, each through the
 * exclusion test of Def. 2, the contraction of Alg. 3 and the bisection of
 * Alg. 2, exactly as inside ibb_solve) on `count` caller-given boxes.
 * All arrays are host memory owned by the caller, boxes row-major [count][n]:
 *   lo, hi    the boxes;
 *   rec       one record per box: bit 0 = uniqueness already proven (the box
 *             skips the exclusion test), bits 8..15 = recontractions so far;
 *             other bits must be zero;
 *   child_*   the next round's boxes and records, at most child_cap;
 *   emit_*    boxes of width <= params->tol (or that cannot be split), with
 *             tag 1 = proven unique root, at most emit_cap.
 * The order of children and of emitted boxes is unspecified (compare as
 * multisets).  params->max_boxes does not apply.  *n_child and *n_emit get the
 * counts; when either exceeds its capacity IBB_ERR_OUTPUT_CAPACITY is
 * returned and the outputs are not written.  stats (may be NULL) gets the
 * round's counters.  Synchronous; uses the context's workspace. */
int ibb_round(ibb_ctx* ctx, const ibb_system* sys, const ibb_params* params, int64_t count,
              const double* lo, const double* hi, const uint32_t* rec, double* child_lo,
              double* child_hi, uint32_t* child_rec, int64_t child_cap, int64_t* n_child,
              double* emit_lo, double* emit_hi, uint8_t* emit_tag, int64_t emit_cap,
              int64_t* n_emit, ibb_stats* stats);

/* ---- backtracking merge (Alg. 5) ----
 * Merges output boxes into cells of the all-coordinate bisection grid of the
 * initial box X0 = [x0_lo, x0_hi] (Alg. 2): cell j = (j_0..j_{n-1}) of round k
 * covers, in coordinate i, [a + j_i (b - a) / 2^k, a + (j_i + 1) (b - a) / 2^k]
 * with [a, b] = [x0_lo[i], x0_hi[i]].  Each of the m boxes (host, row-major
 * [m][n], inside X0) first becomes the round-`level` cells it meets: per
 * coordinate the cells whose interior meets the box's interior (a degenerate
 * coordinate: the cell [B_j, B_{j+1}) holding the point, the last cell
 * closed).  Then, round after round, each cell is replaced by the cell of the
 * previous round it was split from (Alg. 5: j_i -> floor(j_i / 2)) and the
 * duplicates are dropped.  Outputs (host, caller-allocated): counts[k] =
 * distinct cells at round k for k = 0..level ([level + 1]); out_cells = the
 * distinct round-`out_level` cells as index rows [cap][n], sorted
 * lexicographically, *n_out their number.  The paper reads the isolated
 * roots off the first round, from the finest, whose count equals the next
 * coarser round's (Tab. 3, 6, 8).  Grid comparisons are exact.  Errors:
 * IBB_ERR_INVALID_ARG (n outside 1..16, level outside 0..IBB_BACKTRACK_MAX_LEVEL,
 * out_level > level, X0 bounds not finite, not lo < hi, or nonzero with
 * magnitude outside [2^-500, 2^40], a box not inside X0), IBB_ERR_UNSUPPORTED
 * (more than IBB_BACKTRACK_MAX_CELLS round-`level` cells), IBB_ERR_OUTPUT_CAPACITY
 * (*n_out > cap; counts are still written), IBB_ERR_NO_MEMORY.  Host only,
 * no context needed. */
#define IBB_BACKTRACK_MAX_LEVEL 50
#define IBB_BACKTRACK_MAX_CELLS (1 << 21)
int ibb_backtrack(int32_t n, const double* x0_lo, const double* x0_hi, int64_t m, const double* lo,
                  const double* hi, int32_t level, int64_t* counts, int32_t out_level, int64_t* out_cells,
                  int64_t cap, int64_t* n_out);

/* Diagnostics: run the search step on the single box [lo, hi] (one tree
 * level) and copy its intermediates to `dump` (host, >= 6n^2 + 8n + 4
 * doubles): J(X) [n][n][2], F(mid X) [n][2], the single-precision mid J
 * [n][n], the preconditioner Y [n][n], g [n][2], P [n][n][2] (rows by pivot
 * position), the bracket N_i [n][2], the contracted box [n][2], and flags
 * (skipped, empty, unique, ran).  Intervals as (lo, hi). */
int ibb_debug_step(ibb_ctx* ctx, const ibb_system* sys, const double* lo, const double* hi,
                   const ibb_params* params, double* dump, int64_t dump_len);

/* Diagnostics: apply one rounding primitive of the device arithmetic to n
 * operand pairs (host arrays) -- op 0..7 = rd/ru of + - * /, 8 = narrowing to
 * single precision (round to nearest, result widened), 9 = midpoint
 * rd(rd(a+b)*0.5), 10 = single-precision a*b, 11 = single-precision a/b.
 * For checking the device primitives against exact arithmetic. */
int ibb_selftest_ops(ibb_ctx* ctx, int32_t op, int64_t n, const double* a, const double* b,
                     double* out);

#ifdef __cplusplus
}
#endif
#endif /* IBB_H */
