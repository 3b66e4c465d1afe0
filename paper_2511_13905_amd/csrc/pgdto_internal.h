// Internal definitions shared by the kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pgdto.h"

namespace pgdto {

constexpr int BLOCK = 512;                 // threads per workgroup (8 wave64)
constexpr int NWAVE = BLOCK / 64;
constexpr int NT = 2;                      // trial multipliers per 1-D search pass
constexpr int TARGET_TILES = 512;          // bound the partial-sum layout is sized for (instances use half)
constexpr int MAX_TILES = TARGET_TILES + PGDTO_MAX_BLOCKS + 8;
constexpr int TILES_PAD = 704;             // stride of the partial-sum table
constexpr int SMALL_M = 8;                 // coupled rows of the register-accumulating kernel
constexpr int VMAX = 112;                  // partial values per tile (coupled, m = SMALL_M)
constexpr int PART_DOUBLES = 2 * VMAX * TILES_PAD;   // double-buffered
constexpr int GMAX = 1024;                 // workgroups of one launch (upper bound)
constexpr int TOT_MAX = 1024;              // per-segment totals of one pass
constexpr int NREP = 64;                   // copies of the go word, each with the totals beside it
constexpr int REP_WORDS = 128;             // 1 KiB per copy: go word + up to 127 totals
// flags, go-word replicas, error line, totals, then two lines for the arrival
// door of one-instance launches
constexpr size_t SYNC_WORDS = (size_t)GMAX * 16 + (size_t)NREP * REP_WORDS + 16 + TOT_MAX + 32;   // uint64 words

// Largest workgroup count for which every workgroup reads every flag and
// every tile partial of a pass itself (beyond it the polls of the same lines
// would queue up; workgroup 0 then reduces alone and broadcasts the totals).
constexpr int ALLRED_MAX_WG = 256;

// Bounded spin of the grid barrier: about a second of waiting before the
// workgroup gives up, flags PGDTO_ERR_TIMEOUT and leaves the kernel.
constexpr uint32_t SPIN_LIMIT = 1u << 20;

// Longest wait of the arrival door of one-instance launches for the whole
// grid, in ticks of the 100 MHz clock (30 us).
constexpr uint64_t DOOR_WAIT_DEFAULT = 3000;

// Everything one launch needs, passed by value as the kernel argument (the
// multi-instance server kernel reads the same struct from device memory).
struct Desc {
  int32_t kind, dtype, m, nseg;
  int64_t n, lda;
  const void* y;
  const void* A;
  void* x;
  uint32_t* free_mask;
  void* cbuf;            // free-set compaction scratch, n elements of the stream dtype (x, or the
                         // Algorithm 3 step's work buffer); NULL: no compaction
  double lo, hi, kappa;
  double auto_tau;       // > 0: kappa = auto_tau / (largest breakpoint), set after the zero pass
  uint64_t eq_mask;      // bit j: row / block j is an equality a_j.x = b_j
  uint64_t door_wait;    // longest wait of the arrival door for the grid (100 MHz ticks)
  double tol_b, tol_n, c1, c2;
  int32_t max_search, max_newton, max_ls, search, ncp, stage1, compact;
  double b[PGDTO_MAX_BLOCKS];          // right-hand sides (pgd: G - g)
  double lam0[PGDTO_MAX_BLOCKS];       // warm start (warm != 0)
  int32_t warm;
  int64_t off[PGDTO_MAX_BLOCKS + 1];   // segment bounds (single/coupled: 0, n)
  int32_t tile_base[PGDTO_MAX_BLOCKS + 1];
  int64_t tile_elems;
  int32_t ntiles;
  // workgroups that solve this instance: blockIdx.x in [wg_base, wg_base + wg_count)
  int32_t wg_base, wg_count;
  // Algorithm 3 step (pgd != 0)
  int32_t pgd, cg_rule, fallback_forced, zero_step;   // zero_step: t == 0
  const void* rho;
  const void* rho_prev;
  const void* grad;
  const void* grad_prev;
  void* dir;
  double alpha_max, alpha_fallback, omega, eps_alpha, tol_stop;
  // workspace
  double* part;          // [2][VMAX][TILES_PAD]
  uint64_t* sync;        // epoch flags, go word, error word, totals
  double* wide;          // workspace of the wide coupled kernel (m > SMALL_M), else NULL
  uint64_t epoch0;       // epoch base (pass p publishes epoch0 + p + 1): from the arrival
                         // door's generation in one-instance launches, per job in the server
  int32_t allred;        // 1: every workgroup waits for every flag and reduces the partials
                         // itself (up to ALLRED_MAX_WG workgroups); 0: workgroup 0 reduces
                         // them and publishes the totals with the go word
  int32_t buf0;          // partial-sum buffer of the first pass (a batch slot alternates the
                         // two buffers from one instance to the next)
  void* result;          // pgdto_result (pgd: pgdto_pgd_out)
  uint64_t* trace;       // optional [TRACE_MAX][4] per-pass timestamps (workgroup 0)
};

// Per-pass trace record (100 MHz device clock), TRACE_W words: [0] phase << 56
// | start, [1] element loop done, [2] workgroup 0 saw every flag, [3] totals
// reduced, [4] synchronisation left, [5] control done; last workgroup:
// [6] loop done, [7] saw the totals.
constexpr int TRACE_MAX = 128;
constexpr int TRACE_W = 8;
constexpr int TRACE_WG_PASSES = 16;        // per-workgroup records kept for the first passes
constexpr int TRACE_WG_W = 4;              // words per workgroup record
constexpr size_t TRACE_WORDS = (size_t)TRACE_MAX * TRACE_W + (size_t)TRACE_WG_PASSES * GMAX * TRACE_WG_W;

// Tiling: the tile size depends only on n and the dtype, so that an
// instance's reduction order (and hence its bits) does not depend on how many
// workgroups solve it.
inline int64_t vec_elems(int dtype) { return dtype == PGDTO_F32 ? 4 : 2; }
inline int64_t tile_unit(int dtype) { return (int64_t)BLOCK * vec_elems(dtype) * 2; }

}  // namespace pgdto

// ------------------------------------------------------------------ server
// Persistent multi-slot executor (continuous batching).  The host publishes
// job descriptors in pinned host memory; the slots of one long-running launch
// claim them in order, each slot solving one instance on its own workgroups
// with its own synchronisation words, and report completion in pinned memory.
namespace pgdto {

struct SrvHostCtl {            // pinned host memory, written by the host
  uint64_t tail;               // number of jobs published
  uint64_t pad0[15];
  uint64_t shutdown;           // non-zero: slots leave once the queue is empty
  uint64_t pad1[15];
};

struct SrvArgs {
  SrvHostCtl* ctl;             // pinned
  const Desc* jobs;            // pinned [qcap]: job j at j % qcap
  uint64_t* done;              // pinned [qcap]: j + 1 once job j finished
  pgdto_pgd_out* results;      // pinned [qcap] (a projection fills .proj)
  uint64_t* head;              // device: next job to claim
  uint64_t* slot_words;        // device: [slots][16]: broadcast sequence, job index
  double* part;                // device: per-slot partial sums, stride part_stride
  uint64_t* sync;              // device: per-slot barrier words, stride sync_stride
  uint64_t part_stride, sync_stride;
  uint64_t round0;             // launch-unique base of the broadcast sequence
  int32_t slots, wg_per_slot, qcap;
  uint32_t idle_spins;         // master polls without a job before the slot leaves
};

constexpr uint64_t SRV_LEAVE = ~0ull;

// One launch over a fixed list of instances (pgdto_project_batch_async,
// pgdto_pgd_step_batch_async): slot s solves instances s, s + slots, ... in
// order, on its own workgroups, partial sums and barrier words.
struct BatchArgs {
  const Desc* jobs;            // pinned [count], written by the host before the launch
  void* results;               // device: pgdto_result[count] or pgdto_pgd_out[count]
  double* part;                // device: per-slot partial sums, stride part_stride
  uint64_t* sync;              // device: per-slot barrier words, stride sync_stride
  uint64_t part_stride, sync_stride;
  uint64_t epoch_base;         // launch-unique: the k-th job of a slot uses epoch_base + (k << 16)
  int32_t count, slots, wg_per_slot, is_pgd;
};
constexpr int BATCH_MAX = 256;          // instances per batch launch
constexpr int BATCH_RING = 4;           // pinned descriptor areas per context (reused in turn)
constexpr int BATCH_JOB_SHIFT = 16;     // passes per job stay below 2^16

// ------------------------------------------------------------------ wide coupled kernel
// m in (SMALL_M, PGDTO_MAX_M] dense rows: the Newton sums are reduced through
// a table of WV values per tile, in a workspace of its own (per context).
constexpr int WM = PGDTO_MAX_M;                 // rows
constexpr int WNJ = WM * (WM + 1) / 2;          // Jacobian sums (upper triangle)
constexpr int WCAND = 16;                       // Stage-1 candidates per check pass
constexpr int WV_PAD = 2176;                    // values per tile row (>= WM + WNJ, >= WCAND * WM)
constexpr int WTILES = TARGET_TILES / 2;        // tiles of one instance (one segment)
constexpr int WREP = 256;                       // words per go/command replica
static_assert(WV_PAD >= WM + WNJ && WV_PAD >= WCAND * WM, "tile row holds every pass's values");
// workspace layout (8-byte words): per-tile partials, totals, best-trial J,
// barrier flags (one line each), command replicas
constexpr size_t WIDE_PART = 0;
constexpr size_t WIDE_TOT = WIDE_PART + (size_t)WTILES * WV_PAD;
constexpr size_t WIDE_BEST = WIDE_TOT + WV_PAD;
constexpr size_t WIDE_FLAGS = WIDE_BEST + WV_PAD;
constexpr size_t WIDE_REP = WIDE_FLAGS + (size_t)GMAX * 16;
constexpr size_t WIDE_WORDS = WIDE_REP + (size_t)NREP * WREP;
const void* wide_fn(int m);            // the kernel for m rows

hipError_t launch_solve(const Desc& d, int grid, hipStream_t stream, bool cooperative);
int max_coresident(int kind, int dtype, int m, int device);
hipError_t launch_mark_error(void* result, int is_pgd, hipStream_t stream);
hipError_t launch_server(const SrvArgs& a, hipStream_t stream);
int server_coresident(int device);     // workgroups of the server kernel that fit at once
hipError_t launch_batch(const BatchArgs& a, hipStream_t stream);
int batch_coresident(int device);      // workgroups of the batch kernel that fit at once
}  // namespace pgdto
