// The context object behind pgdto_ctx* (host library internal).
#pragma once

#include <hip/hip_runtime.h>

#include <unordered_map>

#include "pgdto_internal.h"

struct pgdto_ctx {
  int device = 0;
  double* part = nullptr;        // per-tile partial sums, double-buffered
  uint64_t* sync = nullptr;      // grid synchronisation words
  uint64_t launch_seq = 0;       // launches so far (the kernel takes its epochs from the door)
  void* res_dev = nullptr;       // device staging of a result struct
  void* res_host = nullptr;      // pinned host staging
  uint64_t* trace = nullptr;     // per-pass timestamps when PGDTO_TRACE is set
  int coop_cap[2][2][PGDTO_MAX_M + 1] = {};   // co-resident workgroups per kernel
  int last_grid = 0;
  int last_ntiles = 0;
  // grid autotuner: workgroups chosen per (kind, dtype, m, tile count)
  int autotune = 0;
  std::unordered_map<uint64_t, int> tuned_grid;
  int forced_grid = 0;                        // set while a candidate is timed
  uint64_t door_wait = pgdto::DOOR_WAIT_DEFAULT;   // arrival-door wait of one-instance launches (100 MHz ticks)
  int reduce_wg0 = 0;                         // one-instance launches: workgroup 0 reduces each pass alone
  // one-launch batches: per-slot workspace (grown on demand) and pinned
  // descriptor areas used in turn, each with the event of its last launch
  int bt_cap = 0;                             // co-resident workgroups of the batch kernel
  int bt_slots = 0;                           // slots the workspace holds
  double* bt_part = nullptr;
  uint64_t* bt_sync = nullptr;
  pgdto::Desc* bt_jobs[pgdto::BATCH_RING] = {};
  hipEvent_t bt_ev[pgdto::BATCH_RING] = {};
  int bt_next = 0;
  uint64_t bt_seq = 0;
  // workspace of the wide coupled kernel (m > SMALL_M), allocated at first use
  double* wide = nullptr;
};

namespace pgdto {
int validate_params(const pgdto_params* p);
int build_desc(const pgdto_problem* pr, const pgdto_params* pp, bool need_y, Desc& d);
int fill_pgd(const pgdto_pgd_args* a, Desc& d);
int grid_for(pgdto_ctx* c, const Desc& d);
// a coupled problem beyond SMALL_M rows (the wide kernel; one-instance projections only)
inline bool is_wide(const Desc& d) { return d.kind == PGDTO_COUPLED && d.m > SMALL_M; }
}  // namespace pgdto
