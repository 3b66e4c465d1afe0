// Host side of one-launch batches (pgdto_project_batch_async,
// pgdto_pgd_step_batch_async): many instances solved by one persistent
// launch, the GPU split into slots of workgroups.  The descriptors go to a
// pinned area of the context that the kernel reads directly; the context
// keeps BATCH_RING such areas and reuses one only after the launch that read
// it has finished (its event), so back-to-back calls do not wait on the GPU.

#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>

#include "pgdto_ctx.h"
#include "pgdto_internal.h"

using namespace pgdto;

namespace {

constexpr int DEFAULT_SLOTS = 16;

// Per-slot partial sums and barrier words for `slots` slots.  Grows only;
// allocation happens on the first call that needs more slots (the device is
// synchronised first: an earlier batch launch may still use the old area).
int ensure_workspace(pgdto_ctx* c, int slots) {
  if (c->bt_slots >= slots) return PGDTO_OK;
  if (hipDeviceSynchronize() != hipSuccess) return PGDTO_ERR_HIP;
  if (c->bt_part) (void)hipFree(c->bt_part);
  if (c->bt_sync) (void)hipFree(c->bt_sync);
  c->bt_part = nullptr;
  c->bt_sync = nullptr;
  c->bt_slots = 0;
  if (hipMalloc(&c->bt_part, sizeof(double) * PART_DOUBLES * (size_t)slots) != hipSuccess) return PGDTO_ERR_NOMEM;
  if (hipMalloc(&c->bt_sync, sizeof(uint64_t) * SYNC_WORDS * (size_t)slots) != hipSuccess) return PGDTO_ERR_NOMEM;
  if (hipMemset(c->bt_sync, 0, sizeof(uint64_t) * SYNC_WORDS * (size_t)slots) != hipSuccess) return PGDTO_ERR_HIP;
  if (hipDeviceSynchronize() != hipSuccess) return PGDTO_ERR_HIP;
  c->bt_slots = slots;
  return PGDTO_OK;
}

int ensure_ring(pgdto_ctx* c) {
  for (int r = 0; r < BATCH_RING; ++r) {
    if (!c->bt_jobs[r] &&
        hipHostMalloc((void**)&c->bt_jobs[r], sizeof(Desc) * BATCH_MAX, hipHostMallocDefault) != hipSuccess)
      return PGDTO_ERR_NOMEM;
    if (!c->bt_ev[r] && hipEventCreateWithFlags(&c->bt_ev[r], hipEventDisableTiming) != hipSuccess)
      return PGDTO_ERR_HIP;
  }
  return PGDTO_OK;
}

// Validated descriptors in, one launch out.
int launch_list(pgdto_ctx* c, const Desc* descs, int count, int slots, void* results, int is_pgd, hipStream_t s) {
  if (hipSetDevice(c->device) != hipSuccess) return PGDTO_ERR_HIP;
  if (c->bt_cap == 0) c->bt_cap = batch_coresident(c->device);
  const int cap = c->bt_cap;
  if (cap <= 0) return PGDTO_ERR_HIP;
  if (slots <= 0) slots = std::min(count, DEFAULT_SLOTS);
  slots = std::min(slots, count);
  const int wg = cap / slots;
  if (wg < 1 || wg > GMAX) return PGDTO_ERR_ARG;
  int st = ensure_workspace(c, slots);
  if (st == PGDTO_OK) st = ensure_ring(c);
  if (st != PGDTO_OK) return st;
  const int r = c->bt_next;
  if (hipEventSynchronize(c->bt_ev[r]) != hipSuccess) return PGDTO_ERR_HIP;   // the area's last reader
  memcpy(c->bt_jobs[r], descs, sizeof(Desc) * (size_t)count);
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.jobs = c->bt_jobs[r];
  a.results = results;
  a.part = c->bt_part;
  a.sync = c->bt_sync;
  a.part_stride = PART_DOUBLES;
  a.sync_stride = SYNC_WORDS;
  a.epoch_base = (++c->bt_seq) << 32;
  a.count = count;
  a.slots = slots;
  a.wg_per_slot = wg;
  a.is_pgd = is_pgd;
  if (launch_batch(a, s) != hipSuccess) {
    (void)hipGetLastError();
    for (int i = 0; i < count; ++i) {
      void* res = is_pgd ? (void*)((pgdto_pgd_out*)results + i) : (void*)((pgdto_result*)results + i);
      (void)launch_mark_error(res, is_pgd, s);
    }
    return PGDTO_ERR_HIP;
  }
  if (hipEventRecord(c->bt_ev[r], s) != hipSuccess) return PGDTO_ERR_HIP;
  c->bt_next = (r + 1) % BATCH_RING;
  c->last_grid = slots * wg;
  c->last_ntiles = descs[0].ntiles;
  return PGDTO_OK;
}

}  // namespace

extern "C" int pgdto_project_batch_async(pgdto_ctx* c, const pgdto_problem* probs, int count,
                                         const pgdto_params* params, pgdto_result* results_dev, int slots,
                                         void* stream) {
  if (!c || !probs || !results_dev || count < 1 || count > BATCH_MAX || slots < 0) return PGDTO_ERR_ARG;
  pgdto_params tmp;
  if (!params) {
    pgdto_params_default(&tmp);
    params = &tmp;
  }
  static thread_local Desc descs[BATCH_MAX];
  for (int i = 0; i < count; ++i) {
    const int st = build_desc(&probs[i], params, true, descs[i]);
    if (st != PGDTO_OK) return st;
    if (descs[i].dtype != PGDTO_F32 || is_wide(descs[i])) return PGDTO_ERR_ARG;
  }
  return launch_list(c, descs, count, slots, results_dev, 0, (hipStream_t)stream);
}

extern "C" int pgdto_pgd_step_batch_async(pgdto_ctx* c, const pgdto_pgd_args* args, int count,
                                          const pgdto_params* params, pgdto_pgd_out* outs_dev, int slots,
                                          void* stream) {
  if (!c || !args || !outs_dev || count < 1 || count > BATCH_MAX || slots < 0) return PGDTO_ERR_ARG;
  pgdto_params tmp;
  if (!params) {
    pgdto_params_default(&tmp);
    params = &tmp;
  }
  static thread_local Desc descs[BATCH_MAX];
  for (int i = 0; i < count; ++i) {
    pgdto_problem pr = args[i].proj;
    double zeros[PGDTO_MAX_BLOCKS] = {0};     // b is formed on the device
    pr.b = zeros;
    int st = build_desc(&pr, params, false, descs[i]);
    if (st == PGDTO_OK) st = fill_pgd(&args[i], descs[i]);
    if (st != PGDTO_OK) return st;
    if (descs[i].dtype != PGDTO_F32) return PGDTO_ERR_ARG;
  }
  return launch_list(c, descs, count, slots, outs_dev, 1, (hipStream_t)stream);
}
