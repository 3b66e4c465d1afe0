// Host side of the C ABI: argument validation, tiling, the launch (an
// ordinary one; the kernel's arrival door admits the workgroups), result
// retrieval.  No allocation happens on the call path: the context owns
// a fixed workspace sized for the largest tile table.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "pgdto_internal.h"
#include "pgdto_ctx.h"

using namespace pgdto;

extern "C" void pgdto_params_default(pgdto_params* p) {
  if (!p) return;
  p->tol_b = 1e-8;
  p->tol_n = 1e-12;
  p->max_search = 64;
  p->max_newton = 50;
  p->max_ls = 12;
  p->search = PGDTO_SEARCH_NEWTON;
  p->ncp = PGDTO_NCP_CONTINUOUS;
  p->stage1 = 1;
  p->c1 = 1e-4;
  p->c2 = 0.9;
  p->compact = 0;
}

extern "C" void pgdto_pgd_args_default(pgdto_pgd_args* a) {
  if (!a) return;
  memset(a, 0, sizeof(*a));
  a->proj.kind = PGDTO_SINGLE;
  a->proj.dtype = PGDTO_F32;
  a->proj.lo = 1e-3;
  a->proj.hi = 1.0;
  a->proj.C = INFINITY;
  a->t_warmup = 50;
  a->cg_rule = PGDTO_CG_PR_PLUS;
  a->alpha_max = 1e2;
  a->alpha_fallback = 0.2;
  a->omega = 1.0;
  a->eps_alpha = 1e-6;
  a->tol_viol = 1e-6;
  a->tol = 1e-4;
}

extern "C" const char* pgdto_status_string(int s) {
  switch (s) {
    case PGDTO_OK: return "ok";
    case PGDTO_PENDING: return "pending";
    case PGDTO_QUEUED: return "queued";
    case PGDTO_ERR_ARG: return "invalid argument";
    case PGDTO_ERR_HIP: return "HIP runtime error";
    case PGDTO_ERR_NOMEM: return "out of memory";
    case PGDTO_ERR_UNKNOWN_TICKET: return "unknown ticket";
    case PGDTO_ERR_TIMEOUT: return "device wait timed out";
    case PGDTO_ERR_BUSY: return "queue full";
    case PGDTO_ERR_CANCELLED: return "cancelled";
    case PGDTO_ERR_SCRATCH: return "problem exceeds the static scratch array";
    default: return "unknown status";
  }
}

extern "C" int pgdto_version(void) { return PGDTO_VERSION; }

extern "C" int pgdto_problem_check(const pgdto_problem* prob, const pgdto_params* params) {
  if (!prob) return PGDTO_ERR_ARG;
  pgdto_params pp;
  if (params) pp = *params; else pgdto_params_default(&pp);
  Desc d;
  return build_desc(prob, &pp, true, d);
}

extern "C" int pgdto_trace_read(pgdto_ctx* c, uint64_t* out, int max_records) {
  if (!c || !out) return PGDTO_ERR_ARG;
  if (!c->trace) return 0;
  if (max_records < 0) {   // per-workgroup table: TRACE_WG_PASSES x GMAX x TRACE_WG_W
    if (hipDeviceSynchronize() != hipSuccess) return PGDTO_ERR_HIP;
    if (hipMemcpy(out, c->trace + (size_t)TRACE_MAX * TRACE_W, sizeof(uint64_t) * TRACE_WG_PASSES * GMAX * TRACE_WG_W,
                  hipMemcpyDeviceToHost) != hipSuccess) return PGDTO_ERR_HIP;
    return TRACE_WG_PASSES;
  }
  const int n = max_records < TRACE_MAX ? max_records : TRACE_MAX;
  if (hipDeviceSynchronize() != hipSuccess) return PGDTO_ERR_HIP;
  if (hipMemcpy(out, c->trace, sizeof(uint64_t) * TRACE_W * n, hipMemcpyDeviceToHost) != hipSuccess) return PGDTO_ERR_HIP;
  if (hipMemset(c->trace, 0, sizeof(uint64_t) * TRACE_WORDS) != hipSuccess) return PGDTO_ERR_HIP;
  return n;
}

extern "C" size_t pgdto_struct_size(int which) {
  switch (which) {
    case 0: return sizeof(pgdto_problem);
    case 1: return sizeof(pgdto_params);
    case 2: return sizeof(pgdto_result);
    case 3: return sizeof(pgdto_pgd_args);
    case 4: return sizeof(pgdto_pgd_out);
    case 5: return sizeof(pgdto_batch_cfg);
    case 6: return sizeof(pgdto_path_point);
    default: return 0;
  }
}

extern "C" int pgdto_ctx_create(int device, pgdto_ctx** out) {
  if (!out) return PGDTO_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PGDTO_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return PGDTO_ERR_HIP;
  pgdto_ctx* c = new (std::nothrow) pgdto_ctx();
  if (!c) return PGDTO_ERR_NOMEM;
  c->device = device;
  int ok = hipMalloc(&c->part, sizeof(double) * PART_DOUBLES) == hipSuccess;
  ok = ok && hipMalloc(&c->sync, SYNC_WORDS * sizeof(uint64_t)) == hipSuccess;
  ok = ok && hipMalloc(&c->res_dev, sizeof(pgdto_pgd_out)) == hipSuccess;
  ok = ok && hipHostMalloc(&c->res_host, sizeof(pgdto_pgd_out), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMemset(c->sync, 0, SYNC_WORDS * sizeof(uint64_t)) == hipSuccess;
  ok = ok && hipMemset(c->part, 0, sizeof(double) * PART_DOUBLES) == hipSuccess;
  {
    const char* av = getenv("PGDTO_AUTOTUNE");
    c->autotune = (av && av[0] && av[0] != '0') ? 1 : 0;
    // PGDTO_GRID=k: one-instance launches use at most k workgroups (the
    // size of a server slot, to study a slot's passes in isolation)
    const char* gv = getenv("PGDTO_GRID");
    if (gv && gv[0]) c->forced_grid = std::max(0, atoi(gv));
    // PGDTO_DOOR_WAIT=t: the arrival door of one-instance launches waits at
    // most t ticks of the 100 MHz clock for the grid (default 3000 = 30 us;
    // 0 closes it at the first arrival, so that late workgroups occur)
    const char* dv = getenv("PGDTO_DOOR_WAIT");
    if (dv && dv[0]) c->door_wait = (uint64_t)std::max(0LL, atoll(dv));
    // PGDTO_REDUCE_WG0=1: one-instance launches take the reduction in which
    // workgroup 0 alone sums the pass partials and publishes the totals (the
    // form launches of more than ALLRED_MAX_WG workgroups use)
    const char* rv = getenv("PGDTO_REDUCE_WG0");
    c->reduce_wg0 = (rv && rv[0] && rv[0] != '0') ? 1 : 0;
  }
  {
    const char* tv = getenv("PGDTO_TRACE");
    if (tv && tv[0] && tv[0] != '0') {
      ok = ok && hipMalloc(&c->trace, sizeof(uint64_t) * TRACE_WORDS) == hipSuccess;
      ok = ok && hipMemset(c->trace, 0, sizeof(uint64_t) * TRACE_WORDS) == hipSuccess;
    }
  }
  ok = ok && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    pgdto_ctx_destroy(c);
    return PGDTO_ERR_NOMEM;
  }
  *out = c;
  return PGDTO_OK;
}

extern "C" int pgdto_ctx_destroy(pgdto_ctx* c) {
  if (!c) return PGDTO_ERR_ARG;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->part) (void)hipFree(c->part);
  if (c->sync) (void)hipFree(c->sync);
  if (c->res_dev) (void)hipFree(c->res_dev);
  if (c->res_host) (void)hipHostFree(c->res_host);
  if (c->trace) (void)hipFree(c->trace);
  if (c->wide) (void)hipFree(c->wide);
  if (c->bt_part) (void)hipFree(c->bt_part);
  if (c->bt_sync) (void)hipFree(c->bt_sync);
  for (int r = 0; r < BATCH_RING; ++r) {
    if (c->bt_jobs[r]) (void)hipHostFree(c->bt_jobs[r]);
    if (c->bt_ev[r]) (void)hipEventDestroy(c->bt_ev[r]);
  }
  delete c;
  return PGDTO_OK;
}

namespace pgdto {

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + na, b0 = (uintptr_t)b, b1 = b0 + nb;
  return a0 < b1 && b0 < a1;
}

int validate_params(const pgdto_params* p) {
  if (!(p->tol_n > 0.0) || !(p->tol_b >= 0.0)) return PGDTO_ERR_ARG;
  if (p->max_search < 1 || p->max_newton < 1 || p->max_ls < 1) return PGDTO_ERR_ARG;
  if (p->search != PGDTO_SEARCH_NEWTON && p->search != PGDTO_SEARCH_BISECT) return PGDTO_ERR_ARG;
  if (p->ncp != PGDTO_NCP_CONTINUOUS && p->ncp != PGDTO_NCP_PAPER) return PGDTO_ERR_ARG;
  if (!(p->c1 > 0.0 && p->c1 < 1.0 && p->c2 > p->c1 && p->c2 < 1.0)) return PGDTO_ERR_ARG;
  if (p->compact != 0 && p->compact != 1) return PGDTO_ERR_ARG;
  return PGDTO_OK;
}

// Validates a problem (host side only; nothing is launched on failure) and
// fills the problem part of the descriptor, including the tile table.
// need_y: the problem's y pointer is used (not for pgd_step).
int build_desc(const pgdto_problem* pr, const pgdto_params* pp, bool need_y, Desc& d) {
  memset(&d, 0, sizeof(d));
  if (!pr || !pp) return PGDTO_ERR_ARG;
  if (validate_params(pp) != PGDTO_OK) return PGDTO_ERR_ARG;
  if (pr->dtype != PGDTO_F32 && pr->dtype != PGDTO_F64) return PGDTO_ERR_ARG;
  if (pr->n < 1) return PGDTO_ERR_ARG;
  const size_t esz = pr->dtype == PGDTO_F32 ? 4 : 8;
  const int64_t n = pr->n;
  switch (pr->kind) {
    case PGDTO_SINGLE: if (pr->m != 1) return PGDTO_ERR_ARG; break;
    case PGDTO_INDEPENDENT: if (pr->m < 1 || pr->m > PGDTO_MAX_BLOCKS) return PGDTO_ERR_ARG; break;
    case PGDTO_COUPLED:
      if (pr->m < 1 || pr->m > PGDTO_MAX_M) return PGDTO_ERR_ARG;
      // beyond SMALL_M rows: float32 projections (the wide kernel)
      if (pr->m > SMALL_M && (pr->dtype != PGDTO_F32 || !need_y)) return PGDTO_ERR_ARG;
      break;
    default: return PGDTO_ERR_ARG;
  }
  if ((need_y && !pr->y) || !pr->A || !pr->x || !pr->b) return PGDTO_ERR_ARG;
  if ((need_y && !aligned16(pr->y)) || !aligned16(pr->A) || !aligned16(pr->x)) return PGDTO_ERR_ARG;
  if (pr->free_mask && ((uintptr_t)pr->free_mask & 3u)) return PGDTO_ERR_ARG;
  if (!isfinite(pr->lo) || !isfinite(pr->hi) || !(pr->lo < pr->hi)) return PGDTO_ERR_ARG;
  // NaN, 0 and -INFINITY rejected; INFINITY allowed; C < 0 asks for the
  // automatic penalty with tolerance -C
  if (!(pr->C > 0.0) && !(pr->C < 0.0 && isfinite(pr->C))) return PGDTO_ERR_ARG;
  size_t abytes = (size_t)n * esz;
  if (pr->kind != PGDTO_INDEPENDENT) {
    if (pr->m > 1) {
      if (pr->lda < n || ((size_t)pr->lda * esz) % 16 != 0) return PGDTO_ERR_ARG;
    }
    abytes = ((size_t)(pr->m - 1) * (size_t)std::max<int64_t>(pr->lda, n) + (size_t)n) * esz;
  }
  const size_t xbytes = (size_t)n * esz;
  if ((need_y && overlaps(pr->x, xbytes, pr->y, xbytes)) || overlaps(pr->x, xbytes, pr->A, abytes))
    return PGDTO_ERR_ARG;
  for (int j = 0; j < pr->m; ++j)
    if (!isfinite(pr->b[j])) return PGDTO_ERR_ARG;

  d.kind = pr->kind;
  d.dtype = pr->dtype;
  d.m = pr->m;
  d.n = n;
  d.lda = pr->kind == PGDTO_INDEPENDENT ? n : (pr->m > 1 ? pr->lda : std::max<int64_t>(pr->lda, n));
  d.y = pr->y;
  d.A = pr->A;
  d.x = pr->x;
  d.free_mask = pr->free_mask;
  d.lo = pr->lo;
  d.hi = pr->hi;
  if (pr->m < 64 && (pr->eq_mask >> pr->m) != 0) return PGDTO_ERR_ARG;
  d.eq_mask = pr->eq_mask;
  if (pr->lambda0) {
    for (int j = 0; j < pr->m; ++j) {
      const double l = pr->lambda0[j];
      const bool eq = (pr->eq_mask >> j) & 1ull;
      if (!isfinite(l) || (!eq && l < 0.0)) return PGDTO_ERR_ARG;
      d.lam0[j] = l;
    }
    d.warm = 1;
  }
  d.auto_tau = pr->C < 0.0 ? -pr->C : 0.0;
  d.kappa = (pr->C < 0.0 || isinf(pr->C)) ? 0.0 : 2.0 / pr->C;
  d.tol_b = pp->tol_b;
  d.tol_n = pp->tol_n;
  d.c1 = pp->c1;
  d.c2 = pp->c2;
  d.max_search = pp->max_search;
  d.max_newton = pp->max_newton;
  d.max_ls = pp->max_ls;
  d.search = pp->search;
  d.ncp = pp->ncp;
  d.stage1 = pp->stage1 ? 1 : 0;
  d.compact = pp->compact;
  d.cbuf = pr->x;                      // a projection's x is free until its final pass
  for (int j = 0; j < pr->m; ++j) d.b[j] = pr->b[j];

  // segments
  if (pr->kind == PGDTO_INDEPENDENT) {
    const int64_t* o = pr->block_offsets;
    if (!o || o[0] != 0 || o[pr->m] != n) return PGDTO_ERR_ARG;
    for (int j = 0; j < pr->m; ++j)
      if (!(o[j + 1] > o[j])) return PGDTO_ERR_ARG;
    d.nseg = pr->m;
    for (int j = 0; j <= pr->m; ++j) d.off[j] = o[j];
  } else {
    d.nseg = 1;
    d.off[0] = 0;
    d.off[1] = n;
  }
  // tiles: size depends only on n and dtype; about n/256 elements (one tile
  // per workgroup of a full-GPU launch, one 512-thread workgroup per CU)
  const int64_t unit = tile_unit(pr->dtype);
  const int64_t target = TARGET_TILES / 2;
  int64_t tile = (n + target - 1) / target;
  tile = std::max<int64_t>(unit, (tile + unit - 1) / unit * unit);
  d.tile_elems = tile;
  int32_t tb = 0;
  for (int s = 0; s < d.nseg; ++s) {
    d.tile_base[s] = tb;
    const int64_t astart = d.off[s] & ~(int64_t)31;
    tb += (int32_t)((d.off[s + 1] - astart + tile - 1) / tile);
  }
  d.tile_base[d.nseg] = tb;
  d.ntiles = tb;
  if (tb > TILES_PAD) return PGDTO_ERR_ARG;
  return PGDTO_OK;
}

static uint64_t tune_key(const Desc& d) {
  return ((uint64_t)d.kind << 40) | ((uint64_t)d.dtype << 36) | ((uint64_t)d.m << 24) | (uint64_t)d.ntiles;
}

static int coresident_cap(pgdto_ctx* c, const Desc& d) {
  const int ki = d.kind == PGDTO_COUPLED ? 1 : 0;
  const int mi = d.kind == PGDTO_COUPLED ? d.m : 0;
  int& cap = c->coop_cap[ki][d.dtype][mi];
  if (cap == 0) cap = max_coresident(d.kind, d.dtype, d.m, c->device);
  return cap;
}

// Workgroups of a one-instance launch: all that fit at once, capped by the
// tile count; or the autotuner's choice for this shape class.
int grid_for(pgdto_ctx* c, const Desc& d) {
  const int cap = coresident_cap(c, d);
  if (cap <= 0) return 0;
  const int full = std::max(1, std::min(d.ntiles, cap));
  if (c->forced_grid > 0) return std::min(c->forced_grid, full);
  auto it = c->tuned_grid.find(tune_key(d));
  return it != c->tuned_grid.end() ? std::min(it->second, full) : full;
}

// The wide kernel's workspace, allocated and cleared at the first wide
// launch of the context (its flags must start below every epoch).
static double* wide_workspace(pgdto_ctx* c) {
  if (c->wide) return c->wide;
  double* w = nullptr;
  if (hipMalloc(&w, WIDE_WORDS * sizeof(double)) != hipSuccess) return nullptr;
  if (hipMemset(w, 0, WIDE_WORDS * sizeof(double)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(w);
    return nullptr;
  }
  c->wide = w;
  return w;
}

int run_launch(pgdto_ctx* c, Desc& d, hipStream_t s, void* result_dev, bool is_pgd) {
  d.part = c->part;
  d.sync = c->sync;
  d.wide = nullptr;
  if (is_wide(d)) {
    if (is_pgd || d.ntiles > WTILES) return PGDTO_ERR_ARG;
    d.wide = wide_workspace(c);
    if (!d.wide) return PGDTO_ERR_NOMEM;
  }
  c->launch_seq += 1;
  d.epoch0 = c->launch_seq << 20;   // replaced on the device by the door's generation
  d.trace = c->trace;
  d.result = result_dev;
  d.pgd = is_pgd ? 1 : 0;
  const int grid = grid_for(c, d);
  if (grid <= 0) return PGDTO_ERR_HIP;
  d.wg_base = 0;
  d.wg_count = grid;
  d.door_wait = c->door_wait;
  // every workgroup reduces the pass partials itself (one round trip less per
  // pass than workgroup 0 publishing totals and a go word)
  d.allred = (grid <= ALLRED_MAX_WG && !c->reduce_wg0) ? 1 : 0;
  d.buf0 = 0;
  // an ordinary launch: the kernel's arrival door admits the workgroups that
  // are running together (normally all of them) and sends late ones home
  hipError_t e = launch_solve(d, grid, s, false);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)launch_mark_error(result_dev, is_pgd ? 1 : 0, s);
    return PGDTO_ERR_HIP;
  }
  c->last_grid = grid;
  c->last_ntiles = d.ntiles;
  return PGDTO_OK;
}

static int finish_blocking(pgdto_ctx* c, hipStream_t s, size_t bytes, void* out) {
  if (hipMemcpyAsync(c->res_host, c->res_dev, bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return PGDTO_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return PGDTO_ERR_HIP;
  memcpy(out, c->res_host, bytes);
  return PGDTO_OK;
}

int fill_pgd(const pgdto_pgd_args* a, Desc& d) {
  const pgdto_problem* pr = &a->proj;
  const size_t esz = pr->dtype == PGDTO_F32 ? 4 : 8;
  const size_t bytes = (size_t)pr->n * esz;
  if (!a->rho || !a->grad || !a->dir || !a->g || !a->G) return PGDTO_ERR_ARG;
  if (a->t < 0) return PGDTO_ERR_ARG;
  if (a->t > 0 && (!a->rho_prev || !a->grad_prev)) return PGDTO_ERR_ARG;
  if (!aligned16(a->rho) || !aligned16(a->grad) || !aligned16(a->dir)) return PGDTO_ERR_ARG;
  if (a->t > 0 && (!aligned16(a->rho_prev) || !aligned16(a->grad_prev))) return PGDTO_ERR_ARG;
  if (!(a->alpha_max > 0.0) || !(a->alpha_fallback > 0.0) || !(a->omega > 0.0) || !(a->eps_alpha >= 0.0))
    return PGDTO_ERR_ARG;
  if (a->cg_rule != PGDTO_CG_PR_PLUS && a->cg_rule != PGDTO_CG_FR && a->cg_rule != PGDTO_CG_NONE) return PGDTO_ERR_ARG;
  const void* ins[] = {a->rho, a->grad, a->rho_prev, a->grad_prev};
  for (const void* p : ins)
    if (p && (overlaps(pr->x, bytes, p, bytes) || overlaps(a->dir, bytes, p, bytes))) return PGDTO_ERR_ARG;
  if (overlaps(pr->x, bytes, a->dir, bytes)) return PGDTO_ERR_ARG;
  if (a->work) {
    // compaction scratch: may reuse rho_prev / grad_prev (read in the first pass only)
    if (!aligned16(a->work)) return PGDTO_ERR_ARG;
    const size_t abytes = pr->kind == PGDTO_INDEPENDENT
                              ? bytes : ((size_t)(pr->m - 1) * (size_t)d.lda + (size_t)pr->n) * esz;
    const void* used[] = {pr->x, a->dir, a->rho, a->grad};
    for (const void* p : used)
      if (overlaps(a->work, bytes, p, bytes)) return PGDTO_ERR_ARG;
    if (overlaps(a->work, bytes, pr->A, abytes)) return PGDTO_ERR_ARG;
  }
  d.cbuf = a->work;                    // x holds rho~ during the search
  double viol = 0.0;
  for (int j = 0; j < pr->m; ++j) {
    if (!isfinite(a->g[j]) || !isfinite(a->G[j])) return PGDTO_ERR_ARG;
    d.b[j] = a->G[j] - a->g[j];           // b_j = G_j - g_j + a_j.rho_t (device adds a_j.rho_t)
    viol = std::max(viol, a->g[j] - a->G[j]);
  }
  d.cg_rule = a->cg_rule;
  d.zero_step = a->t == 0 ? 1 : 0;
  d.fallback_forced = (a->t == 0 || (a->t >= a->t_warmup && viol > a->tol_viol)) ? 1 : 0;
  d.rho = a->rho;
  d.rho_prev = a->rho_prev;
  d.grad = a->grad;
  d.grad_prev = a->grad_prev;
  d.dir = a->dir;
  d.alpha_max = a->alpha_max;
  d.alpha_fallback = a->alpha_fallback;
  d.omega = a->omega;
  d.eps_alpha = a->eps_alpha;
  d.tol_stop = a->tol;
  return PGDTO_OK;
}

}  // namespace pgdto

static const pgdto_params* params_or_default(const pgdto_params* p, pgdto_params& tmp) {
  if (p) return p;
  pgdto_params_default(&tmp);
  return &tmp;
}

extern "C" int pgdto_project_async(pgdto_ctx* c, const pgdto_problem* prob, const pgdto_params* params,
                                   pgdto_result* result_dev, void* stream) {
  if (!c || !prob || !result_dev) return PGDTO_ERR_ARG;
  pgdto_params tmp;
  const pgdto_params* pp = params_or_default(params, tmp);
  Desc d;
  int st = build_desc(prob, pp, true, d);
  if (st != PGDTO_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return PGDTO_ERR_HIP;
  return run_launch(c, d, (hipStream_t)stream, result_dev, false);
}

// Grid autotuner (pgdto_ctx_autotune): the first blocking projection of a
// shape class (kind, dtype, m, tile count) is run once per candidate grid --
// all co-resident workgroups, 1/2, 1/4, 1/8 of them -- timed with events on
// the caller's stream, and the fastest is kept for the class.  Every run gives
// the same bits (reductions follow the tiles, not the workgroups), so the
// candidate runs leave exactly the result of a plain call.
static int autotune_project(pgdto_ctx* c, const pgdto_problem* prob, const pgdto_params* params,
                            hipStream_t s) {
  pgdto_params tmp;
  const pgdto_params* pp = params_or_default(params, tmp);
  Desc d;
  int st = build_desc(prob, pp, true, d);
  if (st != PGDTO_OK) return st;
  const uint64_t key = tune_key(d);
  if (c->tuned_grid.count(key)) return PGDTO_OK;
  const int cap = coresident_cap(c, d);
  if (cap <= 0) return PGDTO_ERR_HIP;
  const int full = std::max(1, std::min(d.ntiles, cap));
  int cand[4], nc = 0;
  for (int div = 1; div <= 8; div *= 2) {
    const int g = std::max(1, full / div);
    if (nc == 0 || cand[nc - 1] != g) cand[nc++] = g;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return PGDTO_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return PGDTO_ERR_HIP; }
  int best = full;
  float best_ms = 1e30f;
  const int saved_grid = c->forced_grid;
  st = PGDTO_OK;
  for (int rep = 0; rep < 2 && st == PGDTO_OK; ++rep) {   // the first round warms up
    for (int i = 0; i < nc && st == PGDTO_OK; ++i) {
      c->forced_grid = cand[i];
      if (hipEventRecord(e0, s) != hipSuccess) { st = PGDTO_ERR_HIP; break; }
      st = pgdto_project_async(c, prob, params, (pgdto_result*)c->res_dev, s);
      if (st != PGDTO_OK) break;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { st = PGDTO_ERR_HIP; break; }
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = PGDTO_ERR_HIP; break; }
      if (rep == 1 && ms < best_ms) { best_ms = ms; best = cand[i]; }
    }
  }
  c->forced_grid = saved_grid;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == PGDTO_OK) c->tuned_grid[key] = best;
  return st;
}

extern "C" int pgdto_ctx_autotune(pgdto_ctx* c, int enable) {
  if (!c) return PGDTO_ERR_ARG;
  const int prev = c->autotune;
  c->autotune = enable ? 1 : 0;
  if (enable < 0) c->tuned_grid.clear();
  return prev;
}

// Persisted autotuner choices: a header line naming the file format, the
// library version and the device (its architecture and compute units), then
// one "key grid" line per shape class.  A file written for another device or
// library version is ignored on load, so a cache never carries a choice to
// hardware it was not measured on.
static int device_tag(int device, char* out, size_t cap) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PGDTO_ERR_HIP;
  snprintf(out, cap, "%s-%dcu", prop.gcnArchName, prop.multiProcessorCount);
  for (char* p = out; *p; ++p)
    if (*p == ' ' || *p == '\n') *p = '_';
  return PGDTO_OK;
}

extern "C" int pgdto_ctx_autotune_save(pgdto_ctx* c, const char* path) {
  if (!c || !path) return PGDTO_ERR_ARG;
  char tag[256];
  const int st = device_tag(c->device, tag, sizeof(tag));
  if (st != PGDTO_OK) return st;
  FILE* f = fopen(path, "w");
  if (!f) return PGDTO_ERR_ARG;
  fprintf(f, "pgdto-grid-tune %d %s\n", PGDTO_VERSION, tag);
  int n = 0;
  for (const auto& kv : c->tuned_grid) {
    fprintf(f, "%llu %d\n", (unsigned long long)kv.first, kv.second);
    ++n;
  }
  return fclose(f) == 0 ? n : PGDTO_ERR_ARG;
}

extern "C" int pgdto_ctx_autotune_load(pgdto_ctx* c, const char* path) {
  if (!c || !path) return PGDTO_ERR_ARG;
  char tag[256], ftag[256];
  int st = device_tag(c->device, tag, sizeof(tag));
  if (st != PGDTO_OK) return st;
  FILE* f = fopen(path, "r");
  if (!f) return PGDTO_ERR_ARG;
  int ver = 0;
  int n = 0;
  if (fscanf(f, "pgdto-grid-tune %d %255s", &ver, ftag) == 2 && ver == PGDTO_VERSION && strcmp(tag, ftag) == 0) {
    unsigned long long key;
    int grid;
    while (fscanf(f, "%llu %d", &key, &grid) == 2) {
      if (grid < 1 || grid > GMAX) continue;
      c->tuned_grid[(uint64_t)key] = grid;
      ++n;
    }
  }
  fclose(f);
  return n;
}

extern "C" int pgdto_ctx_last_launch(pgdto_ctx* c, int32_t* grid, int32_t* tiles) {
  if (!c || !grid || !tiles) return PGDTO_ERR_ARG;
  *grid = c->last_grid;
  *tiles = c->last_ntiles;
  return PGDTO_OK;
}

extern "C" int pgdto_project(pgdto_ctx* c, const pgdto_problem* prob, const pgdto_params* params,
                             pgdto_result* out, void* stream) {
  if (!c || !prob || !out) return PGDTO_ERR_ARG;
  if (c->autotune) {
    if (hipSetDevice(c->device) != hipSuccess) return PGDTO_ERR_HIP;
    const int ts = autotune_project(c, prob, params, (hipStream_t)stream);
    if (ts != PGDTO_OK) return ts;
  }
  int st = pgdto_project_async(c, prob, params, (pgdto_result*)c->res_dev, stream);
  if (st != PGDTO_OK) return st;
  st = finish_blocking(c, (hipStream_t)stream, sizeof(pgdto_result), out);
  if (st != PGDTO_OK) return st;
  return out->error ? out->error : PGDTO_OK;
}

extern "C" int pgdto_pgd_step_async(pgdto_ctx* c, const pgdto_pgd_args* args, const pgdto_params* params,
                                    pgdto_pgd_out* out_dev, void* stream) {
  if (!c || !args || !out_dev) return PGDTO_ERR_ARG;
  pgdto_params tmp;
  const pgdto_params* pp = params_or_default(params, tmp);
  Desc d;
  pgdto_problem pr = args->proj;
  // b is formed on the device; give the validator a finite stand-in
  double zeros[PGDTO_MAX_BLOCKS] = {0};
  pr.b = zeros;
  int st = build_desc(&pr, pp, false, d);
  if (st != PGDTO_OK) return st;
  st = fill_pgd(args, d);
  if (st != PGDTO_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return PGDTO_ERR_HIP;
  return run_launch(c, d, (hipStream_t)stream, out_dev, true);
}

extern "C" int pgdto_pgd_step(pgdto_ctx* c, const pgdto_pgd_args* args, const pgdto_params* params,
                              pgdto_pgd_out* out, void* stream) {
  if (!c || !args || !out) return PGDTO_ERR_ARG;
  int st = pgdto_pgd_step_async(c, args, params, (pgdto_pgd_out*)c->res_dev, stream);
  if (st != PGDTO_OK) return st;
  st = finish_blocking(c, (hipStream_t)stream, sizeof(pgdto_pgd_out), out);
  if (st != PGDTO_OK) return st;
  return out->proj.error ? out->proj.error : PGDTO_OK;
}

extern "C" int pgdto_kappa_path(pgdto_ctx* c, const pgdto_problem* prob, const pgdto_params* params,
                                const double* C_values, int count, double tau, pgdto_path_point* points,
                                void* stream) {
  if (!c || !prob || !C_values || !points || count < 1 || count > 64 || !(tau >= 0.0) || !isfinite(tau))
    return PGDTO_ERR_ARG;
  for (int i = 0; i < count; ++i) {
    const double Ci = C_values[i];
    if (isnan(Ci) || Ci == 0.0 || Ci == -INFINITY) return PGDTO_ERR_ARG;
  }
  pgdto_problem p = *prob;
  double warm[PGDTO_MAX_BLOCKS];
  for (int i = 0; i < count; ++i) {
    p.C = C_values[i];
    pgdto_result r;
    int st = pgdto_project(c, &p, params, &r, stream);
    if (st != PGDTO_OK) return st;
    pgdto_path_point& pt = points[i];
    memset(&pt, 0, sizeof(pt));
    pt.C = C_values[i];
    pt.kappa = r.kappa;
    pt.dist = sqrt(fmax(r.dist2, 0.0));
    pt.outcome = r.outcome;
    pt.passes = r.passes;
    double vmax = 0.0;
    bool warm_ok = true;
    for (int j = 0; j < p.m; ++j) {
      const bool eq = (p.eq_mask >> j) & 1ull;
      pt.lambda[j] = r.lambda[j];
      pt.slack[j] = r.slack[j];
      pt.violation[j] = eq ? fabs(r.resid[j]) : fmax(r.resid[j], 0.0);
      vmax = fmax(vmax, pt.violation[j]);
      warm[j] = r.lambda[j];
      warm_ok = warm_ok && isfinite(r.lambda[j]) && (eq || r.lambda[j] >= 0.0);
    }
    pt.max_violation = vmax;
    pt.violation_over_tau = tau > 0.0 ? vmax / tau : 0.0;
    // the next point starts from these multipliers (continuation)
    p.lambda0 = warm_ok ? warm : nullptr;
  }
  return PGDTO_OK;
}
