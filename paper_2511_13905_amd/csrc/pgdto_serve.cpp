// Batch / serving front end of the C ABI.
//
// Requests are queued on submit and retired through poll/wait.  Admission
// keeps the summed footprint (y, A, x bytes) of the requests in flight under
// the configured HBM budget.  This file holds the request bookkeeping and the
// one-at-a-time executor; the slot-based persistent executor lives in
// pgdto_server.cpp.

#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pgdto_ctx.h"
#include "pgdto_internal.h"
#include "pgdto_serve.h"

namespace pgdto {

static int64_t clock_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t request_footprint(const pgdto_problem& p) {
  const size_t esz = p.dtype == PGDTO_F32 ? 4 : 8;
  const size_t n = (size_t)p.n;
  const size_t rows = p.kind == PGDTO_INDEPENDENT ? 1 : (size_t)p.m;
  return esz * n * (rows + 2);
}

pgdto_problem Request::problem() const {
  pgdto_problem p = pgd ? args.proj : prob;
  p.b = pgd ? nullptr : b;
  p.block_offsets = p.kind == PGDTO_INDEPENDENT ? off : nullptr;
  p.lambda0 = warm ? lam0 : nullptr;
  return p;
}

pgdto_pgd_args Request::pgd_args() const {
  pgdto_pgd_args a = args;
  a.proj = problem();
  a.g = g;
  a.G = G;
  return a;
}

// Host-side validation and the launch descriptor of a request (the same
// checks as pgdto_project / pgdto_pgd_step).
int build_request_desc(const Request& r, Desc& d) {
  if (!r.pgd) {
    const pgdto_problem p = r.problem();
    const int st = build_desc(&p, &r.params, true, d);
    // the served kernel runs the register-accumulating coupled solver only
    return (st == PGDTO_OK && is_wide(d)) ? PGDTO_ERR_ARG : st;
  }
  const pgdto_pgd_args a = r.pgd_args();
  pgdto_problem pr = a.proj;
  double zeros[PGDTO_MAX_BLOCKS] = {0};   // b is formed on the device
  pr.b = zeros;
  int st = build_desc(&pr, &r.params, false, d);
  if (st != PGDTO_OK) return st;
  return fill_pgd(&a, d);
}

}  // namespace pgdto

using namespace pgdto;

extern "C" int pgdto_batch_create(pgdto_ctx* ctx, const pgdto_batch_cfg* cfg, pgdto_batch** out) {
  if (!ctx || !out) return PGDTO_ERR_ARG;
  *out = nullptr;
  pgdto_batch_cfg c{};
  if (cfg) c = *cfg;
  if (c.max_slots < 0 || c.wg_per_slot < 0 || c.queue_capacity < 0) return PGDTO_ERR_ARG;
  if (c.queue_capacity == 0) c.queue_capacity = 65536;
  if (hipSetDevice(ctx->device) != hipSuccess) return PGDTO_ERR_HIP;
  if (c.hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return PGDTO_ERR_HIP;
    c.hbm_budget_bytes = (size_t)(0.9 * (double)fr);
  }
  pgdto_batch* b = new (std::nothrow) pgdto_batch();
  if (!b) return PGDTO_ERR_NOMEM;
  b->ctx = ctx;
  b->cfg = c;
  int st = b->start();
  if (st != PGDTO_OK) {
    delete b;
    return st;
  }
  *out = b;
  return PGDTO_OK;
}

extern "C" int pgdto_batch_submit(pgdto_batch* b, const pgdto_problem* prob, const pgdto_params* params,
                                  uint64_t* ticket) {
  if (!b || !prob || !ticket) return PGDTO_ERR_ARG;
  pgdto_params pp;
  if (params) pp = *params; else pgdto_params_default(&pp);
  // validate now (host only) so that a bad request fails at submit
  Desc d;
  int st = build_desc(prob, &pp, true, d);
  if (st != PGDTO_OK) return st;
  if (is_wide(d)) return PGDTO_ERR_ARG;     // served instances: at most SMALL_M coupled rows
  Request r;
  r.prob = *prob;
  r.params = pp;
  r.m = prob->m;
  for (int j = 0; j < prob->m; ++j) r.b[j] = prob->b[j];
  if (prob->kind == PGDTO_INDEPENDENT)
    for (int j = 0; j <= prob->m; ++j) r.off[j] = prob->block_offsets[j];
  if (prob->lambda0) {
    r.warm = 1;
    for (int j = 0; j < prob->m; ++j) r.lam0[j] = prob->lambda0[j];
  }
  // host arrays live in the request from here on: the descriptor is built
  // again at admission, after this call has returned
  r.prob.b = nullptr;
  r.prob.block_offsets = nullptr;
  r.prob.lambda0 = nullptr;
  r.footprint = request_footprint(*prob);
  if (r.footprint > b->cfg.hbm_budget_bytes) return PGDTO_ERR_NOMEM;
  return b->submit(r, ticket);
}

extern "C" int pgdto_batch_submit_pgd(pgdto_batch* b, const pgdto_pgd_args* args, const pgdto_params* params,
                                      uint64_t* ticket) {
  if (!b || !args || !ticket || !args->g || !args->G) return PGDTO_ERR_ARG;
  const pgdto_problem* prob = &args->proj;
  if (prob->m < 1 || prob->m > PGDTO_MAX_BLOCKS) return PGDTO_ERR_ARG;
  if (prob->kind == PGDTO_INDEPENDENT && !prob->block_offsets) return PGDTO_ERR_ARG;
  Request r;
  if (params) r.params = *params; else pgdto_params_default(&r.params);
  r.pgd = 1;
  r.args = *args;
  r.m = prob->m;
  for (int j = 0; j < prob->m; ++j) { r.g[j] = args->g[j]; r.G[j] = args->G[j]; }
  if (prob->kind == PGDTO_INDEPENDENT)
    for (int j = 0; j <= prob->m; ++j) r.off[j] = prob->block_offsets[j];
  if (prob->lambda0) {
    r.warm = 1;
    for (int j = 0; j < prob->m; ++j) r.lam0[j] = prob->lambda0[j];
  }
  r.args.proj.b = nullptr;
  r.args.proj.block_offsets = nullptr;
  r.args.proj.lambda0 = nullptr;
  r.args.g = nullptr;
  r.args.G = nullptr;
  Desc d;
  int st = build_request_desc(r, d);        // validate now (host only)
  if (st != PGDTO_OK) return st;
  const size_t esz = prob->dtype == PGDTO_F32 ? 4 : 8;
  r.footprint = request_footprint(*prob) + esz * (size_t)prob->n * 5;   // + rho, rho_prev, grad, grad_prev, d
  if (r.footprint > b->cfg.hbm_budget_bytes) return PGDTO_ERR_NOMEM;
  return b->submit(r, ticket);
}

static int poll_result(pgdto_batch* b, uint64_t ticket, pgdto_result* out, int64_t* times, bool wait) {
  pgdto_pgd_out o;
  int is_pgd = 0;
  const int st = b->poll(ticket, &o, wait, times, &is_pgd);
  if (st == PGDTO_OK || st < 0) *out = o.proj;
  return st;
}

extern "C" int pgdto_batch_poll(pgdto_batch* b, uint64_t ticket, pgdto_result* out) {
  if (!b || !out) return PGDTO_ERR_ARG;
  return poll_result(b, ticket, out, nullptr, false);
}

extern "C" int pgdto_batch_wait(pgdto_batch* b, uint64_t ticket, pgdto_result* out) {
  if (!b || !out) return PGDTO_ERR_ARG;
  return poll_result(b, ticket, out, nullptr, true);
}

extern "C" int pgdto_batch_poll_timed(pgdto_batch* b, uint64_t ticket, pgdto_result* out, int64_t* times,
                                      int wait) {
  if (!b || !out || !times) return PGDTO_ERR_ARG;
  return poll_result(b, ticket, out, times, wait != 0);
}

extern "C" int pgdto_batch_poll_pgd(pgdto_batch* b, uint64_t ticket, pgdto_pgd_out* out, int64_t* times,
                                    int wait) {
  if (!b || !out) return PGDTO_ERR_ARG;
  int is_pgd = 0;
  return b->poll(ticket, out, wait != 0, times, &is_pgd);
}

extern "C" int pgdto_batch_shape(pgdto_batch* b, int32_t* slots, int32_t* wg_per_slot) {
  if (!b || !slots || !wg_per_slot) return PGDTO_ERR_ARG;
  int s = 0, w = 0;
  if (b->server && server_shape(b, &s, &w) != PGDTO_OK) return PGDTO_ERR_ARG;
  *slots = s;
  *wg_per_slot = w;
  return PGDTO_OK;
}

extern "C" int pgdto_batch_stats(pgdto_batch* b, int64_t* admitted, int64_t* completed, int64_t* queued,
                                 int64_t* in_flight, int64_t* peak_bytes) {
  if (!b) return PGDTO_ERR_ARG;
  std::lock_guard<std::mutex> lk(b->mu);
  if (admitted) *admitted = b->n_admitted;
  if (completed) *completed = b->n_completed;
  if (queued) *queued = (int64_t)b->queue.size();
  if (in_flight) *in_flight = b->n_in_flight;
  if (peak_bytes) *peak_bytes = (int64_t)b->peak_bytes;
  return PGDTO_OK;
}

extern "C" int pgdto_batch_destroy(pgdto_batch* b) {
  if (!b) return PGDTO_ERR_ARG;
  b->stop();
  delete b;
  return PGDTO_OK;
}

// ------------------------------------------------------------------ shape autotuner

// Times the persistent executor at each candidate shape (slots x workgroups
// per slot, all co-resident workgroups split evenly) on `count` requests
// drawn round-robin from the samples, all submitted at once, twice per shape
// (the faster run counts), and reports the shape with the shortest wall time
// from the first submit to the last completion.
extern "C" int pgdto_batch_autotune(pgdto_ctx* ctx, const pgdto_problem* samples, int nsamples,
                                    const pgdto_params* params, int count, int32_t* slots,
                                    int32_t* wg_per_slot, float* times_ms) {
  if (!ctx || !samples || nsamples < 1 || count < 1 || !slots || !wg_per_slot) return PGDTO_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return PGDTO_ERR_HIP;
  const int cap = server_coresident(ctx->device);
  if (cap <= 0) return PGDTO_ERR_HIP;
  std::vector<pgdto_problem> reqs(nsamples);
  for (int i = 0; i < nsamples; ++i) {
    reqs[i] = samples[i];
    reqs[i].free_mask = nullptr;   // copies of one sample write identical x, and no mask
    if (reqs[i].dtype != PGDTO_F32) return PGDTO_ERR_ARG;
  }
  int best_s = 0, best_w = 0;
  float best_ms = INFINITY;
  for (int c = 0; c < PGDTO_TUNE_SHAPES; ++c) {
    const int s = 4 << c;
    const int w = cap / s;
    float shape_ms = INFINITY;
    if (w >= 1 && w <= GMAX) {
      for (int rep = 0; rep < 2; ++rep) {
        pgdto_batch_cfg cfg{};
        cfg.max_slots = s;
        cfg.wg_per_slot = w;
        cfg.slots_only = 1;
        pgdto_batch* b = nullptr;
        int st = pgdto_batch_create(ctx, &cfg, &b);
        if (st != PGDTO_OK) return st;
        std::vector<uint64_t> tk(count);
        const int64_t t0 = clock_ns();
        for (int i = 0; i < count && st == PGDTO_OK; ++i) st = pgdto_batch_submit(b, &reqs[i % nsamples], params, &tk[i]);
        int64_t t1 = t0;
        for (int i = 0; i < count && st == PGDTO_OK; ++i) {
          pgdto_result r;
          int64_t tm[3];
          st = pgdto_batch_poll_timed(b, tk[i], &r, tm, 1);
          t1 = std::max(t1, tm[2]);
        }
        (void)pgdto_batch_destroy(b);
        if (st != PGDTO_OK) return st;
        shape_ms = std::min(shape_ms, (float)((t1 - t0) * 1e-6));
      }
      if (shape_ms < best_ms) { best_ms = shape_ms; best_s = s; best_w = w; }
    }
    if (times_ms) times_ms[c] = shape_ms;
  }
  if (best_s == 0) return PGDTO_ERR_HIP;
  *slots = best_s;
  *wg_per_slot = best_w;
  return PGDTO_OK;
}

// ------------------------------------------------------------------ pgdto_batch

int pgdto_batch::submit(const Request& r0, uint64_t* ticket) {
  std::lock_guard<std::mutex> lk(mu);
  if (stopping) return PGDTO_ERR_CANCELLED;
  if ((int)queue.size() >= cfg.queue_capacity) return PGDTO_ERR_BUSY;
  Request r = r0;
  r.ticket = next_ticket++;
  r.state = PGDTO_QUEUED;
  records[r.ticket] = Record{PGDTO_QUEUED, {}, clock_ns(), 0, 0, r.pgd};
  queue.push_back(r);
  *ticket = r.ticket;
  cv.notify_all();
  return PGDTO_OK;
}

int pgdto_batch::poll(uint64_t ticket, pgdto_pgd_out* out, bool wait, int64_t* times, int* is_pgd) {
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    auto it = records.find(ticket);
    if (it == records.end()) return PGDTO_ERR_UNKNOWN_TICKET;
    const int st = it->second.state;
    if (is_pgd) *is_pgd = it->second.pgd;
    if (st == PGDTO_OK || st < 0) {
      *out = it->second.out;
      if (times) {
        times[0] = it->second.t_submit;
        times[1] = it->second.t_start;
        times[2] = it->second.t_done;
      }
      records.erase(it);
      return st;
    }
    if (!wait) return st;
    done_cv.wait(lk);
  }
}

void pgdto_batch::finish(uint64_t ticket, int status, const pgdto_pgd_out& res, size_t footprint, int64_t t_start,
                         int64_t t_done) {
  std::lock_guard<std::mutex> lk(mu);
  auto it = records.find(ticket);
  if (it != records.end()) {
    it->second.state = status;
    it->second.out = res;
    it->second.t_start = t_start;
    it->second.t_done = t_done;
  }
  n_completed += 1;
  n_in_flight -= 1;
  bytes_in_flight -= footprint;
  done_cv.notify_all();
  cv.notify_all();
}

// Admits the next request if the budget and a free executor allow it.
bool pgdto_batch::pop_admissible(Request& r, size_t slots_free) {
  if (queue.empty() || slots_free == 0) return false;
  const Request& h = queue.front();
  if (bytes_in_flight + h.footprint > cfg.hbm_budget_bytes && n_in_flight > 0) return false;
  r = h;
  queue.pop_front();
  bytes_in_flight += r.footprint;
  peak_bytes = std::max(peak_bytes, bytes_in_flight);
  n_in_flight += 1;
  n_admitted += 1;
  auto it = records.find(r.ticket);
  if (it != records.end()) it->second.state = PGDTO_PENDING;
  return true;
}

void pgdto_batch::cancel_queued() {
  std::lock_guard<std::mutex> lk(mu);
  for (auto& r : queue) {
    auto it = records.find(r.ticket);
    if (it != records.end()) {
      it->second.state = PGDTO_ERR_CANCELLED;
      memset(&it->second.out, 0, sizeof(pgdto_pgd_out));
    }
  }
  queue.clear();
  done_cv.notify_all();
}

// One-at-a-time executor: the plain per-request path (FIFO, eager launches).
void pgdto_batch::run_plain() {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    Request r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stopping || !queue.empty(); });
      if (stopping && queue.empty()) return;
      if (!pop_admissible(r, 1)) continue;
    }
    pgdto_pgd_out res;
    memset(&res, 0, sizeof(res));
    const int64_t t0 = clock_ns();
    int st;
    if (r.pgd) {
      const pgdto_pgd_args a = r.pgd_args();
      st = pgdto_pgd_step(plain_ctx, &a, &r.params, &res, (void*)plain_stream);
    } else {
      const pgdto_problem p = r.problem();
      st = pgdto_project(plain_ctx, &p, &r.params, &res.proj, (void*)plain_stream);
    }
    if (st == PGDTO_OK && res.proj.error != 0) st = res.proj.error;
    finish(r.ticket, st, res, r.footprint, t0, clock_ns());
  }
}

// max_slots == 1: the plain one-at-a-time executor; otherwise the persistent
// multi-slot server.
int pgdto_batch::start() {
  if (cfg.max_slots != 1) return server_start(this);
  if (hipStreamCreateWithFlags(&plain_stream, hipStreamNonBlocking) != hipSuccess) return PGDTO_ERR_HIP;
  int st = pgdto_ctx_create(ctx->device, &plain_ctx);
  if (st != PGDTO_OK) return st;
  worker = std::thread([this] { run_plain(); });
  return PGDTO_OK;
}

void pgdto_batch::stop() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stopping = true;
    cv.notify_all();
  }
  if (server) {
    // in-flight requests finish; queued ones are cancelled
    cancel_queued();
    server_stop(this);
  }
  if (worker.joinable()) worker.join();
  cancel_queued();
  if (plain_ctx) pgdto_ctx_destroy(plain_ctx);
  if (plain_stream) (void)hipStreamDestroy(plain_stream);
}
