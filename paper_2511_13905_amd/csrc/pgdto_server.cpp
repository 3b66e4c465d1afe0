// Host side of the persistent multi-slot executor (continuous batching).
//
// One thread per batch object admits queued requests (within the HBM budget)
// as job descriptors into a pinned ring, publishes them by advancing `tail`,
// retires finished jobs from the pinned completion words, and keeps the
// server kernel running while work is outstanding.  Requests that arrive
// while others are on the device are admitted as soon as the ring and the
// budget allow; slots of the running launch claim them as they free up, so
// requests of different sizes and kinds overlap on the device.
//
// At light load (one request waiting, nothing on the device) the request
// runs instead as one full-GPU launch: a slot holds only 1/slots of the GPU,
// so a lone request finishes sooner on all of it.  Both routes give the same
// bits (reductions follow the tiles, not the workgroups).

#include <hip/hip_runtime.h>

#include <string.h>

#include <chrono>
#include <thread>
#include <vector>

#include "pgdto_ctx.h"
#include "pgdto_internal.h"
#include "pgdto_serve.h"

namespace pgdto {

namespace {
int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
}  // namespace

struct Server {
  pgdto_batch* b = nullptr;
  int slots = 0, wg = 0, qcap = 0;
  SrvHostCtl* ctl = nullptr;     // pinned
  Desc* jobs = nullptr;          // pinned [qcap]
  uint64_t* done = nullptr;      // pinned [qcap]
  pgdto_pgd_out* results = nullptr;  // pinned [qcap]
  uint64_t* head = nullptr;      // device
  uint64_t* slot_words = nullptr;    // device
  double* part = nullptr;        // device
  uint64_t* sync = nullptr;      // device
  hipStream_t stream = nullptr;
  bool running = false;
  // full-GPU route for a lone request
  pgdto_ctx* os_ctx = nullptr;
  hipStream_t os_stream = nullptr;
  hipEvent_t os_event = nullptr;
  pgdto_pgd_out* os_res = nullptr;   // pinned
  bool os_busy = false;
  uint64_t os_ticket = 0;
  size_t os_footprint = 0;
  int64_t os_t_start = 0;
  int64_t n_oneshot = 0;
  uint64_t launches = 0;
  uint64_t published = 0;        // jobs written and published
  uint64_t oldest = 0;           // oldest job not yet retired
  struct Out {
    uint64_t ticket;
    size_t footprint;
    int64_t t_start;
    bool retired;
  };
  std::vector<Out> out;          // [qcap], indexed by job % qcap
  std::thread th;

  int init();
  void release();
  void loop();
  bool retire();
  bool admit();
  bool oneshot();
  int ensure_running();
  void fail_stranded();
};

int Server::init() {
  if (hipSetDevice(b->ctx->device) != hipSuccess) return PGDTO_ERR_HIP;
  const int cap = server_coresident(b->ctx->device);
  if (cap <= 0) return PGDTO_ERR_HIP;
  slots = b->cfg.max_slots > 0 ? b->cfg.max_slots : 8;
  wg = b->cfg.wg_per_slot > 0 ? b->cfg.wg_per_slot : cap / slots;
  if (wg < 1 || slots * wg > cap || wg > GMAX) return PGDTO_ERR_ARG;
  qcap = 256;
  out.assign(qcap, Out{0, 0, 0, true});
  bool ok = true;
  ok = ok && hipHostMalloc((void**)&ctl, sizeof(SrvHostCtl), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&jobs, sizeof(Desc) * qcap, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&done, sizeof(uint64_t) * qcap, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&results, sizeof(pgdto_pgd_out) * qcap, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMalloc(&head, 256) == hipSuccess;
  ok = ok && hipMalloc(&slot_words, sizeof(uint64_t) * 16 * slots) == hipSuccess;
  ok = ok && hipMalloc(&part, sizeof(double) * PART_DOUBLES * slots) == hipSuccess;
  ok = ok && hipMalloc(&sync, sizeof(uint64_t) * SYNC_WORDS * slots) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&os_stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&os_event, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&os_res, sizeof(pgdto_pgd_out), hipHostMallocDefault) == hipSuccess;
  ok = ok && pgdto_ctx_create(b->ctx->device, &os_ctx) == PGDTO_OK;
  if (!ok) return PGDTO_ERR_NOMEM;
  memset(ctl, 0, sizeof(SrvHostCtl));
  memset(jobs, 0, sizeof(Desc) * qcap);
  memset(done, 0, sizeof(uint64_t) * qcap);
  memset(results, 0, sizeof(pgdto_pgd_out) * qcap);
  ok = ok && hipMemset(head, 0, 256) == hipSuccess;
  ok = ok && hipMemset(slot_words, 0, sizeof(uint64_t) * 16 * slots) == hipSuccess;
  ok = ok && hipMemset(sync, 0, sizeof(uint64_t) * SYNC_WORDS * slots) == hipSuccess;
  ok = ok && hipDeviceSynchronize() == hipSuccess;
  return ok ? PGDTO_OK : PGDTO_ERR_HIP;
}

void Server::release() {
  if (stream) (void)hipStreamSynchronize(stream);
  if (ctl) (void)hipHostFree(ctl);
  if (jobs) (void)hipHostFree(jobs);
  if (done) (void)hipHostFree(done);
  if (results) (void)hipHostFree(results);
  if (head) (void)hipFree(head);
  if (slot_words) (void)hipFree(slot_words);
  if (part) (void)hipFree(part);
  if (sync) (void)hipFree(sync);
  if (stream) (void)hipStreamDestroy(stream);
  if (os_stream) (void)hipStreamSynchronize(os_stream);
  if (os_ctx) pgdto_ctx_destroy(os_ctx);
  if (os_res) (void)hipHostFree(os_res);
  if (os_event) (void)hipEventDestroy(os_event);
  if (os_stream) (void)hipStreamDestroy(os_stream);
}

// The full-GPU route: retire a finished lone launch; start one when exactly
// one request waits and nothing else is on the device.
bool Server::oneshot() {
  if (os_busy) {
    const hipError_t q = hipEventQuery(os_event);
    if (q == hipErrorNotReady) return false;
    os_busy = false;
    pgdto_pgd_out r = *os_res;
    int st = q == hipSuccess ? (r.proj.error != 0 ? r.proj.error : PGDTO_OK) : PGDTO_ERR_HIP;
    if (q != hipSuccess) {
      (void)hipGetLastError();
      memset(&r, 0, sizeof(r));
      r.proj.error = PGDTO_ERR_HIP;
    }
    b->finish(os_ticket, st, r, os_footprint, os_t_start, now_ns());
    return true;
  }
  if (b->cfg.slots_only || oldest < published) return false;
  Request r;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->queue.size() != 1 || !b->pop_admissible(r, 1)) return false;
  }
  // an idle persistent launch still holds the GPU: ask it to leave now (its
  // slots exit at their next poll of an empty queue); the full-GPU launch
  // starts right after it in device order
  if (running) __atomic_store_n(&ctl->shutdown, 1, __ATOMIC_RELEASE);
  const pgdto_problem p = r.problem();
  if (p.dtype != PGDTO_F32) {       // the persistent executor takes float32 only, on either route
    pgdto_pgd_out res;
    memset(&res, 0, sizeof(res));
    res.proj.error = PGDTO_ERR_ARG;
    b->finish(r.ticket, PGDTO_ERR_ARG, res, r.footprint, now_ns(), now_ns());
    return true;
  }
  os_ticket = r.ticket;
  os_footprint = r.footprint;
  os_t_start = now_ns();
  memset(os_res, 0, sizeof(pgdto_pgd_out));
  int st;
  if (r.pgd) {
    const pgdto_pgd_args a = r.pgd_args();
    st = pgdto_pgd_step_async(os_ctx, &a, &r.params, os_res, (void*)os_stream);
  } else {
    st = pgdto_project_async(os_ctx, &p, &r.params, &os_res->proj, (void*)os_stream);
  }
  if (st == PGDTO_OK && hipEventRecord(os_event, os_stream) != hipSuccess) st = PGDTO_ERR_HIP;
  if (st != PGDTO_OK) {
    pgdto_pgd_out res;
    memset(&res, 0, sizeof(res));
    res.proj.error = st;
    b->finish(r.ticket, st, res, r.footprint, os_t_start, now_ns());
    return true;
  }
  os_busy = true;
  n_oneshot += 1;
  return true;
}

// Retire finished jobs (completion word = job + 1).
bool Server::retire() {
  bool any = false;
  for (uint64_t j = oldest; j < published; ++j) {
    Out& o = out[j % qcap];
    if (o.retired) continue;
    const uint64_t w = __atomic_load_n(&done[j % qcap], __ATOMIC_ACQUIRE);
    if (w != j + 1) continue;
    const pgdto_pgd_out& r = results[j % qcap];
    const int st = r.proj.error != 0 ? r.proj.error : PGDTO_OK;
    b->finish(o.ticket, st, r, o.footprint, o.t_start, now_ns());
    o.retired = true;
    any = true;
  }
  while (oldest < published && out[oldest % qcap].retired) ++oldest;
  return any;
}

// Admit queued requests into free ring entries, then publish them.
bool Server::admit() {
  bool any = false;
  while (published - oldest < (uint64_t)qcap) {
    Request r;
    {
      std::lock_guard<std::mutex> lk(b->mu);
      if (!b->pop_admissible(r, 1)) break;
    }
    Desc d;
    int st = build_request_desc(r, d);
    if (st == PGDTO_OK && r.problem().dtype != PGDTO_F32) st = PGDTO_ERR_ARG;
    if (st != PGDTO_OK) {
      pgdto_pgd_out res;
      memset(&res, 0, sizeof(res));
      res.proj.error = st;
      b->finish(r.ticket, st, res, r.footprint, now_ns(), now_ns());
      continue;
    }
    const uint64_t j = published;
    d.epoch0 = (j + 1) << 20;      // per slot barrier words: epochs grow with the job index
    d.pgd = r.pgd;
    d.result = nullptr;
    d.trace = nullptr;
    jobs[j % qcap] = d;
    memset(&results[j % qcap], 0, sizeof(pgdto_pgd_out));
    __atomic_store_n(&done[j % qcap], 0, __ATOMIC_RELAXED);
    out[j % qcap] = Out{r.ticket, r.footprint, now_ns(), false};
    published = j + 1;
    any = true;
  }
  if (any) __atomic_store_n(&ctl->tail, published, __ATOMIC_RELEASE);
  return any;
}

// After the kernel ended: jobs it claimed but did not finish (a device wait
// timed out) are failed, so that no ticket waits forever.
void Server::fail_stranded() {
  uint64_t h = 0;
  if (hipMemcpy(&h, head, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return;
  for (uint64_t j = oldest; j < published && j < h; ++j) {
    Out& o = out[j % qcap];
    if (o.retired) continue;
    if (__atomic_load_n(&done[j % qcap], __ATOMIC_ACQUIRE) == j + 1) continue;
    pgdto_pgd_out res;
    memset(&res, 0, sizeof(res));
    res.proj.error = PGDTO_ERR_TIMEOUT;
    b->finish(o.ticket, PGDTO_ERR_TIMEOUT, res, o.footprint, o.t_start, now_ns());
    o.retired = true;
  }
  while (oldest < published && out[oldest % qcap].retired) ++oldest;
}

int Server::ensure_running() {
  if (running) {
    const hipError_t q = hipStreamQuery(stream);
    if (q == hipErrorNotReady) return PGDTO_OK;
    running = false;
    if (q != hipSuccess) return PGDTO_ERR_HIP;
    retire();
    fail_stranded();
  }
  if (oldest >= published) return PGDTO_OK;      // nothing outstanding
  __atomic_store_n(&ctl->shutdown, 0, __ATOMIC_RELEASE);   // no launch is running here
  SrvArgs a;
  memset(&a, 0, sizeof(a));
  a.ctl = ctl;
  a.jobs = jobs;
  a.done = done;
  a.results = results;
  a.head = head;
  a.slot_words = slot_words;
  a.part = part;
  a.sync = sync;
  a.part_stride = PART_DOUBLES;
  a.sync_stride = SYNC_WORDS;
  a.round0 = (++launches) << 32;
  a.slots = slots;
  a.wg_per_slot = wg;
  a.qcap = qcap;
  a.idle_spins = 1000;           // a few ms without a job
  if (launch_server(a, stream) != hipSuccess) {
    (void)hipGetLastError();
    return PGDTO_ERR_HIP;
  }
  running = true;
  return PGDTO_OK;
}

void Server::loop() {
  (void)hipSetDevice(b->ctx->device);
  int idle_rounds = 0;
  for (;;) {
    bool progress = retire();
    progress |= oneshot();
    progress |= admit();
    bool stop = false;
    {
      std::lock_guard<std::mutex> lk(b->mu);
      stop = b->stopping && b->queue.empty();
    }
    if (stop && oldest >= published && !os_busy) break;
    if (ensure_running() != PGDTO_OK) {
      // the launch failed: fail what is outstanding and what is queued
      for (uint64_t j = oldest; j < published; ++j) {
        Out& o = out[j % qcap];
        if (o.retired) continue;
        pgdto_pgd_out res;
        memset(&res, 0, sizeof(res));
        res.proj.error = PGDTO_ERR_HIP;
        b->finish(o.ticket, PGDTO_ERR_HIP, res, o.footprint, o.t_start, now_ns());
        o.retired = true;
      }
      oldest = published;
      b->cancel_queued();
    }
    if (progress) {
      idle_rounds = 0;
      continue;
    }
    // nothing changed: spin briefly, then sleep in short steps
    if (++idle_rounds < 64) {
      std::this_thread::yield();
    } else {
      std::unique_lock<std::mutex> lk(b->mu);
      b->cv.wait_for(lk, std::chrono::microseconds(oldest < published || os_busy ? 20 : 2000));
    }
  }
  __atomic_store_n(&ctl->shutdown, 1, __ATOMIC_RELEASE);
  if (running) (void)hipStreamSynchronize(stream);
  running = false;
}

int server_start(pgdto_batch* b) {
  Server* s = new (std::nothrow) Server();
  if (!s) return PGDTO_ERR_NOMEM;
  s->b = b;
  const int st = s->init();
  if (st != PGDTO_OK) {
    s->release();
    delete s;
    return st;
  }
  b->server = s;
  s->th = std::thread([s] { s->loop(); });
  return PGDTO_OK;
}

void server_stop(pgdto_batch* b) {
  Server* s = b->server;
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->cv.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  s->release();
  delete s;
  b->server = nullptr;
}

int server_shape(pgdto_batch* b, int* slots, int* wg) {
  if (!b->server) return PGDTO_ERR_ARG;
  *slots = b->server->slots;
  *wg = b->server->wg;
  return PGDTO_OK;
}

}  // namespace pgdto
