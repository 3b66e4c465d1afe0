// Serving bookkeeping shared by the request front end and the executors.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "pgdto_internal.h"

namespace pgdto {

struct Request {
  uint64_t ticket = 0;
  int state = 0;
  pgdto_problem prob{};
  pgdto_params params{};
  int m = 0;
  double b[PGDTO_MAX_BLOCKS] = {};
  int64_t off[PGDTO_MAX_BLOCKS + 1] = {};
  double lam0[PGDTO_MAX_BLOCKS] = {};   // warm start copied at submit (warm != 0)
  int warm = 0;
  size_t footprint = 0;
  // an Algorithm 3 step instead of a projection (pgd != 0): args with its
  // host arrays (g, G, block offsets) pointing into this request
  int pgd = 0;
  pgdto_pgd_args args{};
  double g[PGDTO_MAX_BLOCKS] = {}, G[PGDTO_MAX_BLOCKS] = {};

  // the problem / step arguments with their host arrays bound to this copy
  pgdto_problem problem() const;
  pgdto_pgd_args pgd_args() const;
};

struct Record {
  int state;                 // PGDTO_QUEUED / PGDTO_PENDING / PGDTO_OK / error
  pgdto_pgd_out out;         // projections use out.proj only
  int64_t t_submit, t_start, t_done;   // host monotonic clock, ns
  int pgd;
};

size_t request_footprint(const pgdto_problem& p);
int build_request_desc(const Request& r, Desc& d);   // validation + descriptor (host only)

struct Server;   // slot-based persistent executor (pgdto_server.cpp)

}  // namespace pgdto

struct pgdto_batch {
  pgdto_ctx* ctx = nullptr;
  pgdto_batch_cfg cfg{};
  std::mutex mu;
  std::condition_variable cv;        // work available / state change
  std::condition_variable done_cv;   // a request finished
  std::deque<pgdto::Request> queue;
  std::unordered_map<uint64_t, pgdto::Record> records;
  uint64_t next_ticket = 1;
  bool stopping = false;
  int64_t n_admitted = 0, n_completed = 0, n_in_flight = 0;
  size_t bytes_in_flight = 0, peak_bytes = 0;
  // plain executor
  std::thread worker;
  pgdto_ctx* plain_ctx = nullptr;
  hipStream_t plain_stream = nullptr;
  // persistent executor
  pgdto::Server* server = nullptr;

  int start();
  void stop();
  int submit(const pgdto::Request& r, uint64_t* ticket);
  int poll(uint64_t ticket, pgdto_pgd_out* out, bool wait, int64_t* times, int* is_pgd);
  void finish(uint64_t ticket, int status, const pgdto_pgd_out& res, size_t footprint, int64_t t_start,
              int64_t t_done);
  bool pop_admissible(pgdto::Request& r, size_t slots_free);
  void cancel_queued();
  void run_plain();
};

namespace pgdto {
int server_start(pgdto_batch* b);
void server_stop(pgdto_batch* b);
int server_shape(pgdto_batch* b, int* slots, int* wg);
}  // namespace pgdto
