// Slot-based persistent executor for pgdto_batch (continuous batching).
// Placeholder until the multi-slot kernel lands: runs the plain executor.
#include "pgdto_ctx.h"
#include "pgdto_serve.h"

namespace pgdto {

int server_start(pgdto_batch* b) {
  b->worker = std::thread([b] { b->run_plain(); });
  return PGDTO_OK;
}

void server_stop(pgdto_batch*) {}

}  // namespace pgdto
