// cs_serve.cpp -- batched ensembles and the queued request server.
#include "cs_internal.h"
#include "cs_runtime.h"

extern "C" {
cs_status cs_queue_start(cs_ctx* ctx, int slots, uint64_t resident_budget) {
  (void)ctx; (void)slots; (void)resident_budget;
  return cs::fail(CS_EUNSUPPORTED, "queue: not built yet");
}
cs_status cs_queue_submit(cs_ctx* ctx, const cs_req* req, uint64_t* ticket) {
  (void)ctx; (void)req; (void)ticket;
  return cs::fail(CS_EUNSUPPORTED, "queue: not built yet");
}
cs_status cs_queue_poll(cs_ctx* ctx, uint64_t ticket, cs_result* out, double* timing) {
  (void)ctx; (void)ticket; (void)out; (void)timing;
  return cs::fail(CS_EUNSUPPORTED, "queue: not built yet");
}
cs_status cs_queue_drain(cs_ctx* ctx) { (void)ctx; return CS_OK; }
cs_status cs_queue_stop(cs_ctx* ctx) { (void)ctx; return CS_OK; }
}
