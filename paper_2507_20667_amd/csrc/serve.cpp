// Serving entry points (continuous batching); filled in below the executor.
#include "tn_internal.h"

namespace tn {

struct ServeState {};

void serve_shutdown(tn_ctx *ctx) { (void)ctx; }

}  // namespace tn

extern "C" {

tn_status tn_serve_submit(tn_ctx *ctx, const tn_query *query, uint64_t *ticket) {
  (void)ctx;
  (void)query;
  (void)ticket;
  tn::set_error("tn_serve_submit: serving is not available in this build");
  return TN_E_INVALID_ARG;
}

tn_status tn_serve_poll(tn_ctx *ctx, uint64_t ticket, void *out, tn_dtype out_dtype,
                        double *log2_scale, double *latency_s) {
  (void)ctx;
  (void)ticket;
  (void)out;
  (void)out_dtype;
  (void)log2_scale;
  (void)latency_s;
  tn::set_error("tn_serve_poll: serving is not available in this build");
  return TN_E_UNKNOWN_TICKET;
}

}  // extern "C"
