// Serving runtime (continuous batching) -- placeholder until the slot
// kernel lands; every entry point reports QPX_ERR_UNSUPPORTED.
#include "../../include/qpx.h"

extern "C" {
int qp_server_create(qpx_ctx *, const qp_server_opts *, const qp_opts *, qpx_server **srv) {
  if (srv) *srv = nullptr;
  return QPX_ERR_UNSUPPORTED;
}
int qp_serve_submit(qpx_server *, int32_t, int32_t, int32_t, const float *, const float *,
                    const float *, const float *, const float *, const float *, uint64_t *) {
  return QPX_ERR_UNSUPPORTED;
}
int qp_serve_poll(qpx_server *, uint64_t, float *, float *, float *, float *, qp_timing *) {
  return QPX_ERR_UNSUPPORTED;
}
int qp_serve_stats(qpx_server *, uint64_t *, uint64_t *, int32_t *) { return QPX_ERR_UNSUPPORTED; }
int qp_server_destroy(qpx_server *) { return QPX_OK; }
}
