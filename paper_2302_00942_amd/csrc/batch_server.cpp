// Batched integration and the serving loop (filled in after the single-cloud path).
#include "rfd_internal.h"

extern "C" {

rfd_status rfd_integrate_batch(rfd_plan_t* plans, const float* const* Xs, const int64_t* Ns, const float* const* Fs,
                               const int64_t* ldFs, const int32_t* ds, float* const* outs, const int64_t* ldOs,
                               int32_t n, rfd_stream_t stream) {
  (void)plans; (void)Xs; (void)Ns; (void)Fs; (void)ldFs; (void)ds; (void)outs; (void)ldOs; (void)n; (void)stream;
  return RFD_ERR_INVALID_ARG;
}

rfd_status rfd_server_create(size_t hbm_budget_bytes, int32_t max_inflight, rfd_server_t* out) {
  (void)hbm_budget_bytes; (void)max_inflight;
  if (out) *out = nullptr;
  return RFD_ERR_INVALID_ARG;
}

rfd_status rfd_submit(rfd_server_t server, const rfd_request* req, uint64_t* ticket) {
  (void)server; (void)req; (void)ticket;
  return RFD_ERR_INVALID_ARG;
}

rfd_status rfd_wait(rfd_server_t server, uint64_t ticket, double timeout_s, rfd_result* res) {
  (void)server; (void)ticket; (void)timeout_s; (void)res;
  return RFD_ERR_INVALID_ARG;
}

void rfd_server_destroy(rfd_server_t server) { (void)server; }

}  // extern "C"
