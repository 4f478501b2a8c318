// lpa_serve.cpp -- serving scheduler (filled in below).
#include "lpa_host.hpp"

namespace lpa {
lpa_status serve_init(lpa_ctx*) { return LPA_OK; }
void serve_shutdown(lpa_ctx*) {}
}  // namespace lpa

using namespace lpa;
extern "C" {
lpa_status lpa_submit(lpa_rig*, const lpa_frame*, const lpa_params*, const lpa_output*, int64_t, uint64_t*) {
  return set_error(LPA_ERR_UNSUPPORTED, "serving not built yet");
}
lpa_status lpa_poll(lpa_ctx* ctx, uint64_t, lpa_result* r) {
  if (!ctx || !r) return set_error(LPA_ERR_INVALID_ARG, "context or result is NULL");
  return set_error(LPA_ERR_UNSUPPORTED, "serving not built yet");
}
lpa_status lpa_drain(lpa_ctx*) { return LPA_OK; }
}
