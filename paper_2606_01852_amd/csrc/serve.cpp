// Continuous-batching server: placeholder until the scheduler lands.
#include "serve.hpp"

namespace tnc {
struct Server {};
std::shared_ptr<Server> make_server(Ctx&, int, int) { fail(TNC_E_UNSUPPORTED, "serving not built"); }
}  // namespace tnc

using namespace tnc;

extern "C" {
tnc_status tnc_serve_start(tnc_ctx, int32_t, int32_t) {
  g_error_set("serving not built");
  return TNC_E_UNSUPPORTED;
}
tnc_status tnc_serve_stop(tnc_ctx) { return TNC_OK; }
tnc_status tnc_submit(tnc_ctx, tnc_plan, int64_t, int64_t, double*, tnc_req*) {
  g_error_set("serving not built");
  return TNC_E_UNSUPPORTED;
}
tnc_status tnc_poll(tnc_ctx, tnc_req, int32_t*, double*) {
  g_error_set("serving not built");
  return TNC_E_UNSUPPORTED;
}
tnc_status tnc_wait(tnc_ctx, tnc_req, double*) {
  g_error_set("serving not built");
  return TNC_E_UNSUPPORTED;
}
}
