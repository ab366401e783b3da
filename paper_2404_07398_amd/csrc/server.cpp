// Serving entry points (continuous batching); filled in by the batched engine.
#include "internal.h"

using namespace ifl;

extern "C" {

ifl_status ifl_server_create(size_t, int32_t, ifl_server** out) {
  if (out) *out = nullptr;
  return fail(IFL_EUNSUPPORTED, "serving is not built yet");
}
ifl_status ifl_server_add(ifl_server*, ifl_handle*, int32_t*) { return fail(IFL_EUNSUPPORTED, "serving is not built yet"); }
ifl_status ifl_submit(ifl_server*, int32_t, const double*, int32_t, const double*, double*, ifl_ticket**) {
  return fail(IFL_EUNSUPPORTED, "serving is not built yet");
}
ifl_status ifl_wait(ifl_ticket*, ifl_solve_stats*) { return fail(IFL_EUNSUPPORTED, "serving is not built yet"); }
int32_t ifl_poll(const ifl_ticket*) { return 0; }
double ifl_ticket_latency(const ifl_ticket*) { return 0.0; }
void ifl_server_destroy(ifl_server*) {}

}
