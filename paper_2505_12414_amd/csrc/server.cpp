// Serving loop for many pseudo-experiment fits.
#include "host.h"

using namespace uml;

extern "C" {

void uml_server_options_default(uml_server_options* o) {
  if (!o) return;
  o->max_slots = 256;
  o->hbm_budget = int64_t(4) << 30;
  o->max_pending = 1 << 20;
  uml_fit_options_default(&o->fit);
}
int uml_server_create(const uml_model*, const uml_server_options*, uml_server** out) {
  if (out) *out = nullptr;
  return set_error(UML_E_UNSUPPORTED, "uml_server_create: not built yet");
}
int uml_server_submit(uml_server*, const uml_request*, uint64_t*) {
  return set_error(UML_E_UNSUPPORTED, "uml_server_submit: not built yet");
}
int uml_server_poll(uml_server*, uml_fit_result*, int32_t, int32_t*, int32_t) {
  return set_error(UML_E_UNSUPPORTED, "uml_server_poll: not built yet");
}
int uml_server_stats_get(uml_server*, uml_server_stats*) {
  return set_error(UML_E_UNSUPPORTED, "uml_server_stats_get: not built yet");
}
int uml_server_drain(uml_server*) {
  return set_error(UML_E_UNSUPPORTED, "uml_server_drain: not built yet");
}
void uml_server_destroy(uml_server*) {}

}  // extern "C"
