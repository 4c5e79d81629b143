// Fitting entry points (device-resident BFGS).
#include "host.h"

using namespace uml;

extern "C" {

void uml_fit_options_default(uml_fit_options* o) {
  if (!o) return;
  o->edm_tol = 1e-6;
  o->max_iter = 1000;
  o->polish = 0;
  o->want_cov = 1;
}

int uml_eval_hessian(const uml_model*, const uml_data*, const double*, double*, double*, double*,
                     double*, void*) {
  return set_error(UML_E_UNSUPPORTED, "uml_eval_hessian: not built yet");
}

int uml_fit(const uml_model*, const uml_data*, const double*, const uml_fit_options*,
            uml_fit_result*) {
  return set_error(UML_E_UNSUPPORTED, "uml_fit: not built yet");
}

int uml_fit_batch(const uml_model*, const uml_data* const*, int32_t, const double*,
                  const uml_fit_options*, uml_fit_result*) {
  return set_error(UML_E_UNSUPPORTED, "uml_fit_batch: not built yet");
}

}  // extern "C"
