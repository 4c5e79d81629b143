// Fitting entry points (device-resident BFGS).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host.h"

using namespace uml;

namespace uml {

constexpr int64_t kHessTileEvents = 4096;

// Runs the Hessian pass for theta (host) and returns the raw sums
// [sum w log2 P, sum w s (nfree), H pairs, W2 pairs].
int hessian_host(const uml_model* m, uml_data* d, const double* theta, hipStream_t s,
                 std::vector<double>& out, const char* fn) {
  if (!m || !d || !theta) return set_error(UML_E_INVALID, std::string(fn) + ": null argument");
  if (d->model != m)
    return set_error(UML_E_INVALID, std::string(fn) + ": data was created for another model");
  if (!m->d_hplan)
    return set_error(UML_E_UNSUPPORTED, std::string(fn) + ": " + m->hess_err);
  const Plan& P = m->plan;
  const int row = hess_row_len(P, m->hplan);
  const int M = 1 + P.nfree + 2 * m->hplan.npairs;
  const int n_tiles = int(std::max<int64_t>(1, (d->n + kHessTileEvents - 1) / kHessTileEvents));
  const size_t fixed = hess_lds_bytes(row, 0, P.precision);
  const size_t esz = P.precision == UML_MIXED ? 4 : 8;
  int chunk = 64;
  while (chunk > 1 && fixed + size_t(row) * chunk * esz > 60 * 1024) chunk /= 2;
  if (fixed + size_t(row) * chunk * esz > 64 * 1024)
    return set_error(UML_E_UNSUPPORTED, std::string(fn) + ": model too large for the Hessian pass");
  // workspace: constants | hc | out | partials
  const size_t o_cb = 0, o_hc = (sizeof(ConstBlock) + 255) / 256 * 256;
  const size_t o_out = o_hc + 256 * ((sizeof(double) * 4 * kMaxFac + 255) / 256);
  const size_t o_part = o_out + 256 * ((sizeof(double) * M + 255) / 256);
  if (!d->d_hwork || d->hess_tiles != n_tiles) {
    if (d->d_hwork) (void)hipFree(d->d_hwork);
    d->d_hwork = nullptr;
    hipError_t e = hipMalloc(&d->d_hwork, o_part + sizeof(double) * size_t(M) * n_tiles);
    if (e != hipSuccess) {
      d->d_hwork = nullptr;
      return set_error(UML_E_NOMEM, std::string(fn) + ": " + hipGetErrorString(e));
    }
    d->hess_tiles = n_tiles;
  }
  char* base = static_cast<char*>(d->d_hwork);
  HessArgs A{};
  for (int k = 0; k < P.ndim; ++k) A.col[k] = d->job.col[k];
  A.w = d->job.w;
  A.n = d->n;
  A.plan = m->d_plan;
  A.cb = reinterpret_cast<ConstBlock*>(base + o_cb);
  A.hc = reinterpret_cast<double*>(base + o_hc);
  A.hplan = m->d_hplan;
  A.part = reinterpret_cast<double*>(base + o_part);
  A.n_tiles = n_tiles;
  A.tile_events = kHessTileEvents;
  A.chunk = chunk;
  A.row_len = row;
  A.n_sums = M;
  std::memcpy(d->h_stage, theta, sizeof(double) * P.npar);
  UML_HIP_CHECK(hipMemcpyAsync(d->d_theta, d->h_stage, sizeof(double) * P.npar,
                               hipMemcpyHostToDevice, s));
  launch_hessian(A, d->d_theta, reinterpret_cast<ConstBlock*>(base + o_cb),
                 reinterpret_cast<double*>(base + o_hc), reinterpret_cast<double*>(base + o_out),
                 P.precision, s);
  UML_HIP_CHECK(hipGetLastError());
  out.assign(M, 0.0);
  UML_HIP_CHECK(hipMemcpyAsync(out.data(), base + o_out, sizeof(double) * M, hipMemcpyDeviceToHost, s));
  UML_HIP_CHECK(hipStreamSynchronize(s));
  return UML_OK;
}

// Raw Hessian-pass sums -> NLL, gradient, Hessian, W2 (free parameters).
int unpack_hessian(const uml_model* m, const std::vector<double>& h, double* nll, double* grad,
                   double* hess, double* w2, const char* fn) {
  const int nf = m->plan.nfree, np = m->hplan.npairs;
  const double v = -0.69314718055994530942 * h[0];
  bool bad = !std::isfinite(v);
  for (int k = 0; k < 1 + nf + 2 * np && !bad; ++k) bad = !std::isfinite(h[k]);
  if (nll) *nll = bad ? INFINITY : v;
  for (int a = 0; a < nf; ++a)
    if (grad) grad[a] = bad ? 0.0 : -h[1 + a];
  for (int p = 0; p < np; ++p) {
    const int a = m->hplan.pa[p], b = m->hplan.pb[p];
    if (hess) hess[a * nf + b] = hess[b * nf + a] = bad ? 0.0 : h[1 + nf + p];
    if (w2) w2[a * nf + b] = w2[b * nf + a] = bad ? 0.0 : h[1 + nf + np + p];
  }
  if (bad)
    return set_error(UML_E_PDF_NONPOSITIVE, std::string(fn) +
                     ": P <= 0 or non-finite at some event, or parameters outside the model's domain");
  return UML_OK;
}

}  // namespace uml

extern "C" {

void uml_fit_options_default(uml_fit_options* o) {
  if (!o) return;
  o->edm_tol = 1e-6;
  o->max_iter = 1000;
  o->polish = 0;
  o->want_cov = 1;
}

int uml_eval_hessian(const uml_model* m, const uml_data* d, const double* theta_all, double* nll,
                     double* grad_free, double* hess_free, double* w2_free, void* stream) {
  std::vector<double> h;
  int rc = hessian_host(m, const_cast<uml_data*>(d), theta_all, static_cast<hipStream_t>(stream), h,
                        "uml_eval_hessian");
  if (rc != UML_OK) return rc;
  return unpack_hessian(m, h, nll, grad_free, hess_free, w2_free, "uml_eval_hessian");
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
