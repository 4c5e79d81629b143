// Fitting entry points (device-resident BFGS).
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"
#include "scatter.h"

using namespace uml;

namespace uml {

// Events per Hessian tile: a pure function of n (so is the reduction order),
// small enough to spread a toy-sized dataset over many workgroups (at least
// 256 events, one tile per 256 events up to 65536 events), at most 4096.
static int64_t hess_tile_events(int64_t n) {
  int64_t t = 256;
  while (t < 4096 && t * 256 < n) t *= 2;
  return t;
}

// Hessian workspace: constants | hc | out | partials.
struct HessLayout {
  size_t o_cb, o_hc, o_out, o_part, bytes;
  int n_tiles, M;
};
static HessLayout hess_layout(const uml_model* m, int64_t n) {
  HessLayout L{};
  L.M = 1 + m->plan.nfree + 2 * m->hplan.npairs;
  const int64_t te = hess_tile_events(n);
  L.n_tiles = int(std::max<int64_t>(1, (n + te - 1) / te));
  L.o_cb = 0;
  L.o_hc = (sizeof(ConstBlock) + 255) / 256 * 256;
  L.o_out = L.o_hc + 256 * ((sizeof(double) * 4 * kMaxFac + 255) / 256);
  L.o_part = L.o_out + 256 * ((sizeof(double) * L.M + 255) / 256);
  L.bytes = L.o_part + sizeof(double) * size_t(L.M) * L.n_tiles;
  return L;
}

size_t hess_work_bytes(const uml_model* m, int64_t n, int* n_tiles) {
  const HessLayout L = hess_layout(m, n);
  if (n_tiles) *n_tiles = L.n_tiles;
  return L.bytes;
}

int hess_sums(const uml_model* m) { return 1 + m->plan.nfree + 2 * m->hplan.npairs; }

// The device's LDS per workgroup (160 KiB on gfx950; 64 KiB if it cannot be
// read) and its compute-unit count.
struct DevShape {
  size_t lds;
  int cus;
};
static DevShape dev_shape(int device) {
  static std::mutex mu;
  static std::map<int, DevShape> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(device);
  if (it != cache.end()) return it->second;
  int v = 0, c = 0;
  DevShape d{64 * 1024, 256};
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
    d.lds = size_t(v);
  if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && c > 0)
    d.cus = c;
  cache[device] = d;
  return d;
}

// Events staged at once by the Hessian pass of a launch of `tiles`
// workgroups: as many as LDS allows, up to one per thread (0 if even one
// event does not fit).  With more workgroups than compute units the staging
// is sized so that two workgroups share a CU (one's matrix sums overlap the
// other's event evaluation); with fewer, one workgroup takes up to all of a
// CU's LDS, so more of its threads evaluate events at once.  The sums do not
// depend on the chunk (every order is per event, and chunks are multiples of
// the matrix cores' four events), so the choice cannot change a result.
static int hess_chunk(const uml_model* m, int64_t tiles) {
  const Plan& P = m->plan;
  const int row = hess_row_len(P, m->hplan);
  const int mat = hess_mat_bytes(P, m->hplan);
  const DevShape D = dev_shape(m->device);
  const size_t margin = 8 * 1024;  // the kernel's static LDS and more
  auto fit = [&](size_t cap) {
    int chunk = kBlock;
    while (chunk > 1 && hess_lds_bytes(row, chunk, P.precision, mat) > cap) chunk /= 2;
    return hess_lds_bytes(row, chunk, P.precision, mat) > cap ? 0 : chunk;
  };
  const int shared = fit(D.lds / 2 > margin ? D.lds / 2 - margin : 0);
  if (shared < 4 || tiles > D.cus) return shared;
  return fit(D.lds - margin);
}

// Arguments of the Hessian pass of dataset d at the device parameter vector
// d_theta; its sums go to d_out, or to the dataset's workspace if d_out is
// null.
static int hess_job(const uml_model* m, const uml_data* d, const double* d_theta, double* d_out, int chunk,
                    HessJob& J, const char* fn) {
  if (!m || !d || !d_theta) return set_error(UML_E_INVALID, std::string(fn) + ": null argument");
  if (d->model != m)
    return set_error(UML_E_INVALID, std::string(fn) + ": data was created for another model");
  if (!m->d_hplan)
    return set_error(UML_E_UNSUPPORTED, std::string(fn) + ": " + m->hess_err);
  const Plan& P = m->plan;
  const HessLayout HL = hess_layout(m, d->n);
  if (!chunk) return set_error(UML_E_UNSUPPORTED, std::string(fn) + ": model too large for the Hessian pass");
  if (!d->d_hwork || d->hess_tiles != HL.n_tiles)
    return set_error(UML_E_INVALID, std::string(fn) + ": missing Hessian workspace");
  char* base = static_cast<char*>(d->d_hwork);
  HessArgs& A = J.A;
  A = HessArgs{};
  for (int k = 0; k < P.ndim; ++k) A.col[k] = d->job.col[k];
  A.w = d->job.w;
  A.n = d->n;
  A.plan = m->d_plan;
  A.cb = reinterpret_cast<ConstBlock*>(base + HL.o_cb);
  A.hc = reinterpret_cast<double*>(base + HL.o_hc);
  A.hplan = m->d_hplan;
  A.part = reinterpret_cast<double*>(base + HL.o_part);
  A.n_tiles = HL.n_tiles;
  A.tile_events = hess_tile_events(d->n);
  A.chunk = chunk;
  A.row_len = hess_row_len(P, m->hplan);
  A.n_sums = HL.M;
  A.mat_bytes = hess_mat_bytes(P, m->hplan);
  J.theta = d_theta;
  J.out = d_out ? d_out : reinterpret_cast<double*>(base + HL.o_out);
  return UML_OK;
}

// Queues the Hessian pass at the device parameter vector d_theta on stream s;
// the raw sums [sum w log2 P, sum w s (nfree), H pairs, W2 pairs] are copied
// to h_out (host; pinned memory keeps the call asynchronous) when the stream
// gets there.
int hessian_queue(const uml_model* m, uml_data* d, const double* d_theta, double* h_out,
                  hipStream_t s, const char* fn) {
  if (!h_out) return set_error(UML_E_INVALID, std::string(fn) + ": null argument");
  HessJob J;
  if (!m || !d) return set_error(UML_E_INVALID, std::string(fn) + ": null argument");
  int rc = hess_job(m, d, d_theta, nullptr, hess_chunk(m, hess_layout(m, d->n).n_tiles), J, fn);
  if (rc != UML_OK) return rc;
  launch_hessian(J.A, d_theta, const_cast<ConstBlock*>(J.A.cb), const_cast<double*>(J.A.hc), J.out,
                 m->plan.precision, s);
  UML_HIP_CHECK(hipGetLastError());
  UML_HIP_CHECK(hipMemcpyAsync(h_out, J.out, sizeof(double) * J.A.n_sums, hipMemcpyDeviceToHost, s));
  return UML_OK;
}

// Queues one Hessian pass over n datasets of model m (batched launches):
// dataset i at the device parameter vector d_thetas[i], its sums to
// d_outs + i * hess_sums(m).  The job table and tile map are staged through
// h_jobs / h_map (host, pinned, capacity n and map_cap) into d_jobs / d_map.
int hessian_queue_batch(const uml_model* m, uml_data* const* ds, const double* const* d_thetas, int n,
                        double* d_outs, HessJob* h_jobs, HessJob* d_jobs, int2* h_map, int2* d_map,
                        int map_cap, hipStream_t s, const char* fn) {
  if (n <= 0) return UML_OK;
  const int M = hess_sums(m);
  int64_t tiles = 0;
  for (int i = 0; i < n; ++i) {
    if (!ds[i]) return set_error(UML_E_INVALID, std::string(fn) + ": null argument");
    tiles += hess_layout(m, ds[i]->n).n_tiles;
  }
  const int chunk = hess_chunk(m, tiles);
  int n_map = 0;
  for (int i = 0; i < n; ++i) {
    int rc = hess_job(m, ds[i], d_thetas[i], d_outs + size_t(i) * M, chunk, h_jobs[i], fn);
    if (rc != UML_OK) return rc;
    for (int t = 0; t < h_jobs[i].A.n_tiles; ++t) {
      if (n_map >= map_cap) return set_error(UML_E_INVALID, std::string(fn) + ": Hessian tile map full");
      h_map[n_map++] = make_int2(i, t);
    }
  }
  UML_HIP_CHECK(hipMemcpyAsync(d_jobs, h_jobs, sizeof(HessJob) * n, hipMemcpyHostToDevice, s));
  UML_HIP_CHECK(hipMemcpyAsync(d_map, h_map, sizeof(int2) * n_map, hipMemcpyHostToDevice, s));
  launch_hessian_batch(d_jobs, n, d_map, n_map, h_jobs[0].A.row_len, h_jobs[0].A.chunk, h_jobs[0].A.mat_bytes,
                       M, m->plan.precision, s);
  UML_HIP_CHECK(hipGetLastError());
  return UML_OK;
}

// The Hessian pass for a host parameter vector, synchronously.
int hessian_host(const uml_model* m, uml_data* d, const double* theta, hipStream_t s,
                 std::vector<double>& out, const char* fn) {
  if (!m || !d || !theta) return set_error(UML_E_INVALID, std::string(fn) + ": null argument");
  std::memcpy(d->h_stage, theta, sizeof(double) * m->plan.npar);
  UML_HIP_CHECK(hipMemcpyAsync(d->d_theta, d->h_stage, sizeof(double) * m->plan.npar,
                               hipMemcpyHostToDevice, s));
  out.assign(hess_sums(m), 0.0);
  int rc = hessian_queue(m, d, d->d_theta, out.data(), s, fn);
  if (rc != UML_OK) return rc;
  UML_HIP_CHECK(hipStreamSynchronize(s));
  return UML_OK;
}

// Raw Hessian-pass sums -> NLL, gradient, Hessian, W2 (free parameters).
int unpack_hessian(const uml_model* m, const double* h, double* nll, double* grad,
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

// Inverse of a symmetric positive-definite n x n matrix (row-major, n at
// most UML_MAX_PARAMS) by Cholesky factorisation, in FP64: A = L L^T, W =
// L^-1 (lower triangular, by forward substitution), A^-1 = W^T W (formed
// symmetric).  Each diagonal element of L is divided into once.  Returns
// false if A is not PD.
bool chol_inverse(int n, const double* A, double* Ai) {
  double L[UML_MAX_PARAMS * UML_MAX_PARAMS], W[UML_MAX_PARAMS * UML_MAX_PARAMS], id[UML_MAX_PARAMS];
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0) || !std::isfinite(s)) return false;
    const double d = std::sqrt(s);
    L[j * n + j] = d;
    id[j] = 1.0 / d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t * id[j];
    }
  }
  for (int c = 0; c < n; ++c) {
    W[c * n + c] = id[c];
    for (int i = c + 1; i < n; ++i) {
      double t = 0.0;
      for (int k = c; k < i; ++k) t -= L[i * n + k] * W[k * n + c];
      W[i * n + c] = t * id[i];
    }
  }
  for (int a = 0; a < n; ++a)
    for (int b = a; b < n; ++b) {
      double t = 0.0;
      for (int k = b; k < n; ++k) t += W[k * n + a] * W[k * n + b];
      Ai[a * n + b] = Ai[b * n + a] = t;
    }
  return true;
}

// The start metric: the inverse of the analytic Hessian at the start point
// (its diagonal inverse if the Hessian is not positive definite there).
int metric_from_sums(const uml_model* m, const double* h, double* V0, double* nll0, const char* fn) {
  const int nf = m->plan.nfree;
  double H[UML_MAX_PARAMS * UML_MAX_PARAMS], Vi[UML_MAX_PARAMS * UML_MAX_PARAMS];
  int rc = unpack_hessian(m, h, nll0, nullptr, H, nullptr, fn);
  if (rc != UML_OK) return rc;
  for (int i = 0; i < UML_MAX_PARAMS * UML_MAX_PARAMS; ++i) V0[i] = 0.0;
  if (chol_inverse(nf, H, Vi)) {
    for (int i = 0; i < nf; ++i)
      for (int j = 0; j < nf; ++j) V0[i * UML_MAX_PARAMS + j] = Vi[i * nf + j];
  } else {
    for (int i = 0; i < nf; ++i) {
      const double hii = std::fabs(H[i * nf + i]);
      V0[i * UML_MAX_PARAMS + i] = hii > 0.0 ? 1.0 / hii : 1.0;
    }
  }
  return UML_OK;
}

// Final HESSE-like step at the fitted point (and optional Newton polish):
// covariance = inverse Hessian, errors, EDM with the exact Hessian.
int finish_fit(const uml_model* m, uml_data* d, std::vector<double>& theta,
               const uml_fit_options& o, uml_fit_result* r, hipStream_t s, const char* fn) {
  const Plan& P = m->plan;
  const int nf = P.nfree;
  std::vector<double> h, g(nf), H(size_t(nf) * nf), C(size_t(nf) * nf);
  for (int it = 0; it < o.polish; ++it) {  // Newton steps with the analytic Hessian
    int rc = hessian_host(m, d, theta.data(), s, h, fn);
    if (rc != UML_OK) return rc;
    if (unpack_hessian(m, h.data(), nullptr, g.data(), H.data(), nullptr, fn) != UML_OK ||
        !chol_inverse(nf, H.data(), C.data()))
      break;  // the final pass below reports the state of this point
    for (int a = 0; a < nf; ++a) {
      double st = 0.0;
      for (int b = 0; b < nf; ++b) st -= C[a * nf + b] * g[b];
      theta[P.free_idx[a]] += st;
    }
  }
  int rc = hessian_host(m, d, theta.data(), s, h, fn);
  if (rc != UML_OK) return rc;
  finish_from_sums(m, h.data(), theta.data(), o, r, fn);
  return UML_OK;
}

// Result at the fitted point from its Hessian-pass sums: NLL, EDM with the
// exact Hessian, and the covariance (with the errors its diagonal gives):
// H^-1, or for weighted fits the sandwich H^-1 W2 H^-1.
void finish_from_sums(const uml_model* m, const double* h, const double* theta,
                      const uml_fit_options& o, uml_fit_result* r, const char* fn) {
  const Plan& P = m->plan;
  const int nf = P.nfree;
  constexpr int kN2 = UML_MAX_PARAMS * UML_MAX_PARAMS;
  double g[UML_MAX_PARAMS], H[kN2], C[kN2], W2[kN2], V[kN2];
  double nll = 0.0;
  for (int k = 0; k < UML_MAX_PARAMS; ++k) r->params[k] = k < P.npar ? theta[k] : 0.0;
  if (unpack_hessian(m, h, &nll, g, H, W2, fn) != UML_OK) {
    r->status = UML_FIT_PDF_NONPOSITIVE;
    r->nll = INFINITY;
    return;
  }
  if (!chol_inverse(nf, H, C)) {
    if (r->status == UML_FIT_CONVERGED) r->status = UML_FIT_HESSIAN_NOT_PD;
    for (int i = 0; i < nf * nf; ++i) C[i] = 0.0;
  }
  double edm = 0.0;
  for (int a = 0; a < nf; ++a)
    for (int b = 0; b < nf; ++b) edm += 0.5 * g[a] * C[a * nf + b] * g[b];
  for (int i = 0; i < nf * nf; ++i) V[i] = C[i];
  if (o.cov_kind == UML_COV_SANDWICH) {  // V = C W2 C
    double T[kN2];
    for (int i = 0; i < nf * nf; ++i) T[i] = 0.0;
    for (int a = 0; a < nf; ++a)
      for (int k = 0; k < nf; ++k)
        for (int b = 0; b < nf; ++b) T[a * nf + b] += C[a * nf + k] * W2[k * nf + b];
    for (int a = 0; a < nf; ++a)
      for (int b = 0; b < nf; ++b) {
        double v = 0.0;
        for (int k = 0; k < nf; ++k) v += T[a * nf + k] * C[k * nf + b];
        V[a * nf + b] = v;
      }
  }
  for (int k = 0; k < UML_MAX_PARAMS; ++k) r->errors[k] = 0.0;
  for (int a = 0; a < nf; ++a) {
    r->errors[P.free_idx[a]] = std::sqrt(std::max(V[a * nf + a], 0.0));
    for (int b = 0; b < nf; ++b) r->cov[a * nf + b] = o.want_cov ? V[a * nf + b] : 0.0;
  }
  r->nll = nll;
  r->edm = edm;
}

// The parts of a fit's start state that need no evaluation.
void fit_state_begin(const uml_model* m, const double* start, const uml_fit_options& o, FitState& F) {
  const Plan& P = m->plan;
  std::memset(&F, 0, sizeof(F));
  for (int k = 0; k < P.npar; ++k) F.theta[k] = start[k];
  F.phase = 0;
  F.alpha = 1.0;
  F.edm = INFINITY;
  F.edm_tol = o.edm_tol;
  F.max_iter = o.max_iter;
  // NLL rounding: FP64 sums to ~1e-15 relative.  In mixed mode each
  // parameter-only constant is rounded to FP32 once per point, which moves
  // ln P of every event of a component together by up to ~2^-24 |log2 K|:
  // the NLL steps by a few 1e-8 of itself between nearby points.
  F.tol_f_rel = P.precision == UML_MIXED ? 2e-7 : 1e-14;
}

// Completes a start state from the Hessian-pass sums at the start point (the
// start metric).  A start with P <= 0 somewhere gives a finished state.
int fit_state_metric(const uml_model* m, const double* h, FitState& F, const char* fn) {
  double nll0 = 0.0;
  int rc = metric_from_sums(m, h, F.V0, &nll0, fn);
  if (rc == UML_E_PDF_NONPOSITIVE) {
    F.done = 1;
    F.status = UML_FIT_PDF_NONPOSITIVE;
    return UML_OK;
  }
  if (rc != UML_OK) return rc;
  std::memcpy(F.V, F.V0, sizeof(F.V));
  return UML_OK;
}

// A fit's device state at its start point, synchronously.
int init_fit_state(const uml_model* m, uml_data* d, const double* start, const uml_fit_options& o,
                   FitState& F, hipStream_t s, const char* fn) {
  fit_state_begin(m, start, o, F);
  std::vector<double> h;
  int rc = hessian_host(m, d, start, s, h, fn);
  if (rc != UML_OK) return rc;
  return fit_state_metric(m, h.data(), F, fn);
}

int check_fit_options(const uml_fit_options& o, const char* fn) {
  if (!(o.edm_tol > 0.0) || !std::isfinite(o.edm_tol) || o.max_iter < 1 || o.polish < 0 ||
      o.polish > 16 || (o.cov_kind != UML_COV_HESSE && o.cov_kind != UML_COV_SANDWICH) ||
      (o.method != UML_METHOD_BFGS && o.method != UML_METHOD_NEWTON))
    return set_error(UML_E_INVALID, std::string(fn) +
                                        ": fit options out of range (edm_tol > 0, max_iter >= 1, "
                                        "0 <= polish <= 16, cov_kind HESSE or SANDWICH, method "
                                        "BFGS or NEWTON)");
  return UML_OK;
}

// Newton iterations with the analytic Hessian: each iteration is one
// Hessian pass (NLL, gradient, Hessian at the current point) and a Newton
// step, shortened by backtracking until the Armijo condition holds (event
// kernel evaluations).  With exact second derivatives the minimisation takes
// a few iterations (the analytic-derivative fits of Sec. 3.2-3.3).  Where the
// Hessian is not positive definite the step uses its inverse diagonal.
// Stops at EDM = 0.5 g^T H^-1 g < edm_tol; the last Hessian pass gives the
// covariance, so no pass is added at the end.
static int newton_fit(const uml_model* m, uml_data* d, const double* start, const uml_fit_options& o,
                      uml_fit_result* r, const char* fn) {
  const Plan& P = m->plan;
  const int nf = P.nfree;
  const double tol_f_rel = P.precision == UML_MIXED ? 2e-7 : 1e-14;
  std::vector<double> th(start, start + P.npar), tt(P.npar), h, g(nf), H(size_t(nf) * nf),
      C(size_t(nf) * nf), p(nf);
  int status = UML_FIT_MAX_ITER, it = 0, n_eval = 0;
  for (;; ++it) {
    int rc = hessian_host(m, d, th.data(), nullptr, h, fn);
    if (rc != UML_OK) return rc;
    ++n_eval;
    double f = 0.0;
    if (unpack_hessian(m, h.data(), &f, g.data(), H.data(), nullptr, fn) != UML_OK) {
      status = UML_FIT_PDF_NONPOSITIVE;  // only at the start: steps to +inf are rejected
      break;
    }
    const bool pd = chol_inverse(nf, H.data(), C.data());
    if (!pd) {
      std::fill(C.begin(), C.end(), 0.0);
      for (int a = 0; a < nf; ++a) {
        const double haa = std::fabs(H[a * nf + a]);
        C[a * nf + a] = haa > 0.0 ? 1.0 / haa : 1.0;
      }
    }
    double gp = 0.0;
    for (int a = 0; a < nf; ++a) {
      double pa = 0.0;
      for (int b = 0; b < nf; ++b) pa -= C[a * nf + b] * g[b];
      p[a] = pa;
      gp += g[a] * pa;
    }
    const double edm = -0.5 * gp;
    if (pd && edm < o.edm_tol) {
      status = UML_FIT_CONVERGED;
      break;
    }
    if (it >= o.max_iter) break;
    bool accepted = false;
    double alpha = 1.0;
    for (int ls = 0; ls < 40 && !accepted; ++ls, alpha *= 0.5) {
      tt = th;
      for (int a = 0; a < nf; ++a) tt[P.free_idx[a]] += alpha * p[a];
      double ft = 0.0;
      rc = uml_eval_nll(m, d, tt.data(), &ft, nullptr);
      ++n_eval;
      if (rc != UML_OK && rc != UML_E_PDF_NONPOSITIVE) return rc;
      accepted = rc == UML_OK && ft <= f + 1e-4 * alpha * gp + tol_f_rel * std::fabs(f);
    }
    if (!accepted) {
      status = edm < 100.0 * o.edm_tol ? UML_FIT_CONVERGED : UML_FIT_LINESEARCH_FAIL;
      break;
    }
    th.swap(tt);
  }
  r->n_free = nf;
  r->n_iter = it;
  r->n_eval = n_eval;
  r->status = status;
  if (status == UML_FIT_PDF_NONPOSITIVE) {
    for (int k = 0; k < UML_MAX_PARAMS; ++k) r->params[k] = k < P.npar ? th[k] : 0.0;
    r->nll = INFINITY;
    return UML_OK;
  }
  finish_from_sums(m, h.data(), th.data(), o, r, fn);  // h is the pass at th
  return UML_OK;
}

int fit_batch_impl(const uml_model* m, const uml_data* const* ds, int n, const double* starts,
                   const uml_fit_options* opts, uml_fit_result* out, const char* fn) {
  uml_fit_options o;
  uml_fit_options_default(&o);
  if (opts) o = *opts;
  if (int rc = check_fit_options(o, fn)) return rc;
  if (n == 0) return UML_OK;
  const Plan& P = m->plan;
  for (int i = 0; i < n; ++i) {
    if (!ds[i] || ds[i]->model != m)
      return set_error(UML_E_INVALID, std::string(fn) + ": data " + std::to_string(i) +
                                          " is null or belongs to another model");
    for (int j = 0; j < i; ++j)
      if (ds[j] == ds[i])
        return set_error(UML_E_INVALID, std::string(fn) + ": the same data handle appears twice");
  }
  if (o.method == UML_METHOD_NEWTON) {
    for (int i = 0; i < n; ++i) {
      std::memset(&out[i], 0, sizeof(uml_fit_result));
      int rc = newton_fit(m, const_cast<uml_data*>(ds[i]), starts + size_t(i) * P.npar, o, &out[i], fn);
      if (rc == UML_OK) rc = fill_bad_count(m, ds[i], &out[i], nullptr, fn);
      if (rc != UML_OK) return rc;
    }
    return UML_OK;
  }
  std::vector<FitState> fs(n);
  std::vector<int> live;
  for (int i = 0; i < n; ++i) {
    std::memset(&out[i], 0, sizeof(uml_fit_result));
    out[i].n_free = P.nfree;
    int rc = init_fit_state(m, const_cast<uml_data*>(ds[i]), starts + size_t(i) * P.npar, o, fs[i],
                            nullptr, fn);
    if (rc != UML_OK) return rc;
    if (!fs[i].done) live.push_back(i);
  }
  // device state: fit states | jobs | tile map
  int total_tiles = 0;
  for (int i : live) total_tiles += ds[i]->n_tiles;
  const size_t o_fs = 0, o_job = (sizeof(FitState) * n + 255) / 256 * 256;
  const size_t o_map = o_job + (sizeof(Job) * n + 255) / 256 * 256;
  const size_t bytes = o_map + sizeof(int2) * std::max(total_tiles, 1);
  if (m->fitws_bytes < bytes) {  // the model's fit workspace and its staging, grown on demand
    if (m->d_fitws) (void)hipFree(m->d_fitws);
    if (m->h_fitstage) (void)hipHostFree(m->h_fitstage);
    m->d_fitws = nullptr;
    m->h_fitstage = nullptr;
    m->fitws_bytes = 0;
    hipError_t e = hipMalloc(&m->d_fitws, bytes);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&m->h_fitstage), bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      if (m->d_fitws) (void)hipFree(m->d_fitws);
      if (m->h_fitstage) (void)hipHostFree(m->h_fitstage);
      m->d_fitws = nullptr;
      m->h_fitstage = nullptr;
      return set_error(UML_E_NOMEM, std::string(fn) + ": " + hipGetErrorString(e));
    }
    m->fitws_bytes = bytes;
  }
  if (m->fitdone_n < n) {  // the done flags' mapped pinned buffer, grown on demand
    if (m->h_fitdone) (void)hipHostFree(m->h_fitdone);
    m->h_fitdone = m->h_fitdone_dev = nullptr;
    m->fitdone_n = 0;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&m->h_fitdone), sizeof(int) * n, hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&m->h_fitdone_dev), m->h_fitdone, 0);
    if (e != hipSuccess) {
      if (m->h_fitdone) (void)hipHostFree(m->h_fitdone);
      m->h_fitdone = m->h_fitdone_dev = nullptr;
      return set_error(UML_E_NOMEM, std::string(fn) + ": " + hipGetErrorString(e));
    }
    m->fitdone_n = n;
  }
  char* base = static_cast<char*>(m->d_fitws);
  FitState* d_fs = reinterpret_cast<FitState*>(base + o_fs);
  Job* d_jobs = reinterpret_cast<Job*>(base + o_job);
  int2* d_map = reinterpret_cast<int2*>(base + o_map);
  std::vector<Job> jobs(n);
  for (int i = 0; i < n; ++i) {
    jobs[i] = ds[i]->job;
    jobs[i].fit = d_fs + i;
    jobs[i].theta = d_fs[i].theta;
    jobs[i].out = d_fs[i].out;
  }
  hipStream_t s = nullptr;
  auto build_map = [&](std::vector<int2>& map) {
    map.clear();
    for (int i : live)
      for (int t = 0; t < ds[i]->n_tiles; ++t) map.push_back(make_int2(i, t));
  };
  std::vector<int2> map;
  build_map(map);
  // fit states, jobs and map in one copy from the pinned staging (same layout)
  char* stage = m->h_fitstage;
  std::memcpy(stage + o_fs, fs.data(), sizeof(FitState) * n);
  std::memcpy(stage + o_job, jobs.data(), sizeof(Job) * n);
  if (!map.empty()) std::memcpy(stage + o_map, map.data(), sizeof(int2) * map.size());
  UML_HIP_CHECK(hipMemcpyAsync(base, stage, o_map + sizeof(int2) * map.size(), hipMemcpyHostToDevice, s));
  const int* done = m->h_fitdone;
  int launches = 0, since_poll = 0, poll_every = 2;
  const int max_launches = std::max(1, o.max_iter) * 64 + 64;
  while (!map.empty() && launches < max_launches) {
    LaunchArgs a{};
    a.job0 = jobs[0];
    a.jobs = d_jobs;
    a.tmap = d_map;
    a.grid = int(map.size());
    a.precision = P.precision;
    a.stream = s;
    m->family->eval(a);
    UML_HIP_CHECK(hipGetLastError());
    ++launches;
    if (++since_poll < poll_every) continue;
    since_poll = 0;
    poll_every = std::min(poll_every * 2, 16);
    launch_collect_ints(&d_fs[0].done, int64_t(sizeof(FitState)), n, m->h_fitdone_dev, s);
    UML_HIP_CHECK(hipGetLastError());
    UML_HIP_CHECK(hipStreamSynchronize(s));
    std::vector<int> still;
    for (int i : live)
      if (!done[i]) still.push_back(i);
    if (still.size() != live.size()) {
      live.swap(still);
      build_map(map);
      if (!map.empty()) {  // (the staging's earlier copies have completed: the poll waited)
        std::memcpy(stage + o_map, map.data(), sizeof(int2) * map.size());
        UML_HIP_CHECK(hipMemcpyAsync(d_map, stage + o_map, sizeof(int2) * map.size(), hipMemcpyHostToDevice, s));
      }
      poll_every = 2;
    }
  }
  UML_HIP_CHECK(hipMemcpyAsync(stage + o_fs, d_fs, sizeof(FitState) * n, hipMemcpyDeviceToHost, s));
  UML_HIP_CHECK(hipStreamSynchronize(s));
  std::memcpy(fs.data(), stage + o_fs, sizeof(FitState) * n);
  for (int i = 0; i < n; ++i) {
    FitState& F = fs[i];
    uml_fit_result& r = out[i];
    r.n_free = P.nfree;
    r.n_iter = F.n_iter;
    r.n_eval = F.n_eval;
    r.status = F.done ? F.status : UML_FIT_MAX_ITER;
    std::vector<double> theta(F.theta, F.theta + P.npar);
    if (!F.done)
      for (int a = 0; a < P.nfree; ++a) theta[P.free_idx[a]] = F.x[a];
    int rc = UML_OK;
    if (r.status == UML_FIT_PDF_NONPOSITIVE) {
      for (int k = 0; k < P.npar; ++k) r.params[k] = theta[k];
      r.nll = INFINITY;
    } else {
      rc = finish_fit(m, const_cast<uml_data*>(ds[i]), theta, o, &r, nullptr, fn);
    }
    if (rc == UML_OK) rc = fill_bad_count(m, ds[i], &r, nullptr, fn);
    if (rc != UML_OK) return rc;
  }
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
  o->cov_kind = UML_COV_HESSE;
  o->method = UML_METHOD_BFGS;
}

int uml_eval_hessian(const uml_model* m, const uml_data* d, const double* theta_all, double* nll,
                     double* grad_free, double* hess_free, double* w2_free, void* stream) {
  std::vector<double> h;
  int rc = hessian_host(m, const_cast<uml_data*>(d), theta_all, static_cast<hipStream_t>(stream), h,
                        "uml_eval_hessian");
  if (rc != UML_OK) return rc;
  return unpack_hessian(m, h.data(), nll, grad_free, hess_free, w2_free, "uml_eval_hessian");
}

int uml_fit(const uml_model* m, const uml_data* d, const double* start_all,
            const uml_fit_options* opts, uml_fit_result* out) {
  const uml_data* ds[1] = {d};
  if (!m) return set_error(UML_E_INVALID, "uml_fit: null model");
  std::vector<double> st(m->plan.npar);
  for (int k = 0; k < m->plan.npar; ++k) st[k] = start_all ? start_all[k] : m->theta0[k];
  return fit_batch_impl(m, ds, 1, st.data(), opts, out, "uml_fit");
}

int uml_fit_batch(const uml_model* m, const uml_data* const* ds, int32_t n_fits, const double* starts,
                  const uml_fit_options* opts, uml_fit_result* out) {
  if (!m || !ds || n_fits < 0 || (n_fits > 0 && (!starts || !out)))
    return set_error(UML_E_INVALID, "uml_fit_batch: bad argument");
  return fit_batch_impl(m, ds, n_fits, starts, opts, out, "uml_fit_batch");
}

}  // extern "C"
