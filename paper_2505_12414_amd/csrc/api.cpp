// extern "C" entry points of libuml: models, event data and evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"
#include "scatter.h"

namespace uml {

static thread_local std::string g_err;

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

static int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Pinned host staging blocks of datasets (parameter vectors going up,
// results coming down), carved from pinned allocations of 256 blocks that
// live until the process ends: creating a dataset does not pay for a pinned
// allocation, which is slow.
namespace {
constexpr size_t kStageBytes = 1152;  // >= 4 (UML_MAX_PARAMS + 2) doubles, 128-byte multiple
static_assert(kStageBytes >= sizeof(double) * 4 * (UML_MAX_PARAMS + 2), "staging block too small");
std::mutex g_stage_mu;
std::vector<double*> g_stage_free;
}  // namespace

double* pinned_stage_get() {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  if (g_stage_free.empty()) {
    constexpr int kBlocks = 256;
    char* p = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&p), kStageBytes * kBlocks, hipHostMallocDefault) !=
        hipSuccess)
      return nullptr;
    for (int i = kBlocks - 1; i >= 0; --i) g_stage_free.push_back(reinterpret_cast<double*>(p + i * kStageBytes));
  }
  double* b = g_stage_free.back();
  g_stage_free.pop_back();
  return b;
}

void pinned_stage_put(double* p) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  g_stage_free.push_back(p);
}

int convert_events(const Plan& P, int64_t n, const void* const* cols, int32_t dtype, const void* w,
                   std::vector<char>& host, const char* fn) {
  if (n < 0) return set_error(UML_E_INVALID, std::string(fn) + ": negative event count");
  if (dtype != UML_F32 && dtype != UML_F64)
    return set_error(UML_E_INVALID, std::string(fn) + ": dtype must be UML_F32 or UML_F64");
  if (n > 0 && !cols) return set_error(UML_E_INVALID, std::string(fn) + ": cols is NULL");
  if (n > 0)
    for (int ud = 0; ud < P.ndim; ++ud)
      if (!cols[ud]) return set_error(UML_E_INVALID, std::string(fn) + ": column pointer is NULL");
  const bool mixed = P.precision == UML_MIXED;
  const size_t esz = mixed ? 4 : 8;
  const int ncols = P.ndim + (w ? 1 : 0);
  const int64_t stride = align_up(std::max<int64_t>(n, 1), 64);  // elements per column
  host.assign(size_t(stride) * esz * ncols, 0);
  for (int kd = 0; kd < ncols; ++kd) {
    const bool is_w = kd == P.ndim;
    const int ud = is_w ? -1 : P.user_of_dim[kd];
    const void* sp = is_w ? w : (n > 0 ? cols[ud] : nullptr);
    const double lo = is_w ? 0 : P.lo[kd], hi = is_w ? 0 : P.hi[kd];
    char* dst = host.data() + size_t(kd) * stride * esz;
    for (int64_t i = 0; i < n; ++i) {
      double v = dtype == UML_F32 ? double(static_cast<const float*>(sp)[i])
                                  : static_cast<const double*>(sp)[i];
      double stored = mixed ? double(float(v)) : v;
      if (is_w) {
        if (!std::isfinite(stored))
          return set_error(UML_E_EVENT_DOMAIN,
                           std::string(fn) + ": weight " + std::to_string(i) + " is not finite");
      } else if (!(stored >= lo && stored <= hi)) {
        return set_error(UML_E_EVENT_DOMAIN,
                         std::string(fn) + ": event " + std::to_string(i) + " dimension " +
                             std::to_string(ud) + " value " + std::to_string(v) +
                             " is outside [" + std::to_string(lo) + ", " + std::to_string(hi) +
                             "] or NaN" + (mixed ? " (after rounding to FP32)" : ""));
      }
      if (mixed)
        reinterpret_cast<float*>(dst)[i] = float(stored);
      else
        reinterpret_cast<double*>(dst)[i] = stored;
    }
  }
  return UML_OK;
}

DataLayout data_layout(const Plan& P, int64_t n, bool weighted) {
  DataLayout L{};
  const size_t esz = P.precision == UML_MIXED ? 4 : 8;
  L.stride = align_up(std::max<int64_t>(n, 1), 64);
  // columns: the dimensions, the weights, then any precomputed terms (the
  // host buffer of an upload fills the first part)
  L.bytes_events = size_t(L.stride) * esz * (P.ncol + (weighted ? 1 : 0));
  L.E = events_per_thread(n, P.precision);
  const int64_t tsize = int64_t(L.E) * kBlock;
  L.n_tiles = int(std::max<int64_t>(1, (n + tsize - 1) / tsize));
  // work area: job | constants | theta | out | counters | bad-event count | partials
  L.o_job = 0;
  L.o_cst = align_up(L.o_job + sizeof(Job), 256);
  L.o_theta = align_up(L.o_cst + sizeof(ConstBlock), 256);
  L.o_out = align_up(L.o_theta + sizeof(double) * UML_MAX_PARAMS, 256);
  L.o_cnt = align_up(L.o_out + sizeof(double) * (1 + UML_MAX_PARAMS), 256);
  L.o_bad = align_up(L.o_cnt + sizeof(unsigned) * kCounterWords, 256);
  L.o_epoch = align_up(L.o_bad + sizeof(unsigned long long), 256);
  L.o_part = align_up(L.o_epoch + sizeof(unsigned long long), 256);
  L.o_spart = align_up(L.o_part + sizeof(double) * P.K * (L.n_tiles + kGroups), 256);
  L.bytes_work = L.o_spart + 2 * sizeof(double) * P.K * L.n_tiles;
  return L;
}

void data_bind(uml_data* d, const uml_model* m, int64_t n, bool weighted, const DataLayout& L,
               void* d_events, void* d_work) {
  const Plan& P = m->plan;
  const size_t esz = P.precision == UML_MIXED ? 4 : 8;
  d->model = m;
  d->n = n;
  d->weighted = weighted ? 1 : 0;
  d->E = L.E;
  d->n_tiles = L.n_tiles;
  d->bytes_events = int64_t(L.bytes_events);
  d->bytes_work = int64_t(L.bytes_work);
  d->d_events = d_events;
  d->d_work = d_work;
  char* wbase = static_cast<char*>(d_work);
  d->d_job = reinterpret_cast<Job*>(wbase + L.o_job);
  d->d_theta = reinterpret_cast<double*>(wbase + L.o_theta);
  d->d_out = reinterpret_cast<double*>(wbase + L.o_out);
  d->d_bad = reinterpret_cast<unsigned long long*>(wbase + L.o_bad);
  Job& J = d->job;
  std::memset(&J, 0, sizeof(J));
  for (int kd = 0; kd < P.ndim; ++kd)
    J.col[kd] = static_cast<char*>(d_events) + size_t(kd) * L.stride * esz;
  J.w = weighted ? static_cast<char*>(d_events) + size_t(P.ndim) * L.stride * esz : nullptr;
  for (int kc = P.ndim; kc < P.ncol; ++kc)
    J.col[kc] = static_cast<char*>(d_events) + size_t(kc + (weighted ? 1 : 0)) * L.stride * esz;
  J.n = n;
  J.n_tiles = L.n_tiles;
  J.events_per_thread = L.E;
  J.cst = reinterpret_cast<ConstBlock*>(wbase + L.o_cst);
  J.partials = reinterpret_cast<double*>(wbase + L.o_part);
  J.spart = reinterpret_cast<double*>(wbase + L.o_spart);
  J.epoch = reinterpret_cast<unsigned long long*>(wbase + L.o_epoch);
  J.counter = reinterpret_cast<unsigned int*>(wbase + L.o_cnt);
  J.out = d->d_out;
  J.plan = m->d_plan;
  J.fit = nullptr;
  J.theta = d->d_theta;
  J.npar = P.npar;
  J.key = P.key;
}

// The precomputed event-only terms of a model that stores them (nothing
// otherwise), from the dataset's event columns.
hipError_t data_precompute(uml_data* d, hipStream_t s) {
  const Plan& P = d->model->plan;
  if (P.pre_fac < 0 || d->n <= 0) return hipSuccess;
  const FactorPlan& F = P.fac[P.pre_fac];
  PrecomputeArgs a{};
  for (int k = 0; k < 3; ++k) a.in[k] = d->job.col[F.dim[k]];
  for (int k = 0; k < kPWaveTerms; ++k) a.out[k] = const_cast<void*>(d->job.col[F.pre + k]);
  a.n = d->n;
  launch_pwave_terms(a, P.precision, s);
  return hipGetLastError();
}

// The work area of a freshly placed dataset: counters and caches cleared,
// the job descriptor copied.
hipError_t data_init_work(uml_data* d, const DataLayout& L, hipStream_t s) {
  hipError_t e = data_precompute(d, s);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(d->d_work, 0, L.o_part, s);
  if (e == hipSuccess) {
    launch_fill_sentinel(d->job.spart, 2 * int64_t(d->model->plan.K) * L.n_tiles, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(d->d_job, &d->job, sizeof(Job), hipMemcpyHostToDevice, s);
  return e;
}

hipError_t data_upload(uml_data* d, const DataLayout& L, const std::vector<char>& host, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(d->d_events, host.data(), host.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = data_init_work(d, L, s);
  return e;
}

// Unfolds the subtree at node id into steps of G, with `cont` the step that
// follows it; returns its entry step, or -2 if the steps exceed the plan.  A
// product is no step of its own: its children are chained in order, the
// last one followed by `cont`.  A node under two parents is unfolded once
// under each.
static int gen_unfold(GenPlan& G, int id, int cont) {
  const GenNode& nd = G.node[id];
  if (nd.kind == UML_PROD) {
    int c = cont;
    for (int k = nd.nchild - 1; k >= 0 && c != -2; --k) c = gen_unfold(G, nd.child[k], c);
    return c;
  }
  if (G.nstep >= kMaxGenSteps) return -2;
  const int s = G.nstep++;
  G.step[s] = GenStep{nd.kind, id, cont, {-1, -1}};
  if (nd.kind == UML_SUM) {
    const int a = gen_unfold(G, nd.child[0], cont);
    const int b = a == -2 ? -2 : gen_unfold(G, nd.child[1], cont);
    if (b == -2) return -2;
    G.step[s].child[0] = a;
    G.step[s].child[1] = b;
  }
  return s;
}

// Parameters a model can be sampled at: fractions in [0, 1], Gaussian
// widths > 0, everything finite.
int check_generation_theta(const uml_model* m, const double* th, const char* fn) {
  const GenPlan& G = m->gplan;
  if (G.nstep < 0)
    return set_error(UML_E_UNSUPPORTED, std::string(fn) + ": the model tree unfolds into more than " +
                                            std::to_string(kMaxGenSteps) + " generation steps");
  for (int k = 0; k < G.npar; ++k)
    if (!std::isfinite(th[k]))
      return set_error(UML_E_INVALID, std::string(fn) + ": parameter " + std::to_string(k) + " is not finite");
  for (int i = 0; i < G.nnode; ++i) {
    const GenNode& nd = G.node[i];
    if (nd.kind == UML_SUM && !(th[nd.par[0]] >= 0.0 && th[nd.par[0]] <= 1.0))
      return set_error(UML_E_INVALID, std::string(fn) + ": a fraction is outside [0, 1]");
    if (nd.kind == UML_GAUSS && !(th[nd.par[1]] > 0.0))
      return set_error(UML_E_INVALID, std::string(fn) + ": a Gaussian width is not positive");
  }
  return UML_OK;
}

int count_bad_events(const uml_model* m, const uml_data* d, const double* theta, int64_t* n_bad,
                     hipStream_t s, const char* fn) {
  const Plan& P = m->plan;
  unsigned long long h = 0;
  UML_HIP_CHECK(hipMemcpyAsync(d->d_theta, theta, sizeof(double) * P.npar, hipMemcpyHostToDevice, s));
  UML_HIP_CHECK(hipMemsetAsync(d->d_bad, 0, sizeof(unsigned long long), s));
  LaunchArgs a{};
  a.job0 = d->job;
  a.grid = d->n_tiles;
  a.theta = d->d_theta;
  a.precision = P.precision;
  a.stream = s;
  m->family->count(a, d->d_bad);
  UML_HIP_CHECK(hipGetLastError());
  UML_HIP_CHECK(hipMemcpyAsync(&h, d->d_bad, sizeof(h), hipMemcpyDeviceToHost, s));
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(UML_E_HIP, std::string(fn) + ": " + hipGetErrorString(e));
  *n_bad = int64_t(h);
  return UML_OK;
}

int fill_bad_count(const uml_model* m, const uml_data* d, uml_fit_result* r, hipStream_t s,
                   const char* fn) {
  r->n_bad_events = 0;
  if (r->status != UML_FIT_PDF_NONPOSITIVE) return UML_OK;
  return count_bad_events(m, d, r->params, &r->n_bad_events, s, fn);
}

GenOut gen_out(const uml_data* d, unsigned int* d_bad) {
  GenOut o{};
  for (int kd = 0; kd < d->model->plan.ndim; ++kd) o.col[kd] = const_cast<void*>(d->job.col[kd]);
  o.n = d->n;
  o.bad = d_bad;
  return o;
}

// A dataset's device memory (events | work area | Hessian workspace, one
// allocation) and pinned staging block; the caller fills the events.
static int data_alloc(const uml_model* m, int64_t n, bool weighted, const DataLayout& L, uml_data** out,
                      const char* fn) {
  uml_data* d = new (std::nothrow) uml_data();
  if (!d) return set_error(UML_E_NOMEM, std::string(fn) + ": out of host memory");
  int hess_tiles = 0;
  const size_t o_work = align_up(L.bytes_events, 256), o_hess = o_work + align_up(L.bytes_work, 256);
  const size_t hbytes = m->d_hplan ? hess_work_bytes(m, n, &hess_tiles) : 0;
  hipError_t e = hipMalloc(&d->d_alloc, o_hess + hbytes);
  if (e != hipSuccess) {
    delete d;
    return set_error(e == hipErrorOutOfMemory ? UML_E_NOMEM : UML_E_HIP,
                     std::string(fn) + ": device buffer: " + hipGetErrorString(e));
  }
  d->h_stage = pinned_stage_get();
  if (!d->h_stage) {
    (void)hipFree(d->d_alloc);
    delete d;
    return set_error(UML_E_NOMEM, std::string(fn) + ": pinned staging");
  }
  char* base = static_cast<char*>(d->d_alloc);
  data_bind(d, m, n, weighted, L, base, base + o_work);
  if (hbytes) {
    d->d_hwork = base + o_hess;
    d->hess_tiles = hess_tiles;
  }
  d->owns_memory = 1;
  *out = d;
  return UML_OK;
}

// UML_DATA_BORROW: the dataset reads the caller's device columns in place;
// only the work area is allocated.  The values are checked on the device.
static int data_borrow(const uml_model* m, int64_t n, const void* const* cols, int32_t dtype, const void* w,
                       int32_t flags, hipStream_t s, uml_data** out) {
  const char* fn = "uml_data_create";
  const Plan& P = m->plan;
  if (!(flags & UML_DATA_DEVICE_SRC))
    return set_error(UML_E_INVALID, std::string(fn) + ": UML_DATA_BORROW needs UML_DATA_DEVICE_SRC");
  if (dtype != (P.precision == UML_MIXED ? UML_F32 : UML_F64))
    return set_error(UML_E_INVALID, std::string(fn) + ": a borrowed column must have the model's storage type");
  if (P.pre_fac >= 0)
    return set_error(UML_E_UNSUPPORTED, std::string(fn) + ": a model with precomputed terms cannot borrow columns");
  if (n < 0) return set_error(UML_E_INVALID, std::string(fn) + ": negative event count");
  if (n > 0 && !cols) return set_error(UML_E_INVALID, std::string(fn) + ": cols is NULL");
  for (int ud = 0; n > 0 && ud < P.ndim; ++ud)
    if (!cols[ud] || reinterpret_cast<uintptr_t>(cols[ud]) % 16)
      return set_error(UML_E_INVALID, std::string(fn) + ": a borrowed column must be 16-byte aligned");
  if (w && reinterpret_cast<uintptr_t>(w) % 16)
    return set_error(UML_E_INVALID, std::string(fn) + ": borrowed weights must be 16-byte aligned");
  DataLayout L = data_layout(P, n, w != nullptr);
  L.bytes_events = 0;  // no event storage of its own
  uml_data* d = nullptr;
  int rc = data_alloc(m, n, w != nullptr, L, &d, fn);
  if (rc != UML_OK) return rc;
  CheckArgs a{};
  for (int kd = 0; kd < P.ndim; ++kd) {
    d->job.col[kd] = cols[P.user_of_dim[kd]];
    a.col[kd] = cols[P.user_of_dim[kd]];
    a.lo[kd] = P.lo[kd];
    a.hi[kd] = P.hi[kd];
  }
  d->job.w = w;
  a.w = w;
  a.ndim = P.ndim;
  a.fp64 = P.precision == UML_FP64 ? 1 : 0;
  a.n = n;
  // the output slot doubles as the violation counter until the work area is
  // initialised
  a.bad = reinterpret_cast<unsigned int*>(d->d_out);
  unsigned int* h_bad = reinterpret_cast<unsigned int*>(d->h_stage);
  hipError_t e = hipMemsetAsync(a.bad, 0, sizeof(unsigned int), s);
  if (e == hipSuccess) {
    launch_check_events(a, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h_bad, a.bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = data_init_work(d, L, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    uml_data_destroy(d);
    return set_error(UML_E_HIP, std::string(fn) + ": " + hipGetErrorString(e));
  }
  if (*h_bad) {
    const unsigned bad = *h_bad;
    uml_data_destroy(d);
    return set_error(UML_E_EVENT_DOMAIN, std::string(fn) + ": " + std::to_string(bad) +
                                             " borrowed values outside their range or not finite");
  }
  *out = d;
  return UML_OK;
}

}  // namespace uml

using namespace uml;

extern "C" {

const char* uml_last_error(void) { return g_err.c_str(); }
const char* uml_version(void) { return UML_VERSION_STRING; }

int uml_model_create(const uml_model_desc* desc, uml_model** out) {
  if (!out) return set_error(UML_E_INVALID, "uml_model_create: out is NULL");
  *out = nullptr;
  uml_model* m = new (std::nothrow) uml_model();
  if (!m) return set_error(UML_E_NOMEM, "uml_model_create: out of host memory");
  std::string err;
  int rc = build_plan(desc, m->plan, err);
  if (rc != UML_OK) {
    delete m;
    return set_error(rc, "uml_model_create: " + err);
  }
  static std::atomic<long long> serial{0};
  m->plan.key = ++serial;  // never 0: a cleared constant block matches no model
  const std::string sig = plan_signature(m->plan);
  m->family = find_family(sig);
  if (!m->family) {
    delete m;
    return set_error(UML_E_UNSUPPORTED, "uml_model_create: no compiled kernel for model shape '" +
                                            sig + "' (compiled: " + family_list() + ")");
  }
  if (m->family->K != m->plan.K || m->family->ncst != m->plan.ncst) {
    delete m;
    return set_error(UML_E_INVALID, "uml_model_create: internal layout mismatch for " + sig);
  }
  m->theta0.resize(desc->n_params);
  for (int k = 0; k < desc->n_params; ++k) m->theta0[k] = desc->params[k].value;
  const bool have_hess = build_hess_plan(m->plan, m->hplan, m->hess_err);
  GenPlan& G = m->gplan;
  G = GenPlan{};
  G.nnode = desc->n_nodes;
  G.root = desc->root;
  G.ndim = desc->n_dims;
  G.npar = desc->n_params;
  for (int i = 0; i < desc->n_nodes; ++i) {
    const uml_node& s = desc->nodes[i];
    GenNode& g = G.node[i];
    g.kind = s.kind;
    for (int k = 0; k < 3; ++k) g.dim[k] = s.dims[k];
    g.npar = s.n_params;
    for (int k = 0; k < 8; ++k) g.par[k] = s.params[k];
    g.nchild = s.n_children;
    for (int k = 0; k < 4; ++k) g.child[k] = s.children[k];
  }
  G.root_step = gen_unfold(G, G.root, -1);
  if (G.root_step < 0) G.nstep = -1;
  for (int ud = 0; ud < desc->n_dims; ++ud) {
    G.lo[ud] = desc->dims[ud].lo;
    G.hi[ud] = desc->dims[ud].hi;
    G.col_of_user[ud] = m->plan.dim_of_user[ud];
  }
  hipError_t e = hipGetDevice(&m->device);
  if (e == hipSuccess) e = hipMalloc(&m->d_plan, sizeof(Plan));
  if (e == hipSuccess) e = hipMemcpy(m->d_plan, &m->plan, sizeof(Plan), hipMemcpyHostToDevice);
  if (e == hipSuccess && have_hess) e = hipMalloc(&m->d_hplan, sizeof(HessPlan));
  if (e == hipSuccess && have_hess)
    e = hipMemcpy(m->d_hplan, &m->hplan, sizeof(HessPlan), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&m->d_gplan, sizeof(GenPlan));
  if (e == hipSuccess) e = hipMemcpy(m->d_gplan, &m->gplan, sizeof(GenPlan), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (m->d_plan) (void)hipFree(m->d_plan);
    if (m->d_hplan) (void)hipFree(m->d_hplan);
    if (m->d_gplan) (void)hipFree(m->d_gplan);
    delete m;
    return set_error(UML_E_HIP, std::string("uml_model_create: ") + hipGetErrorString(e));
  }
  *out = m;
  return UML_OK;
}

void uml_model_destroy(uml_model* m) {
  if (!m) return;
  if (m->d_plan) (void)hipFree(m->d_plan);
  if (m->d_hplan) (void)hipFree(m->d_hplan);
  if (m->d_fitws) (void)hipFree(m->d_fitws);
  if (m->h_fitdone) (void)hipHostFree(m->h_fitdone);
  if (m->h_fitstage) (void)hipHostFree(m->h_fitstage);
  if (m->d_gplan) (void)hipFree(m->d_gplan);
  delete m;
}

int uml_model_n_free(const uml_model* m) { return m ? m->plan.nfree : UML_E_INVALID; }

int uml_model_describe(const uml_model* m, char* buf, int32_t len) {
  if (!m || !buf || len <= 0) return set_error(UML_E_INVALID, "uml_model_describe: bad argument");
  std::string s = plan_describe(m->plan);
  std::strncpy(buf, s.c_str(), size_t(len) - 1);
  buf[len - 1] = 0;
  return UML_OK;
}

int uml_data_create(const uml_model* m, int64_t n, const void* const* cols, int32_t dtype,
                    const void* w, int32_t flags, void* stream, uml_data** out) {
  if (!out) return set_error(UML_E_INVALID, "uml_data_create: out is NULL");
  *out = nullptr;
  if (!m) return set_error(UML_E_INVALID, "uml_data_create: model is NULL");
  const Plan& P = m->plan;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t ssz = dtype == UML_F32 ? 4 : 8;  // source element
  if (n > 0 && cols)
    for (int ud = 0; ud < P.ndim; ++ud)
      if (!cols[ud]) return set_error(UML_E_INVALID, "uml_data_create: column pointer is NULL");
  if (flags & UML_DATA_BORROW) return data_borrow(m, n, cols, dtype, w, flags, s, out);
  // device sources are copied back to the host first
  std::vector<char> hsrc;
  std::vector<const void*> src(P.ndim, nullptr);
  const void* wsrc = w;
  if (n > 0 && cols && (flags & UML_DATA_DEVICE_SRC) && (dtype == UML_F32 || dtype == UML_F64)) {
    hsrc.resize(size_t(n) * ssz * (P.ndim + (w ? 1 : 0)));
    for (int ud = 0; ud < P.ndim; ++ud) {
      UML_HIP_CHECK(hipMemcpy(hsrc.data() + size_t(ud) * n * ssz, cols[ud], n * ssz,
                              hipMemcpyDeviceToHost));
      src[ud] = hsrc.data() + size_t(ud) * n * ssz;
    }
    if (w) {
      UML_HIP_CHECK(hipMemcpy(hsrc.data() + size_t(P.ndim) * n * ssz, w, n * ssz,
                              hipMemcpyDeviceToHost));
      wsrc = hsrc.data() + size_t(P.ndim) * n * ssz;
    }
  } else if (n > 0 && cols) {
    for (int ud = 0; ud < P.ndim; ++ud) src[ud] = cols[ud];
  }
  std::vector<char> host;
  int rc = convert_events(P, n, n > 0 ? src.data() : nullptr, dtype, wsrc, host, "uml_data_create");
  if (rc != UML_OK) return rc;
  const DataLayout L = data_layout(P, n, w != nullptr);
  uml_data* d = nullptr;
  rc = data_alloc(m, n, w != nullptr, L, &d, "uml_data_create");
  if (rc != UML_OK) return rc;
  hipError_t e = data_upload(d, L, host, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    uml_data_destroy(d);
    return set_error(UML_E_HIP, std::string("uml_data_create: upload: ") + hipGetErrorString(e));
  }
  *out = d;
  return UML_OK;
}

int uml_data_generate(const uml_model* m, int64_t n, uint64_t seed, const double* theta_all,
                      void* stream, uml_data** out) {
  if (!out) return set_error(UML_E_INVALID, "uml_data_generate: out is NULL");
  *out = nullptr;
  if (!m) return set_error(UML_E_INVALID, "uml_data_generate: model is NULL");
  if (n < 0) return set_error(UML_E_INVALID, "uml_data_generate: negative event count");
  const Plan& P = m->plan;
  const double* th = theta_all ? theta_all : m->theta0.data();
  int rc = check_generation_theta(m, th, "uml_data_generate");
  if (rc != UML_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DataLayout L = data_layout(P, n, false);
  uml_data* d = nullptr;
  rc = data_alloc(m, n, false, L, &d, "uml_data_generate");
  if (rc != UML_OK) return rc;
  // the output slot doubles as the failure counter until the work area is
  // initialised
  unsigned int* d_bad = reinterpret_cast<unsigned int*>(d->d_out);
  unsigned int* h_bad = reinterpret_cast<unsigned int*>(d->h_stage + UML_MAX_PARAMS);
  std::memcpy(d->h_stage, th, sizeof(double) * P.npar);
  hipError_t e = hipMemcpyAsync(d->d_theta, d->h_stage, sizeof(double) * P.npar, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(d_bad, 0, sizeof(unsigned int), s);
  if (e == hipSuccess) {
    launch_generate(m->d_gplan, d->d_theta, seed, gen_out(d, d_bad), P.precision, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h_bad, d_bad, sizeof(unsigned int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = data_init_work(d, L, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    uml_data_destroy(d);
    return set_error(UML_E_HIP, std::string("uml_data_generate: ") + hipGetErrorString(e));
  }
  if (*h_bad) {
    const unsigned bad = *h_bad;
    uml_data_destroy(d);
    return set_error(UML_E_GENERATION, "uml_data_generate: " + std::to_string(bad) +
                                           " events needed more accept-reject attempts than the cap");
  }
  *out = d;
  return UML_OK;
}

int uml_data_download(const uml_data* d, void* const* cols, void* stream) {
  if (!d || (d->n > 0 && !cols)) return set_error(UML_E_INVALID, "uml_data_download: null argument");
  const Plan& P = d->model->plan;
  const size_t esz = P.precision == UML_MIXED ? 4 : 8;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int ud = 0; ud < P.ndim && d->n > 0; ++ud) {
    if (!cols[ud]) return set_error(UML_E_INVALID, "uml_data_download: column pointer is NULL");
    UML_HIP_CHECK(hipMemcpyAsync(cols[ud], d->job.col[P.dim_of_user[ud]], size_t(d->n) * esz,
                                 hipMemcpyDeviceToHost, s));
  }
  UML_HIP_CHECK(hipStreamSynchronize(s));
  return UML_OK;
}

void uml_data_destroy(uml_data* d) {
  if (!d) return;
  if (d->owns_memory) {
    if (d->d_alloc) (void)hipFree(d->d_alloc);
    if (d->h_stage) pinned_stage_put(d->h_stage);
  }
  delete d;
}

int64_t uml_data_n_events(const uml_data* d) { return d ? d->n : UML_E_INVALID; }

}  // extern "C"

namespace uml {

static int check_pair(const uml_model* m, const uml_data* d, const char* fn) {
  if (!m || !d) return set_error(UML_E_INVALID, std::string(fn) + ": null handle");
  if (d->model != m)
    return set_error(UML_E_INVALID, std::string(fn) + ": data was created for another model");
  return UML_OK;
}

// Queues the event kernel for one dataset (one launch per evaluation).
static int queue_eval(const uml_model* m, const uml_data* d, const double* d_theta, double* d_out,
                      hipStream_t s) {
  LaunchArgs a{};
  a.job0 = d->job;
  a.jobs = d->d_job;
  a.tmap = nullptr;
  a.grid = d->n_tiles;
  a.out = d_out;
  a.theta = d_theta;
  a.precision = m->plan.precision;
  a.stream = s;
  m->family->eval(a);
  UML_HIP_CHECK(hipGetLastError());
  return UML_OK;
}

static int eval_host(const uml_model* m, const uml_data* d, const double* theta, double* nll,
                     double* grad, void* stream, const char* fn) {
  int rc = check_pair(m, d, fn);
  if (rc) return rc;
  if (!theta || !nll) return set_error(UML_E_INVALID, std::string(fn) + ": null argument");
  const Plan& P = m->plan;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* hs = d->h_stage;
  std::memcpy(hs, theta, sizeof(double) * P.npar);
  UML_HIP_CHECK(hipMemcpyAsync(d->d_theta, hs, sizeof(double) * P.npar, hipMemcpyHostToDevice, s));
  rc = queue_eval(m, d, nullptr, nullptr, s);
  if (rc) return rc;
  double* ho = hs + UML_MAX_PARAMS;
  UML_HIP_CHECK(hipMemcpyAsync(ho, d->d_out, sizeof(double) * (1 + P.nfree), hipMemcpyDeviceToHost, s));
  UML_HIP_CHECK(hipStreamSynchronize(s));
  *nll = ho[0];
  if (grad) std::memcpy(grad, ho + 1, sizeof(double) * P.nfree);
  if (!std::isfinite(ho[0]))
    return set_error(UML_E_PDF_NONPOSITIVE,
                     std::string(fn) + ": P <= 0 or non-finite at some event, or parameters "
                     "outside the model's domain");
  return UML_OK;
}

}  // namespace uml

extern "C" {

int uml_eval_nll(const uml_model* m, const uml_data* d, const double* theta_all, double* nll,
                 void* stream) {
  return eval_host(m, d, theta_all, nll, nullptr, stream, "uml_eval_nll");
}

int uml_eval_nll_grad(const uml_model* m, const uml_data* d, const double* theta_all,
                      double* nll, double* grad_free, void* stream) {
  return eval_host(m, d, theta_all, nll, grad_free, stream, "uml_eval_nll_grad");
}

int uml_eval_bad_events(const uml_model* m, const uml_data* d, const double* theta_all, int64_t* n_bad,
                        void* stream) {
  int rc = check_pair(m, d, "uml_eval_bad_events");
  if (rc) return rc;
  if (!theta_all || !n_bad) return set_error(UML_E_INVALID, "uml_eval_bad_events: null argument");
  return count_bad_events(m, d, theta_all, n_bad, static_cast<hipStream_t>(stream), "uml_eval_bad_events");
}

int uml_eval_nll_grad_dev(const uml_model* m, const uml_data* d, const double* d_theta_all,
                          double* d_out, void* stream) {
  int rc = check_pair(m, d, "uml_eval_nll_grad_dev");
  if (rc) return rc;
  if (!d_theta_all || !d_out)
    return set_error(UML_E_INVALID, "uml_eval_nll_grad_dev: null device pointer");
  return queue_eval(m, d, d_theta_all, d_out, static_cast<hipStream_t>(stream));
}

}  // extern "C"
