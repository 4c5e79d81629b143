// Host-runtime internals of libuml (opaque handle layouts, helpers).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "gen.h"
#include "hess.h"
#include "kernels.h"
#include "uml_internal.h"

struct uml_model {
  uml::Plan plan;
  std::vector<double> theta0;      // parameter values of the description
  uml::Plan* d_plan = nullptr;     // device copy
  const uml::Family* family = nullptr;
  int device = 0;
  uml::HessPlan hplan;
  uml::HessPlan* d_hplan = nullptr;  // device copy (nullptr: no Hessian, see hess_err)
  std::string hess_err;
  // device workspace of uml_fit / uml_fit_batch (fit states, jobs, tile map),
  // grown on demand and kept until the model is destroyed
  mutable void* d_fitws = nullptr;
  mutable size_t fitws_bytes = 0;
  // the fits' done flags, written by a kernel into mapped pinned memory
  // (host address and device address), grown on demand
  mutable int* h_fitdone = nullptr;
  mutable int* h_fitdone_dev = nullptr;
  mutable int fitdone_n = 0;
  // pinned staging in the layout of the fit workspace, grown with it
  mutable char* h_fitstage = nullptr;
  uml::GenPlan gplan;                // the model tree for generation
  uml::GenPlan* d_gplan = nullptr;   // device copy
};

struct uml_data {
  const uml_model* model = nullptr;
  int64_t n = 0;
  int weighted = 0;
  int E = 0;                        // events per thread per tile
  int n_tiles = 0;
  void* d_events = nullptr;         // columns (+ weights), one allocation
  void* d_work = nullptr;           // job, constants, partials, counter, outputs
  uml::Job job{};                   // host copy of the device job
  uml::Job* d_job = nullptr;
  double* d_theta = nullptr;        // staging for host theta
  double* d_out = nullptr;          // [1 + nfree]
  unsigned long long* d_bad = nullptr;  // count of events with P <= 0 (count pass)
  void* d_hwork = nullptr;          // Hessian workspace (allocated on first use)
  int hess_tiles = 0;
  double* h_stage = nullptr;        // pinned host staging (a block of the process pool)
  void* d_alloc = nullptr;          // the device allocation this dataset owns
  int64_t bytes_events = 0;
  int64_t bytes_work = 0;
  int owns_memory = 0;              // 0: memory belongs to a server's arena
};

namespace uml {

int build_plan(const uml_model_desc* d, Plan& P, std::string& err);
std::string plan_signature(const Plan& P);
std::string plan_describe(const Plan& P);

// thread-local error message
int set_error(int code, const std::string& msg);

// The precomputed event-only terms of a model that stores them (no-op otherwise).
hipError_t data_precompute(uml_data* d, hipStream_t s);

// Event storage and work-area layout of a dataset.
struct DataLayout {
  int E, n_tiles;
  int64_t stride;
  size_t bytes_events, bytes_work;
  size_t o_job, o_cst, o_theta, o_out, o_cnt, o_bad, o_epoch, o_part, o_spart;
};
int convert_events(const Plan& P, int64_t n, const void* const* cols, int32_t dtype, const void* w,
                   std::vector<char>& host, const char* fn);
DataLayout data_layout(const Plan& P, int64_t n, bool weighted);
void data_bind(uml_data* d, const uml_model* m, int64_t n, bool weighted, const DataLayout& L,
               void* d_events, void* d_work);
hipError_t data_upload(uml_data* d, const DataLayout& L, const std::vector<char>& host, hipStream_t s);
hipError_t data_init_work(uml_data* d, const DataLayout& L, hipStream_t s);
int check_generation_theta(const uml_model* m, const double* theta, const char* fn);
// Events with P <= 0 or not finite at theta (host, all parameters); synchronous.
int count_bad_events(const uml_model* m, const uml_data* d, const double* theta, int64_t* n_bad,
                     hipStream_t s, const char* fn);
// Sets r->n_bad_events for a result whose status is UML_FIT_PDF_NONPOSITIVE (the
// count at r->params), 0 otherwise.
int fill_bad_count(const uml_model* m, const uml_data* d, uml_fit_result* r, hipStream_t s,
                   const char* fn);
GenOut gen_out(const uml_data* d, unsigned int* d_bad);
size_t hess_work_bytes(const uml_model* m, int64_t n, int* n_tiles);
double* pinned_stage_get();
void pinned_stage_put(double* p);

int hess_sums(const uml_model* m);
int hessian_queue(const uml_model* m, uml_data* d, const double* d_theta, double* h_out,
                  hipStream_t s, const char* fn);
int hessian_queue_batch(const uml_model* m, uml_data* const* ds, const double* const* d_thetas, int n,
                        double* d_outs, HessJob* h_jobs, HessJob* d_jobs, int2* h_map, int2* d_map,
                        int map_cap, hipStream_t s, const char* fn);
int hessian_host(const uml_model* m, uml_data* d, const double* theta, hipStream_t s,
                 std::vector<double>& out, const char* fn);
int unpack_hessian(const uml_model* m, const double* h, double* nll, double* grad, double* hess,
                   double* w2, const char* fn);
bool chol_inverse(int n, const double* A, double* Ai);
int metric_from_sums(const uml_model* m, const double* h, double* V0, double* nll0, const char* fn);
void finish_from_sums(const uml_model* m, const double* h, const double* theta,
                      const uml_fit_options& o, uml_fit_result* r, const char* fn);
int finish_fit(const uml_model* m, uml_data* d, std::vector<double>& theta,
               const uml_fit_options& o, uml_fit_result* r, hipStream_t s, const char* fn);
int init_fit_state(const uml_model* m, uml_data* d, const double* start, const uml_fit_options& o,
                   FitState& F, hipStream_t s, const char* fn);
void fit_state_begin(const uml_model* m, const double* start, const uml_fit_options& o, FitState& F);
int fit_state_metric(const uml_model* m, const double* h, FitState& F, const char* fn);
int check_fit_options(const uml_fit_options& o, const char* fn);
int fit_batch_impl(const uml_model* m, const uml_data* const* ds, int n, const double* starts,
                   const uml_fit_options* opts, uml_fit_result* out, const char* fn);

#define UML_HIP_CHECK(expr)                                                         \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::uml::set_error(UML_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace uml
