/*
 * uml.h -- C ABI of the MI355X unbinned maximum-likelihood library.
 *
 * The library evaluates, on one GPU, the negative log-likelihood of an
 * unbinned fit (MoreFit paper, Eq. 1)
 *
 *     NLL(theta) = - sum_i w_i ln P(x_i | theta)
 *
 * together with its analytic gradient (Sec. 2.1-2.2) and Hessian, runs a
 * quasi-Newton minimisation on the device (the BFGS variant of the
 * variable-metric method, Sec. 2.1) with the inverse Hessian at the minimum
 * as covariance (the HESSE step of the benchmark protocol, Sec. 3.1), and
 * serves many independent pseudo-experiment fits (the coverage-study
 * workload, Sec. 1) with continuous batching.
 *
 * Conventions for every call:
 *   - Return 0 (UML_OK) on success or a negative UML_E_* code; the library
 *     never aborts.  uml_last_error() gives a message for the calling thread.
 *   - Parameter order is the order of uml_model_desc.params.  "theta_all"
 *     arrays hold every parameter (fixed ones included); gradients, Hessians
 *     and covariances cover the free parameters only, in parameter order.
 *   - Pointers named d_* are device pointers; all others are host pointers.
 *     The caller owns every buffer it passes; the library copies what it
 *     keeps.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls on a model or data handle are not thread-safe: use one handle
 *     per thread and stream.  The server is thread-safe (see below).
 *   - A non-positive or non-finite P at any event makes the NLL +inf, the
 *     gradient zero and the call return UML_E_PDF_NONPOSITIVE.
 */
#ifndef UML_H
#define UML_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UML_VERSION_STRING "0.1.0"

/* ---- error codes ------------------------------------------------------- */
#define UML_OK 0
#define UML_E_INVALID -1         /* bad argument or model description         */
#define UML_E_UNSUPPORTED -2     /* model shape with no compiled kernel       */
#define UML_E_EVENT_DOMAIN -3    /* event outside its range, NaN, or bad weight */
#define UML_E_PDF_NONPOSITIVE -4 /* P <= 0 or non-finite: NLL = +inf          */
#define UML_E_HIP -5             /* HIP runtime failure                       */
#define UML_E_NOMEM -6           /* device or host allocation failed          */
#define UML_E_NOT_PD -7          /* Hessian not positive definite             */
#define UML_E_BUDGET -8          /* server: request exceeds the memory budget */
#define UML_E_QUEUE_FULL -9      /* server: too many pending requests         */
#define UML_E_TIMEOUT -10        /* server: nothing finished within timeout   */
#define UML_E_GENERATION -11     /* generation: an accept-reject draw hit its cap */

/* ---- limits ------------------------------------------------------------ */
#define UML_MAX_DIMS 8
#define UML_MAX_PARAMS 32
#define UML_MAX_NODES 32

/* ---- model description --------------------------------------------------
 * A model is a tree over the PDF catalogue.  Leaves are normalised on their
 * dimensions' [lo, hi]:
 *   UML_GAUSS  dims[0]; params {mu, sigma}: Gaussian (Eq. 2)
 *   UML_EXP    dims[0]; params {lambda}: e^{lambda x} (Eq. 2), lambda = 0 allowed
 *   UML_CHEB   dims[0]; params {c_1..c_k}, 1 <= k <= 4: 1 + sum_j c_j T_j(u),
 *              u = (2x - lo - hi)/(hi - lo), T_j Chebyshev polynomials of the
 *              first kind
 *   UML_PWAVE  dims {cos theta_l, cos theta_K, phi} with ranges exactly
 *              [-1,1], [-1,1], [-pi,pi]; params {FL, S3, S4, S5, AFB, S7, S8, S9}:
 *              the P-wave angular decay rate (Eq. 4), unit norm
 *   UML_PROD   children (2..4) over pairwise disjoint dimensions: their product
 *   UML_SUM    children {A, B}; params {f}: f*A + (1-f)*B
 * Every term of the expanded mixture must cover all dimensions.
 */
enum { UML_GAUSS = 1, UML_EXP = 2, UML_CHEB = 3, UML_PWAVE = 4, UML_PROD = 5, UML_SUM = 6 };

/* Arithmetic of the event kernels. */
enum {
  UML_FP64 = 0,  /* FP64 throughout                                           */
  UML_MIXED = 1  /* FP32 per-event PDF/log arithmetic, FP64 accumulation,
                    FP64 normalisations, reductions and minimiser             */
};

/* Storage type of event columns and weights passed to uml_data_create. */
enum { UML_F32 = 0, UML_F64 = 1 };

typedef struct {
  double lo, hi;
} uml_dim;

typedef struct {
  double value;  /* start / default value */
  double lo, hi; /* informational; no transform is applied */
  int32_t fixed; /* non-zero: not a free parameter */
} uml_param;

typedef struct {
  int32_t kind;        /* UML_GAUSS .. UML_SUM                 */
  int32_t dims[3];     /* leaf dimensions (indices into dims)  */
  int32_t n_params;    /* number of entries used in params    */
  int32_t params[8];   /* parameter indices                   */
  int32_t n_children;  /* PROD: 2..4, SUM: 2                  */
  int32_t children[4]; /* node indices                        */
} uml_node;

typedef struct {
  int32_t n_dims;
  const uml_dim* dims;
  int32_t n_params;
  const uml_param* params;
  int32_t n_nodes;
  const uml_node* nodes;
  int32_t root;
  int32_t precision; /* UML_FP64 or UML_MIXED */
  int32_t flags;     /* UML_MODEL_PRECOMPUTE_ANGULAR or 0 */
} uml_model_desc;

/* The event-only terms of the P-wave density (the eight angular functions of
 * Eq. 4 and the F_L-free term) are computed once per dataset and stored as
 * nine extra columns, which the event kernel reads instead of recomputing
 * them (the paper's optimisation of event-dependent terms, Sec. 2.4.2).  For
 * models with one P-wave factor. */
#define UML_MODEL_PRECOMPUTE_ANGULAR 1

typedef struct uml_model uml_model;
typedef struct uml_data uml_data;
typedef struct uml_server uml_server;

/* Validates and compiles a description (copied).  The model is expanded into
 * a mixture of products of catalogue factors and bound to the matching
 * compiled kernel family; a shape without one gives UML_E_UNSUPPORTED. */
int uml_model_create(const uml_model_desc* desc, uml_model** out);
void uml_model_destroy(uml_model* m);
int uml_model_n_free(const uml_model* m);
/* Writes a short text describing the expanded mixture and kernel family. */
int uml_model_describe(const uml_model* m, char* buf, int32_t len);

/* ---- event data ---------------------------------------------------------
 * The events x_i of Eq. 1.  A minimisation evaluates the same sample at many
 * parameter points and host-to-accelerator transfers are an overhead to keep
 * small (Sec. 2.1), so the events are moved to the device once, here, and
 * every later evaluation moves only the parameters and its results.
 * n events as a structure of arrays: cols[d] points to n values of dimension
 * d (model order) in storage type dtype.  w (same dtype) is NULL or one
 * weight per event (the weighted NLL -sum w_i ln P_i).  Events are copied
 * into device buffers in the model's arithmetic (FP32 for UML_MIXED, FP64
 * for UML_FP64).  Every value must lie in its dimension's [lo, hi] after that
 * conversion and every weight must be finite, else UML_E_EVENT_DOMAIN.
 * flags: UML_DATA_DEVICE_SRC -- cols and w are device pointers.
 *        UML_DATA_BORROW (with UML_DATA_DEVICE_SRC) -- no copy: the dataset
 *        reads the caller's device columns (and weights) in place.  dtype must
 *        be the model's storage type (UML_F32 for UML_MIXED, UML_F64 for
 *        UML_FP64), every pointer 16-byte aligned, and the model must not store
 *        precomputed terms (UML_E_INVALID / UML_E_UNSUPPORTED otherwise).  The
 *        values are checked on the device as above.  The caller keeps the
 *        buffers alive and unchanged until uml_data_destroy.
 * The copy (or check) runs on stream and is complete when the call returns. */
#define UML_DATA_DEVICE_SRC 1
#define UML_DATA_BORROW 2
int uml_data_create(const uml_model* m, int64_t n, const void* const* cols, int32_t dtype,
                    const void* w, int32_t flags, void* stream, uml_data** out);
void uml_data_destroy(uml_data* d);
int64_t uml_data_n_events(const uml_data* d);

/* A pseudo-experiment drawn on the device (the toy studies of Sec. 2.5): n
 * events of the model at theta_all (NULL: the description's values), event i
 * drawn from its own counter-based stream (Philox4x64-10 at counters
 * (b, i, 0, 0), key (seed, 0)), so the events depend only on (seed, i).  Sums
 * pick a child by their fraction, products draw every child, Gaussians by
 * Box-Muller with rejection outside the range, exponentials by their inverse
 * distribution function, Chebyshev series and the P-wave density by
 * accept-reject.  Values are stored in the model's arithmetic (FP32 for
 * UML_MIXED: the nearest FP32 value inside the range).  Returns
 * UML_E_INVALID for a fraction outside [0, 1] or a width <= 0, and
 * UML_E_GENERATION if an accept-reject draw needed more than 65536 attempts.
 * Complete when the call returns. */
int uml_data_generate(const uml_model* m, int64_t n, uint64_t seed, const double* theta_all,
                      void* stream, uml_data** out);
/* Copies the stored event columns to host columns cols[d] (model order) of
 * the storage type (FP32 for UML_MIXED models, FP64 otherwise). */
int uml_data_download(const uml_data* d, void* const* cols, void* stream);

/* ---- evaluation (Eq. 1 and its derivatives) -----------------------------
 * Synchronous: return when the results are in the host buffers. */
int uml_eval_nll(const uml_model* m, const uml_data* d, const double* theta_all, double* nll,
                 void* stream);
int uml_eval_nll_grad(const uml_model* m, const uml_data* d, const double* theta_all,
                      double* nll, double* grad_free, void* stream);

/* Stream-ordered and asynchronous: reads d_theta_all (n_params doubles) and
 * writes d_out = [nll, grad_free...] (1 + n_free doubles) on stream.  Both
 * buffers stay owned by the caller and must outlive the queued work.  A
 * non-positive P shows as d_out[0] = +inf.  No host synchronisation; safe to
 * capture in a HIP graph. */
int uml_eval_nll_grad_dev(const uml_model* m, const uml_data* d, const double* d_theta_all,
                          double* d_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * evaluation of uml_eval_nll_grad_dev over the caller's own device columns,
 * with no dataset handle, that allocates nothing.  The event kernel's scratch
 * memory (its constant cache and tile partials) is a
 * fixed array of UML_NOALLOC_SCRATCH_BYTES in the library's device code, one
 * per GPU, held until the process ends.
 *   d_cols   n_dims device pointers (model dimension order), each a column of
 *            n events in the model's storage type (FP32 for UML_MIXED, FP64
 *            otherwise), 16-byte aligned; read in place, not copied and not
 *            range-checked: the caller guarantees every value lies in its
 *            dimension's range (as uml_data_create would have checked).
 *   d_w      device weights (same type and alignment) or NULL.
 *   d_theta_all, d_out  as in uml_eval_nll_grad_dev.
 * Stream-ordered and asynchronous; results are bitwise equal to
 * uml_eval_nll_grad_dev on a dataset holding the same events.  The limit:
 * 2 * K * tiles * 8 bytes of tile partials, with K the model's moment count
 * and tiles about n / 4096 (n / 8192 above 2^23 events), must fit in the
 * array (about 2e8 events for the 4-D model); larger n, a model with
 * precomputed terms, or a null or misaligned pointer give UML_E_INVALID /
 * UML_E_UNSUPPORTED before anything is queued.  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (different streams or
 * threads) race and must be serialised by the caller. */
#define UML_NOALLOC_SCRATCH_BYTES (8u << 20)
int uml_eval_nll_grad_noalloc(const uml_model* m, int64_t n, const void* const* d_cols,
                              const void* d_w, const double* d_theta_all, double* d_out,
                              void* stream);

/* The number of events at which P(x_i | theta) <= 0 or is not finite: the
 * events outside the domain of Eq. 1's logarithm, which make the NLL +inf.
 * Every event counts when theta is outside the model's domain (a fraction
 * outside [0, 1], a Gaussian width <= 0).  The decision is taken in the
 * model's arithmetic (FP32 per event for UML_MIXED), with the same per-event
 * arithmetic as the evaluation, so a count > 0 is exactly when an evaluation
 * at theta_all gives +inf.  A separate pass over the events, not part of the
 * evaluation: call it after an evaluation returned UML_E_PDF_NONPOSITIVE.
 * theta_all: host, all parameters.  *n_bad receives the count.  Synchronous. */
int uml_eval_bad_events(const uml_model* m, const uml_data* d, const double* theta_all, int64_t* n_bad,
                        void* stream);

/* NLL, gradient and Hessian (n_free x n_free, row-major) in one pass over the
 * events.  w2_free, if not NULL, receives sum_i w_i^2 s_i s_i^T with s_i the
 * per-event score d ln P_i / d theta (the middle of the sandwich covariance
 * of weighted fits).  Synchronous. */
int uml_eval_hessian(const uml_model* m, const uml_data* d, const double* theta_all,
                     double* nll, double* grad_free, double* hess_free, double* w2_free,
                     void* stream);

/* ---- fitting ------------------------------------------------------------ */
typedef struct {
  double edm_tol;    /* stop when EDM = 0.5 g^T V g < edm_tol (default 1e-6) */
  int32_t max_iter;  /* BFGS iterations (default 1000)                        */
  int32_t polish;    /* Newton steps with the analytic Hessian after BFGS      */
  int32_t want_cov;  /* return the covariance matrix in uml_fit_result.cov    */
  int32_t cov_kind;  /* UML_COV_HESSE: H^-1; UML_COV_SANDWICH: H^-1 W2 H^-1,
                        W2 = sum w_i^2 s_i s_i^T (the covariance of weighted
                        fits, Sec. 2.2); errors follow the chosen matrix      */
  int32_t method;    /* UML_METHOD_BFGS: quasi-Newton steps on the device, one
                        event pass per step; UML_METHOD_NEWTON: Newton steps
                        with the analytic Hessian (one Hessian pass per
                        iteration, host-driven; few iterations, Sec. 3.2)   */
} uml_fit_options;

enum { UML_COV_HESSE = 0, UML_COV_SANDWICH = 1 };
enum { UML_METHOD_BFGS = 0, UML_METHOD_NEWTON = 1 };

/* Fit status */
enum {
  UML_FIT_CONVERGED = 0,
  UML_FIT_MAX_ITER = 1,
  UML_FIT_LINESEARCH_FAIL = 2,
  UML_FIT_HESSIAN_NOT_PD = 3,
  UML_FIT_PDF_NONPOSITIVE = 4,
  UML_FIT_CANCELLED = 5,
  UML_FIT_GENERATION_FAILED = 6 /* server: the request's events could not be drawn */
};

typedef struct {
  double params[UML_MAX_PARAMS];                 /* all parameters, fitted       */
  double errors[UML_MAX_PARAMS];                 /* sqrt(diag cov); 0 for fixed  */
  double cov[UML_MAX_PARAMS * UML_MAX_PARAMS];   /* n_free x n_free, row-major   */
  double nll, edm;
  int32_t n_free, n_iter, n_eval, status;
  uint64_t ticket;                               /* server requests              */
  double latency_s;                              /* server: submit -> finished   */
  int64_t n_bad_events;                          /* status UML_FIT_PDF_NONPOSITIVE:
                                                    events with P <= 0 or not finite
                                                    at params (uml_eval_bad_events);
                                                    0 otherwise                   */
} uml_fit_result;

void uml_fit_options_default(uml_fit_options* o);

/* One fit, minimiser state resident on the device (one kernel launch per
 * function evaluation; the host only polls a convergence flag). */
int uml_fit(const uml_model* m, const uml_data* d, const double* start_all,
            const uml_fit_options* opts, uml_fit_result* out);

/* n_fits independent fits of the same model, advanced together: every launch
 * evaluates one trial point for every unfinished fit.  starts is
 * n_fits x n_params (row-major).  Each result equals, bit for bit, the result
 * of uml_fit on that dataset alone. */
int uml_fit_batch(const uml_model* m, const uml_data* const* ds, int32_t n_fits,
                  const double* starts, const uml_fit_options* opts, uml_fit_result* out);

/* ---- serving --------------------------------------------------------------
 * A device-resident loop over many pseudo-experiment fits of one model.
 * Requests are admitted while free slots and device memory allow, packed into
 * one ragged launch per iteration (captured as a HIP graph), retired when
 * converged; results are polled.  submit, poll and stats may be called from
 * any thread. */
typedef struct {
  int32_t max_slots;       /* fits resident at once (default 256)             */
  int64_t hbm_budget;      /* bytes of event storage resident at once (<=0: 4 GiB) */
  int32_t max_pending;     /* queued requests before UML_E_QUEUE_FULL (<=0: 1<<20) */
  uml_fit_options fit;     /* per-fit options                                 */
} uml_server_options;

typedef struct {
  int64_t n_events;
  const void* const* cols; /* host SoA columns, model order, storage dtype  */
  int32_t dtype;           /* UML_F32 or UML_F64                             */
  const void* w;           /* host weights or NULL                           */
  const double* start;     /* n_params start values, or NULL for the model's */
  int32_t generate;        /* non-zero: ignore cols/dtype/w and draw the
                              n_events events on the device, as
                              uml_data_generate does with this seed           */
  uint64_t seed;
  const double* gen_theta; /* parameters to draw at (NULL: the model's)      */
} uml_request;

typedef struct {
  int64_t submitted, admitted, finished, pending, active;
  int64_t iterations;      /* launches of the batched iteration              */
  int64_t resident_bytes;  /* device bytes held by admitted requests          */
  int64_t peak_resident_bytes;
  int64_t budget_waits;    /* admission passes that stopped for lack of memory */
  double t_admit_s;        /* worker time admitting requests (upload, start metric) */
  double t_iterate_s;      /* worker time in batched iterations (graph replays)   */
  double t_retire_s;       /* worker time retiring fits (final Hessian, results)  */
} uml_server_stats;

void uml_server_options_default(uml_server_options* o);
int uml_server_create(const uml_model* m, const uml_server_options* opts, uml_server** out);
/* Copies the request (events included) and returns its ticket. */
int uml_server_submit(uml_server* s, const uml_request* req, uint64_t* ticket);
/* Moves up to max finished results into out; waits up to timeout_us (0: no
 * wait, <0: until at least one result or nothing left in flight). */
int uml_server_poll(uml_server* s, uml_fit_result* out, int32_t max, int32_t* n_out,
                    int32_t timeout_us);
int uml_server_stats_get(uml_server* s, uml_server_stats* st);
/* Blocks until every submitted request has finished (results stay pollable). */
int uml_server_drain(uml_server* s);
void uml_server_destroy(uml_server* s);

/* ---- misc --------------------------------------------------------------- */
const char* uml_last_error(void);
const char* uml_version(void);

#ifdef __cplusplus
}
#endif
#endif
