/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of what the GPU
 * library computes: the normalised PDFs of the model catalogue, the unbinned
 * negative log-likelihood -sum_i w_i ln P(x_i | theta) (MoreFit paper, Eq. 1),
 * its analytic gradient and Hessian (Sec. 2.2), a quasi-Newton (BFGS) fit
 * with a Hessian-based covariance (Sec. 2.1), and the generation of
 * pseudo-experiments from a model (Sec. 2.5).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this.  It shares no code, header or constant with the GPU library.
 */
#ifndef ORACLE_H
#define ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXP 32   /* parameters per model */
#define ORC_MAXD 8    /* event dimensions     */
#define ORC_MAXN 64   /* nodes per model      */

enum {
  ORC_GAUSS = 1, /* Gaussian in dim[0]; par = {mu, sigma}              (Eq. 2) */
  ORC_EXP = 2,   /* exponential in dim[0]; par = {lambda}              (Eq. 2) */
  ORC_CHEB = 3,  /* 1 + sum_j c_j T_j(u) in dim[0]; par = {c_1..c_k}           */
  ORC_PWAVE = 4, /* P-wave density in dim = {ctl, ctk, phi};
                    par = {FL, S3, S4, S5, AFB, S7, S8, S9}             (Eq. 4) */
  ORC_PROD = 5,  /* product of children over disjoint dimensions               */
  ORC_SUM = 6    /* f*child[0] + (1-f)*child[1]; par = {f}; f outside [0,1]
                    is outside the model's domain (P treated as non-finite)   */
};

/* One node: 18 ints in this order (the layout the Python wrapper writes). */
typedef struct {
  int kind;
  int dim[3];
  int npar;
  int par[8];
  int nchild;
  int child[4];
} orc_node;

typedef struct {
  int ndim;
  double lo[ORC_MAXD], hi[ORC_MAXD];
  int nnode;
  orc_node node[ORC_MAXN];
  int root;
  int npar;
} orc_model;

/* Builds a model from flat arrays; returns 0 or a negative error. */
int orc_model_init(orc_model* m, int ndim, const double* lo, const double* hi,
                   int nnode, const int* nodes18, int root, int npar);

/* Normalised density at n points; x is SoA [ndim][n]. */
void orc_pdf(const orc_model* m, long n, const double* x, const double* theta,
             double* out);

/*
 * NLL over n events (SoA [ndim][n]); w may be NULL (all weights 1).
 * order 0: nll only; 1: + grad[npar]; 2: + hess[npar*npar] (row-major).
 * Gradient and Hessian cover all parameters (fixed ones included).
 * Every sum is Neumaier-compensated.  Returns the number of events with
 * P <= 0 or non-finite P; if that is non-zero, *nll = +inf.
 */
long orc_nll(const orc_model* m, long n, const double* x, const double* w,
             const double* theta, int order, double* nll, double* grad,
             double* hess);

/* Weighted score variance W2 = sum_i w_i^2 s_i s_i^T, s_i = d ln P / d theta
   (npar x npar, row-major); returns the count of events with P <= 0. */
long orc_w2(const orc_model* m, long n, const double* x, const double* w,
            const double* theta, double* w2);

/* Philox4x64-10 block of a counter and a key (the counter-based generator
   of Salmon et al., SC11). */
void orc_philox4x64(const unsigned long long ctr[4], const unsigned long long key[2],
                    unsigned long long out[4]);

/* Events i0 .. i0+n-1 of the pseudo-experiment `seed`, drawn from the model
   at theta into x (SoA [ndim][n]).  Event i uses the uniform stream of
   Philox counters (b, i, 0, 0), key (seed, 0), so any event can be drawn on
   its own.  Returns the number of events whose sampling hit the attempt cap
   (their values are the lower range edges). */
long orc_generate(const orc_model* m, long i0, long n, unsigned long long seed,
                  const double* theta, double* x);

typedef struct {
  double edm_tol;  /* stop when 0.5 g^T V g < edm_tol                   */
  int max_iter;    /* BFGS iterations                                   */
  int polish;      /* number of Newton steps after BFGS (0 = none)      */
} orc_fit_opts;

typedef struct {
  double nll, edm;
  int n_iter, n_eval, status; /* status 0 = converged, 1 = max_iter,
                                 2 = line search failed, 3 = Hessian not PD */
} orc_fit_info;

/*
 * BFGS fit over the free parameters (free_mask[k] != 0).  theta holds the
 * start on entry (all parameters) and the fitted values on exit.  cov is
 * nfree*nfree (inverse Hessian of the NLL at the minimum, free order).
 */
int orc_fit(const orc_model* m, long n, const double* x, const double* w,
            double* theta, const int* free_mask, const orc_fit_opts* opts,
            double* cov, orc_fit_info* info);

#ifdef __cplusplus
}
#endif
#endif
