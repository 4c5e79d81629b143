// Internal layout shared by the host runtime and the kernels of libuml.
//
// A model tree is expanded into a mixture of products
//     P(x) = sum_c F_c prod_{f in c} p_f(x_{dims(f)}),
// with F_c the product of the SUM fractions (f or 1 - f) on the path to
// component c.  Each factor is a catalogue leaf (Gaussian, exponential,
// Chebyshev series, P-wave density).  The event kernels work in base-2 log
// space per component:
//     S_c = 2^{E_c} V_c,   E_c = log2 K_c + sum_{exp-type f} e_f(x),
//     V_c = prod_{polynomial-type f} v_f(x),
// where K_c collects every parameter-only factor (fractions, the Gaussian and
// exponential normalisations).  Those parameter-only terms are computed once
// per parameter point by the prologue (the paper's hoisting of
// parameter-dependent terms, Sec. 2.4.1 and Eq. 3).
//
// Per event the kernels accumulate, weighted by w:
//     slot 0:            log2 P
//     per component c:   r_c = S_c / P                     (responsibility)
//     Gaussian f in c:   r_c d, r_c d^2 with d = x - mu
//     exponential f:     r_c x'   (x' = x - xref, a per-dimension shift)
//     Chebyshev f:       q_{c,f} T_j(u), j = 1..k
//     P-wave f:          q_{c,f} b_k, the 8 angular terms
// where q_{c,f} = r_c / v_f.  The epilogue turns these sums into the NLL and
// its gradient in FP64 (chain rule through the mixture).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uml.h"

namespace uml {

constexpr int kBlock = 256;           // threads per workgroup
constexpr int kMaxComp = 4;           // mixture components
constexpr int kMaxFacPerComp = 4;     // factors per component
constexpr int kMaxFac = 16;           // factors in the whole mixture
constexpr int kMaxK = 64;             // accumulators per event
constexpr int kMaxCst = 128;          // kernel constants
constexpr int kMaxECst = 128;         // epilogue constants
constexpr int kMaxCheb = 4;
constexpr int kMaxCols = 16;          // stored event columns (dimensions + precomputed terms)
constexpr int kPWaveTerms = 9;        // precomputed P-wave columns: u0 and the 8 angular terms

enum FactorKind { FK_GAUSS = 1, FK_EXP = 2, FK_CHEB = 3, FK_PWAVE = 4 };

// Kernel constants, moments and epilogue constants per factor kind; the
// compile-time shapes and the host plan builder both use these.
//   Gaussian     kernel {c0_hi, c1_hi, c1_lo, k2}, epilogue 5
//   exponential  kernel {c_hi, c_lo}, epilogue 2
//   Chebyshev    kernel {s_hi, s_lo, t, sgn, sgn c_1 .. sgn c_N}, epilogue 2N
//   P-wave       kernel the 8 angular coefficients (hi), then their lo parts, epilogue 8
// The "_lo" entries carry the part of an FP64 constant that its FP32 value
// drops (zero in the FP64 set); see compute_constants.
__host__ __device__ constexpr int fk_ncst(int kind, int order) {
  return kind == FK_GAUSS ? 4 : kind == FK_EXP ? 2 : kind == FK_CHEB ? order + 4 : 16;
}
__host__ __device__ constexpr int fk_nmom(int kind, int order) {
  return kind == FK_GAUSS ? 2 : kind == FK_EXP ? 1 : kind == FK_CHEB ? order : 8;
}
__host__ __device__ constexpr int fk_necst(int kind, int order) {
  return kind == FK_GAUSS ? 5 : kind == FK_EXP ? 2 : kind == FK_CHEB ? 2 * order : 8;
}
// Kernel constants of a component ahead of its factors' own: log2 K_c as an
// FP32 pair (hi, lo).
constexpr int kCompCst = 2;
__host__ __device__ constexpr bool fk_expo(int kind) {
  return kind == FK_GAUSS || kind == FK_EXP;
}

struct FactorPlan {
  int kind, order;   // order: Chebyshev order (0 otherwise)
  int dim[3];        // kernel dimensions (canonical order)
  int par[8];        // parameter indices
  int cst;           // offset of its kernel constants
  int ecst;          // offset of its epilogue constants
  int mom;           // first moment slot
  double lo[3], hi[3];
  double xref;       // shift of dim[0] (0 if the dimension is not shifted)
  int pre;           // P-wave: first precomputed column, or -1
};

struct CompPlan {
  int nfac;
  int fac[kMaxFacPerComp];  // factor indices, in kernel order
  int nfrac;
  int frac_par[8];          // SUM fraction parameters on the path
  int frac_sign[8];         // +1: f, -1: 1 - f
  int frac_ec[8];           // epilogue constant d ln F_c / d f of each entry
  int cst_lk2;              // offset of log2 K_c (hi), followed by its lo part
  int slot_r;               // moment slot of r_c
};

// One term of the gradient: d NLL / d theta_p = -sum_t e[ec_t] * M[mom_t]
// over the terms of parameter p (e: epilogue constants of the point,
// M: the moment sums).
struct EpiTerm {
  short mom, ec;
};
constexpr int kMaxTerms = 128;

struct Plan {
  long long key;  // identifies the model (see ConstBlock::key)
  int ncomp;
  CompPlan comp[kMaxComp];
  int nfac;
  FactorPlan fac[kMaxFac];
  int K;       // accumulators (slot 0 = log2 P)
  int ncst;    // kernel constants
  int necst;   // epilogue constants
  int ndim;    // kernel dimensions
  int ncol;    // stored columns: the dimensions, then any precomputed terms
  int pre_fac; // the factor whose terms are precomputed, or -1
  int npar, nfree;
  int free_idx[UML_MAX_PARAMS];  // free position -> parameter
  int free_pos[UML_MAX_PARAMS];  // parameter -> free position or -1
  int dim_of_user[UML_MAX_DIMS]; // user dimension -> kernel dimension
  int user_of_dim[UML_MAX_DIMS]; // kernel dimension -> user dimension
  double lo[UML_MAX_DIMS], hi[UML_MAX_DIMS];  // per kernel dimension
  double xref[UML_MAX_DIMS];     // per kernel dimension (0: not shifted)
  int precision;
  int nterm;
  EpiTerm term[kMaxTerms];              // grouped by parameter
  int term_begin[UML_MAX_PARAMS + 1];   // terms of parameter p: [begin[p], begin[p+1])
  int pad_[1];
};
static_assert(sizeof(Plan) % 16 == 0, "Plan is copied in 16-byte units");

// Parameter-dependent constants for one evaluation (written by the prologue).
struct ConstBlock {
  double d[kMaxCst];    // kernel constants, FP64
  float f[kMaxCst];     // the same, rounded to FP32 (mixed arithmetic)
  double e[kMaxECst];   // epilogue constants
  double theta[UML_MAX_PARAMS];
  double xd[UML_MAX_DIMS];  // per-dimension shifts (FP64)
  float xf[UML_MAX_DIMS];   // the same in FP32 (exact: FP32 values)
  int domain_ok;        // 0 if theta is outside the model's domain
  int valid;            // 1 once written: (key, theta[]) identify this block
  long long key;        // the model whose plan wrote it (Plan::key)
};
static_assert(sizeof(ConstBlock) % 16 == 0, "ConstBlock is copied in 16-byte units");

// Device-resident state of one BFGS fit (one per job in fit mode).  Every
// launch evaluates the NLL and gradient at theta; the workgroup that
// completes the evaluation takes the BFGS step and writes the next theta.
struct FitState {
  double theta[UML_MAX_PARAMS];       // point evaluated by the next launch (all parameters)
  double out[1 + UML_MAX_PARAMS];     // NLL and free gradient at theta (epilogue output)
  double x[UML_MAX_PARAMS];           // accepted point (free parameters)
  double g[UML_MAX_PARAMS];           // gradient at x
  double p[UML_MAX_PARAMS];           // search direction
  double V[UML_MAX_PARAMS * UML_MAX_PARAMS];   // inverse-Hessian estimate
  double V0[UML_MAX_PARAMS * UML_MAX_PARAMS];  // the start metric (restart value)
  double f;          // NLL at x
  double gp;         // g . p
  double alpha;      // current step length along p
  double edm;        // 0.5 g^T V g at x
  double edm_tol;
  double tol_f_rel;  // accepted NLL rise from rounding, relative to |f|
  int phase;         // 0: evaluating the start point; 1: line search along p
  int n_iter, n_eval, n_ls;
  int done;          // 0 running; 1 finished (status set)
  int status;        // UML_FIT_*
  int max_iter;
  int pad_;
};

// One dataset's share of a launch.
struct Job {
  const void* col[kMaxCols];      // event columns: kernel dimensions, then precomputed terms
  const void* w;                  // weights or nullptr
  int64_t n;                      // events
  int32_t n_tiles;
  int32_t events_per_thread;      // E: events per thread per tile
  ConstBlock* cst;                // constants of the last evaluated point (cache)
  double* partials;               // [K][n_tiles] tile partials, then [K][kGroups] group partials
                                  // (batched launches)
  double* spart;                  // 2 x [K][n_tiles] tile partials of single-dataset launches
                                  // (alternating), each kSentinel until written (see eval_kernel)
  unsigned long long* epoch;      // single-dataset launches so far (picks the buffer)
  unsigned int* counter;          // completion counters: kGroups group counters
                                  // and one global, each on its own 128-byte line
  double* out;                    // [1 + nfree]: nll, gradient
  const Plan* plan;               // device copy of the plan
  FitState* fit;                  // BFGS state (fit mode) or nullptr
  const double* theta;            // parameter vector to evaluate (device)
  int32_t npar;                   // parameters in theta
  long long key;                  // the model (Plan::key): part of the constant cache's key
};

// The bit pattern of a tile partial not yet written by the current launch: a
// signalling NaN, which FP64 arithmetic never produces (its NaNs are quiet).
constexpr unsigned long long kSentinel = 0x7ff4dead0000beefull;

// Completion counting: tile t reports to group counter t % kGroups; the last
// tile of a group reports to the global counter.  Same-address device-scope
// atomics serialise across the chip, so a single counter would cost one
// round of that serialisation per tile.
constexpr int kGroups = 64;
constexpr int kCounterStride = 32;  // uints: one counter per 128-byte line
constexpr int kCounterWords = (kGroups + 1) * kCounterStride;

// Events per thread per tile for a dataset of n events: about 256 tiles
// (one per CU) for mid-sized datasets, where the fixed cost of a launch
// dominates, with at most 16 events per thread up to 2M events, 32 up to 16M
// and 64 beyond (measured best with a new parameter point per launch: 4-D
// mixed 1e6 / 4e6 events, 1-D mixed 1e6 / 1e7 / 5e7).  A pure function of n
// and the precision, so a dataset is reduced in the same order whatever else
// shares the launch.
inline int events_per_thread(int64_t n, int precision) {
  const int vw = precision == UML_MIXED ? 4 : 2;
  const int64_t per = n / (int64_t(kBlock) * 256);
  const int cap = n <= (int64_t(1) << 21) ? 16 : n <= (int64_t(1) << 24) ? 32 : 64;
  int e = vw;
  while (e < per && e < cap) e *= 2;
  return e;
}

}  // namespace uml
