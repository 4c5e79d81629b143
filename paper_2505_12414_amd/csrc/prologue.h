// The prologue: FP64 parameter-only terms of one parameter point, shared by
// the event kernels and the Hessian kernel.  Everything here runs once per
// point on one lane.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "uml_internal.h"

namespace uml {

// The FP64 library functions are called, not inlined, from the once-per-point
// code below: the event kernels' register budget is the maximum over every
// function they can reach, and the event loop must not pay for erfc.
static __device__ __noinline__ double nl_erfc(double x) { return erfc(x); }
static __device__ __noinline__ double nl_exp(double x) { return exp(x); }
static __device__ __noinline__ double nl_log(double x) { return log(x); }
static __device__ __noinline__ double nl_log2(double x) { return log2(x); }
static __device__ __noinline__ double nl_expm1(double x) { return expm1(x); }

// Phi(zb) - Phi(za), za < zb, with erfc where both share a sign.
static __device__ __noinline__ double d_phi_diff(double za, double zb) {
  const double r = 0.70710678118654752440;
  if (za >= 0.0) return 0.5 * (nl_erfc(za * r) - nl_erfc(zb * r));
  if (zb <= 0.0) return 0.5 * (nl_erfc(-zb * r) - nl_erfc(-za * r));
  return 1.0 - 0.5 * nl_erfc(zb * r) - 0.5 * nl_erfc(-za * r);
}

// Mean offset of a truncated exponential: E[x] - a = L * h(lambda L),
// h(z) = 1/(1 - e^{-z}) - 1/z, by its Taylor series near z = 0.
static __device__ __noinline__ double d_exp_h(double z) {
  if (fabs(z) < 0.05) {
    const double z2 = z * z;
    return 0.5 + z * (1.0 / 12.0 + z2 * (-1.0 / 720.0 + z2 * (1.0 / 30240.0 - z2 / 1209600.0)));
  }
  return -1.0 / nl_expm1(-z) - 1.0 / z;
}

static constexpr double kLog2e = 1.4426950408889634074;
static constexpr double kSqrt2Pi = 2.5066282746310005024;

// Gaussian normalised on [a, b] (Eq. 2): constants of the kernel, the
// epilogue coefficients of its gradient terms, and log2 of its prefactor
// 1 / (sigma sqrt(2 pi) (Phi(zb) - Phi(za))).
//   d ln g / d mu    = d / sigma^2 - (phi(za) - phi(zb)) / (sigma D)
//   d ln g / d sigma = d^2 / sigma^3 - 1/sigma - (za phi(za) - zb phi(zb)) / (sigma D)
static __device__ __noinline__ bool gauss_constants(const FactorPlan& F, const double* __restrict__ th,
                                             double* kc, double* ec, double* lnorm2) {
  const double a = F.lo[0], b = F.hi[0];
  const double mu = th[F.par[0]], sg = th[F.par[1]];
  const double za = (a - mu) / sg, zb = (b - mu) / sg;
  const double D = d_phi_diff(za, zb);
  const double pa = nl_exp(-0.5 * za * za) / kSqrt2Pi, pb = nl_exp(-0.5 * zb * zb) / kSqrt2Pi;
  kc[0] = mu - F.xref;
  kc[1] = kLog2e / (2.0 * sg * sg);
  *lnorm2 = -nl_log2(sg * kSqrt2Pi * D);
  ec[0] = 1.0 / (sg * sg);                           // x sum r d
  ec[1] = -(pa - pb) / (sg * D);                     // x sum r
  ec[2] = 1.0 / (sg * sg * sg);                      // x sum r d^2
  ec[3] = -(1.0 / sg + (za * pa - zb * pb) / (sg * D));  // x sum r
  return sg > 0.0;
}

// Exponential e^{lambda x} normalised on [a, b] (Eq. 2), evaluated as
// 2^{lambda log2(e) x'} with x' = x - xref; the prefactor e^{lambda xref}/N
// is written through expm1 so that small |lambda| keeps full precision.
//   d ln p / d lambda = x' - (E[x] - xref)
static __device__ __noinline__ bool exp_constants(const FactorPlan& F, const double* __restrict__ th,
                                           double* kc, double* ec, double* lnorm2) {
  const double a = F.lo[0], b = F.hi[0], xr = F.xref, L = b - a;
  const double lam = th[F.par[0]];
  kc[0] = lam * kLog2e;
  ec[0] = 1.0;
  if (lam == 0.0) {
    *lnorm2 = -nl_log2(L);
    ec[1] = -(a + 0.5 * L - xr);
  } else {
    const double z = lam * L;
    *lnorm2 = (lam * (xr - a) - nl_log(nl_expm1(z) / lam)) * kLog2e;
    ec[1] = -(a - xr + L * d_exp_h(z));
  }
  return true;
}

// Chebyshev series 1 + sum_j c_j T_j(u) on [a, b], u = (2x - a - b)/(b - a),
// with norm N_C = (b - a) + sum_{j even} c_j (b - a)/(1 - j^2).
//   d ln p / d c_j = T_j / (1 + sum c T) - J_j / N_C,  J_j = d N_C / d c_j
static __device__ __noinline__ bool cheb_constants(const FactorPlan& F, const double* __restrict__ th,
                                            double* kc, double* ec) {
  const double a = F.lo[0], b = F.hi[0], xr = F.xref;
  const int k = F.order;
  double N = b - a;
  for (int jj = 1; jj <= k; ++jj) {
    const double J = (jj % 2 == 0) ? (b - a) / (1.0 - double(jj * jj)) : 0.0;
    N += th[F.par[jj - 1]] * J;
    ec[k + jj - 1] = J;
  }
  kc[0] = 2.0 / (b - a);
  kc[1] = (2.0 * xr - a - b) / (b - a);
  kc[2] = 1.0 / N;
  for (int jj = 1; jj <= k; ++jj) {
    kc[2 + jj] = th[F.par[jj - 1]] / N;
    ec[jj - 1] = 1.0 / N;                      // x sum q T_j
    ec[k + jj - 1] = -ec[k + jj - 1] / N;      // x sum r
  }
  return true;
}

// P-wave density (Eq. 4): coefficients 9/(32 pi) {1, FL, S3, 4 S4, 2 S5,
// 4/3 AFB, 2 S7, 4 S8, 2 S9}; d ln A / d S_k = 9/(32 pi) s_k b_k / A.
static __device__ __noinline__ void pwave_constants(const FactorPlan& F, const double* __restrict__ th,
                                             double* kc, double* ec) {
  const double kap = 9.0 / (32.0 * M_PI);
  const double scale[8] = {1.0, 1.0, 4.0, 2.0, 4.0 / 3.0, 2.0, 4.0, 2.0};
  kc[0] = kap;
  for (int k = 0; k < 8; ++k) {
    kc[1 + k] = kap * scale[k] * th[F.par[k]];
    ec[k] = kap * scale[k];
  }
}

// The prologue: every parameter-only term of the point theta (Sec. 2.4.1).
static __device__ __noinline__ void compute_constants(const Plan& P, const double* __restrict__ th,
                                               ConstBlock* cb) {
  bool ok = true;
  for (int i = 0; i < P.npar; ++i) cb->theta[i] = th[i];
  for (int ci = 0; ci < P.ncomp; ++ci) {
    const CompPlan& C = P.comp[ci];
    double lk2 = 0.0;
    for (int k = 0; k < C.nfrac; ++k) {
      const double f = th[C.frac_par[k]];
      if (!(f >= 0.0 && f <= 1.0)) ok = false;
      lk2 += nl_log2(C.frac_sign[k] > 0 ? f : 1.0 - f);
      cb->e[C.frac_ec[k]] = C.frac_sign[k] > 0 ? 1.0 / f : -1.0 / (1.0 - f);  // d ln F_c / d f
    }
    for (int j = 0; j < C.nfac; ++j) {
      const FactorPlan& F = P.fac[C.fac[j]];
      double* kc = cb->d + F.cst;
      double* ec = cb->e + F.ecst;
      double ln2 = 0.0;
      switch (F.kind) {
        case FK_GAUSS: ok = gauss_constants(F, th, kc, ec, &ln2) && ok; break;
        case FK_EXP: ok = exp_constants(F, th, kc, ec, &ln2) && ok; break;
        case FK_CHEB: ok = cheb_constants(F, th, kc, ec) && ok; break;
        case FK_PWAVE: pwave_constants(F, th, kc, ec); break;
        default: ok = false;
      }
      lk2 += ln2;
    }
    cb->d[C.cst_lk2] = lk2;
  }
  for (int i = 0; i < P.ncst; ++i) cb->f[i] = float(cb->d[i]);
  for (int d = 0; d < P.ndim; ++d) {
    cb->xd[d] = P.xref[d];
    cb->xf[d] = float(P.xref[d]);
  }
  cb->domain_ok = ok ? 1 : 0;
  cb->valid = 1;
}

}  // namespace uml
