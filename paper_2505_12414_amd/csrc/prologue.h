// The prologue: FP64 parameter-only terms of one parameter point, shared by
// the event kernels and the Hessian kernel.  A workgroup runs it in three
// stages: each factor and each mixture fraction is the task of one lane, and
// the slow pieces (the erfc, exp and expm1 of the Gaussian and exponential
// normalisations, then the per-kind constants) run in different waves, so its
// latency is that of the slowest piece rather than the sum over all factors.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "uml_internal.h"

namespace uml {

// Everything here is inlined into its callers (no call ABI): the prologue's
// FP64 work runs before the event loop, so the register allocator can give
// the loop its full budget, and each out-of-line call would save and restore
// registers through scratch memory (measured to dominate the latency of a
// one-lane prologue built from such calls).
static __device__ __forceinline__ double p_erfc(double x) { return erfc(x); }
static __device__ __forceinline__ double p_exp(double x) { return exp(x); }
static __device__ __forceinline__ double p_log(double x) { return log(x); }
static __device__ __forceinline__ double p_log2(double x) { return log2(x); }
static __device__ __forceinline__ double p_expm1(double x) { return expm1(x); }

// Phi(zb) - Phi(za), za < zb, from two erfc values, taken where both
// arguments share a sign: phi_diff_args gives the arguments (u, v),
// phi_diff_from combines erfc(u) and erfc(v).
static __device__ __forceinline__ void phi_diff_args(double za, double zb, double& u, double& v) {
  const double r = 0.70710678118654752440;
  if (za >= 0.0) {
    u = za * r;
    v = zb * r;
  } else if (zb <= 0.0) {
    u = -zb * r;
    v = -za * r;
  } else {
    u = zb * r;
    v = -za * r;
  }
}
static __device__ __forceinline__ double phi_diff_from(double za, double zb, double eu, double ev) {
  if (za >= 0.0 || zb <= 0.0) return 0.5 * (eu - ev);
  return 1.0 - 0.5 * eu - 0.5 * ev;
}
static __device__ __forceinline__ double d_phi_diff(double za, double zb) {
  double u, v;
  phi_diff_args(za, zb, u, v);
  return phi_diff_from(za, zb, p_erfc(u), p_erfc(v));
}

static constexpr double kLog2e = 1.4426950408889634074;
static constexpr double kSqrt2Pi = 2.5066282746310005024;

// Stage 1 of the prologue: one transcendental function of a Gaussian or
// exponential factor per task; piece p of a factor runs on wave
// stage1_wave(kind, p), its half h (the two ends of the range) on lanes
// f and 16 + f of that wave, so both halves take one pass of the same code.
//   Gaussian     piece 0: tr[h] = erfc(u), erfc(v)
//                piece 1: tr[2 + h] = exp(-za^2/2), exp(-zb^2/2)
//   exponential  piece 0: tr[h] = expm1(lambda L), expm1(-lambda L) (the latter
//                unused near lambda L = 0)
static __device__ __forceinline__ void factor_stage1(const FactorPlan& F, const double* __restrict__ th,
                                                     int piece, int half, double* tr) {
  if (F.kind == FK_GAUSS) {
    const double mu = th[F.par[0]], sg = th[F.par[1]];
    const double za = (F.lo[0] - mu) / sg, zb = (F.hi[0] - mu) / sg;
    if (piece == 0) {
      double u, v;
      phi_diff_args(za, zb, u, v);
      tr[half] = p_erfc(half ? v : u);
    } else {
      const double z = half ? zb : za;
      tr[2 + half] = p_exp(-0.5 * z * z);
    }
  } else if (F.kind == FK_EXP) {
    const double lam = th[F.par[0]], z = lam * (F.hi[0] - F.lo[0]);
    if (half == 0)
      tr[0] = lam == 0.0 ? 0.0 : p_expm1(z);
    else
      tr[1] = (lam == 0.0 || fabs(z) < 0.05) ? 0.0 : p_expm1(-z);
  }
}

static constexpr double kInvSqrt2Pi = 0.39894228040143267794;

// Output of one factor's kernel constants, written in both precisions from
// registers (the FP32 copies are what the mixed-precision kernels load).
//   put:       the same value in both sets;
//   put2:      different values in the FP64 and FP32 sets;
//   put_pair:  v in the FP64 set (and 0 after it); in the FP32 set its
//              nearest FP32 value and the remainder, also in FP32, so that
//              the two carry v to about 2^-48 relative.
// A constant rounded once to FP32 is off by up to 2^-24 relative at every
// event alike: summed over N events such an error grows as N while the
// statistical uncertainty shrinks as 1/sqrt(N), so the constants through
// which every event's value depends on a parameter go to the kernels as
// pairs.
struct KOut {
  double* d;
  float* f;
  __device__ __forceinline__ void put(int i, double v) const {
    d[i] = v;
    f[i] = float(v);
  }
  __device__ __forceinline__ void put2(int i, double vd, double vf) const {
    d[i] = vd;
    f[i] = float(vf);
  }
  __device__ __forceinline__ void put_pair(int i, double v) const {
    const float hi = float(v);
    d[i] = v;
    d[i + 1] = 0.0;
    f[i] = hi;
    f[i + 1] = float(v - double(hi));
  }
};

// Gaussian normalised on [a, b] (Eq. 2): constants of the kernel, the
// epilogue coefficients of its gradient terms, and log2 of its prefactor
// 1 / (sigma sqrt(2 pi) (Phi(zb) - Phi(za))); tr from stage 1.
//   d ln g / d mu    = d / sigma^2 - (phi(za) - phi(zb)) / (sigma D)
//   d ln g / d sigma = d^2 / sigma^3 - 1/sigma - (za phi(za) - zb phi(zb)) / (sigma D)
// (1/sigma and 1/D are formed once: the divisions are long dependent chains.)
//
// Mixed precision: the events are FP32 values shifted by xref (an FP32
// value), exactly, so x' lies on the grid G = ulp(xref) / 2 wherever
// x is within a factor two of xref.  The centre c0 = mu - xref is split
// into c0_hi, a multiple of G, and the rest c0_lo (below G / 2): the
// kernel's d = x' - c0_hi is then exact, and
//   -c1 (d - c0_lo)^2 = -c1 d^2 + k2 d - c1 c0_lo^2,   k2 = 2 c1 c0_lo,
// with c1 = log2(e) / (2 sigma^2) as an FP32 pair and the last term folded
// into the prefactor.  (Rounding d itself would shift the centre by the
// same amount at every event of a binade of |d|.)  The moments are sums of
// d and d^2, so the epilogue coefficients take the shift by c0_lo:
//   sum r (d - c0_lo)   = M_d - c0_lo R,
//   sum r (d - c0_lo)^2 = M_dd - 2 c0_lo M_d + c0_lo^2 R.
// In FP64 c0_hi = c0 and c0_lo = 0.
static __device__ __forceinline__ bool gauss_constants(const FactorPlan& F, const double* __restrict__ th,
                                                       const double* tr, const KOut& k, double* ec,
                                                       double* lnorm2, bool mixed) {
  const double a = F.lo[0], b = F.hi[0];
  const double mu = th[F.par[0]], sg = th[F.par[1]];
  const double za = (a - mu) / sg, zb = (b - mu) / sg;  // as in stage 1
  const double isg = 1.0 / sg;
  const double D = phi_diff_from(za, zb, tr[0], tr[1]);
  const double iD = 1.0 / D;
  const double pa = tr[2] * kInvSqrt2Pi, pb = tr[3] * kInvSqrt2Pi;
  const double c0 = mu - F.xref, c1 = 0.5 * kLog2e * (isg * isg);
  double c0_hi = c0;
  if (mixed) {
    const double G = F.xref != 0.0 ? ldexp(1.0, ilogb(F.xref) - 24) : 0.0;
    c0_hi = double(float(G > 0.0 ? rint(c0 / G) * G : c0));
  }
  const double c0_lo = c0 - c0_hi;
  k.put2(0, c0, c0_hi);
  k.put_pair(1, c1);
  k.put2(3, 0.0, 2.0 * c1 * c0_lo);
  *lnorm2 = -p_log2(sg * kSqrt2Pi * D) - c1 * c0_lo * c0_lo;
  const double is2 = isg * isg, is3 = is2 * isg;
  ec[0] = is2;                                                        // x sum r d
  ec[1] = -(pa - pb) * (isg * iD) - c0_lo * is2;                      // x sum r
  ec[2] = is3;                                                        // x sum r d^2
  ec[3] = -(isg + (za * pa - zb * pb) * (isg * iD)) + c0_lo * c0_lo * is3;  // x sum r
  ec[4] = -2.0 * c0_lo * is3;                                         // x sum r d
  return sg > 0.0;
}

// Exponential e^{lambda x} normalised on [a, b] (Eq. 2), evaluated as
// 2^{lambda log2(e) x'} with x' = x - xref; the prefactor e^{lambda xref}/N
// is written through expm1 so that small |lambda| keeps full precision.
//   d ln p / d lambda = x' - (E[x] - xref)
// with E[x] - a = L h(lambda L), h(z) = 1/(1 - e^{-z}) - 1/z, by its Taylor
// series near z = 0; tr from stage 1.
static __device__ __forceinline__ bool exp_constants(const FactorPlan& F, const double* __restrict__ th,
                                                     const double* tr, const KOut& k, double* ec,
                                                     double* lnorm2) {
  const double a = F.lo[0], b = F.hi[0], xr = F.xref, L = b - a;
  const double lam = th[F.par[0]];
  k.put_pair(0, lam * kLog2e);
  ec[0] = 1.0;
  if (lam == 0.0) {
    *lnorm2 = -p_log2(L);
    ec[1] = -(a + 0.5 * L - xr);
  } else {
    const double z = lam * L;
    *lnorm2 = (lam * (xr - a) - p_log(tr[0] / lam)) * kLog2e;
    double h;
    if (fabs(z) < 0.05) {
      const double z2 = z * z;
      h = 0.5 + z * (1.0 / 12.0 + z2 * (-1.0 / 720.0 + z2 * (1.0 / 30240.0 - z2 / 1209600.0)));
    } else {
      h = -1.0 / tr[1] - 1.0 / z;
    }
    ec[1] = -(a - xr + L * h);
  }
  return true;
}

// Chebyshev series 1 + sum_j c_j T_j(u) on [a, b], u = (2x - a - b)/(b - a),
// with norm N_C = (b - a) + sum_{j even} c_j (b - a)/(1 - j^2).  The kernel
// evaluates v = sgn (1 + sum c_j T_j), sgn the sign of N_C, with u = x s + t
// (the scale s = 2/(b - a) as a pair); 1/|N_C| goes to the prefactor.
//   d ln p / d c_j = sgn T_j / v - J_j / N_C,  J_j = d N_C / d c_j
// Unrolled to the maximum order, so the coefficient reads go out together.
// N_C = 0 is outside the domain.
static __device__ __forceinline__ bool cheb_constants(const FactorPlan& F, const double* __restrict__ th,
                                                      const KOut& k, double* ec, double* lnorm2) {
  const double a = F.lo[0], b = F.hi[0], xr = F.xref, L = b - a;
  const int n = F.order;
  double J[kMaxCheb], c[kMaxCheb];
#pragma unroll
  for (int j = 0; j < kMaxCheb; ++j) {
    const int jj = j + 1;
    J[j] = (jj % 2 == 0) ? L / (1.0 - double(jj * jj)) : 0.0;
    c[j] = th[F.par[j < n ? j : 0]];
  }
  double N = L;
#pragma unroll
  for (int j = 0; j < kMaxCheb; ++j)
    if (j < n) N += c[j] * J[j];
  const double iL = 1.0 / L, iN = 1.0 / N, sgn = N < 0.0 ? -1.0 : 1.0;
  k.put_pair(0, 2.0 * iL);
  k.put(2, (2.0 * xr - a - b) * iL);
  k.put(3, sgn);
#pragma unroll
  for (int j = 0; j < kMaxCheb; ++j)
    if (j < n) {
      k.put(4 + j, sgn * c[j]);
      ec[j] = sgn;             // x sum q T_j
      ec[n + j] = -J[j] * iN;  // x sum r
    }
  *lnorm2 = -p_log2(fabs(N));
  return N != 0.0;
}

// P-wave density (Eq. 4), evaluated without its factor 9/(32 pi), which goes
// to the prefactor: coefficients {FL, S3, 4 S4, 2 S5, 4/3 AFB, 2 S7, 4 S8,
// 2 S9} as FP32 pairs (the 8 hi parts, then the 8 lo parts: an FP32 F_L alone
// is off by up to 4e-8, a shift every event shares); d ln A / d S_k =
// s_k b_k / A' with A' the density without 9/(32 pi).
static __device__ __forceinline__ void pwave_constants(const FactorPlan& F, const double* __restrict__ th,
                                                       const KOut& k, double* ec, double* lnorm2) {
  const double scale[8] = {1.0, 1.0, 4.0, 2.0, 4.0 / 3.0, 2.0, 4.0, 2.0};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double c = scale[i] * th[F.par[i]];
    const float hi = float(c);
    k.put2(i, c, hi);
    k.put2(8 + i, 0.0, c - double(hi));
    ec[i] = scale[i];
  }
  *lnorm2 = -3.4815711280300066;  // log2(9 / (32 pi))
}

// Stage 2 for one factor: kernel constants, epilogue constants ec and log2
// of its parameter-only prefactor; false outside the factor's domain.
static __device__ __forceinline__ bool factor_constants(const FactorPlan& F, const double* __restrict__ th,
                                                        const double* tr, const KOut& k, double* ec,
                                                        double* lnorm2, bool mixed) {
  *lnorm2 = 0.0;
  switch (F.kind) {
    case FK_GAUSS: return gauss_constants(F, th, tr, k, ec, lnorm2, mixed);
    case FK_EXP: return exp_constants(F, th, tr, k, ec, lnorm2);
    case FK_CHEB: return cheb_constants(F, th, k, ec, lnorm2);
    case FK_PWAVE: pwave_constants(F, th, k, ec, lnorm2); return true;
  }
  return false;
}

static_assert(kMaxFac <= 16 && kMaxComp * 8 <= 32, "prologue tasks: factors on lanes 0-31, fractions on 32-63");
static_assert((kMaxFac & (kMaxFac - 1)) == 0, "factor indices are masked with kMaxFac - 1");

// The waves of the two stages, chosen so that the slow pieces run side by
// side on different SIMDs: stage 1 puts the Gaussians' erfc on wave 0, their
// exp on wave 1, the exponentials' expm1 on wave 2 and the fractions on wave 3;
// stage 2 gives each factor kind a wave of its own.
static constexpr int kFracWave = 3;
static __device__ __forceinline__ int stage1_wave(int kind, int piece, int nwaves) {
  return (kind == FK_GAUSS ? piece : 2) % nwaves;
}
static __device__ __forceinline__ int prologue_wave(int kind, int nwaves) {
  return (kind >= FK_GAUSS && kind <= FK_PWAVE) ? (kind - FK_GAUSS) % nwaves : 0;
}

// LDS-qualified views: the prologue's inputs and output are typed as LDS, so
// every access is a direct LDS one.  (A generic, flat, access is tracked by
// both the vector-memory and the LDS counters: each later LDS read would wait
// for it.)
using LdsPlan = const __attribute__((address_space(3))) Plan;
using LdsDouble = const __attribute__((address_space(3))) double;
using LdsConstBlock = __attribute__((address_space(3))) ConstBlock;
template <class T>
static __device__ __forceinline__ auto lds(T* p) {
  return (__attribute__((address_space(3))) T*)p;
}

// The prologue: every parameter-only term of the point th (Sec. 2.4.1 and
// Eq. 3) written to cb.  Called by every thread of a workgroup whose size is
// a multiple of 64, at most 1024 (it synchronises the workgroup; the caller
// synchronises again before other threads read cb).  P, th (all npar
// parameters) and cb sit in LDS (store_const_block copies cb out).
//   stage 1  lanes f and 16 + f of the waves of stage1_wave: the
//            transcendental functions of factor f; lane 32 + 8c + k of
//            wave kFracWave: fraction entry k of component c (log2 and
//            d ln F_c / d f);
//   stage 2  lane f of the wave of its kind: factor f's constants;
//   stage 3  lane c of wave 0: component c's log2 prefactor, summed in a
//            fixed order (its fractions, then its factors), so the result
//            does not depend on timing.
static __device__ __forceinline__ void compute_constants(LdsPlan* P_lds, LdsDouble* __restrict__ th_lds,
                                                         LdsConstBlock* cb_lds) {
  __shared__ double s_tr[kMaxFac][4];      // stage-1 results per factor
  __shared__ double s_ln2[kMaxFac];        // log2 prefactor of each factor
  __shared__ double s_fl2[kMaxComp * 8];   // log2 of each fraction entry
  __shared__ int s_bad[16];                // per wave: a task left the domain
  const Plan& P = *(const Plan*)P_lds;
  const double* __restrict__ th = (const double*)th_lds;
  ConstBlock* cb = (ConstBlock*)cb_lds;
  const int tid = threadIdx.x;
  const int nw = blockDim.x >> 6, w = tid >> 6, lane = tid & 63;
  bool ok = true;
  // Plan entries of stages 2 and 3, and the point's copy, read before stage 1
  // so that their LDS round trips overlap it: the factor kind of lane f, and
  // the fraction count, factor count, factors and output slot of component c
  // (lane c of wave 0).
  const int nfac = P.nfac, npar = P.npar, ncomp = P.ncomp;
  const int kind2 = lane < nfac ? P.fac[lane].kind : -1;
  const double th_copy = (w == nw - 1 && lane >= 32 && lane - 32 < npar) ? th[lane - 32] : 0.0;
  int c_nfrac = 0, c_nfac = 0, c_lk2 = 0, c_fac[kMaxFacPerComp];
#pragma unroll
  for (int j = 0; j < kMaxFacPerComp; ++j) c_fac[j] = 0;
  if (tid < ncomp) {
    const CompPlan& C = P.comp[tid];
    c_nfrac = C.nfrac;
    c_nfac = C.nfac;
    c_lk2 = C.cst_lk2;
#pragma unroll
    for (int j = 0; j < kMaxFacPerComp; ++j) c_fac[j] = C.fac[j] & (kMaxFac - 1);
  }
  // stage 1
  if (lane < 32 && (lane & 15) < P.nfac) {
    const int f = lane & 15, half = lane >> 4;
    const FactorPlan& F = P.fac[f];
    if (F.kind == FK_GAUSS || F.kind == FK_EXP)
      for (int piece = 0; piece < (F.kind == FK_GAUSS ? 2 : 1); ++piece)
        if (stage1_wave(F.kind, piece, nw) == w) factor_stage1(F, th, piece, half, s_tr[f]);
  }
  if (lane >= 32 && w == kFracWave % nw) {
    const int c = (lane - 32) >> 3, k = (lane - 32) & 7;
    if (c < P.ncomp && k < P.comp[c].nfrac) {
      const CompPlan& C = P.comp[c];
      const double f = th[C.frac_par[k]];
      ok = f >= 0.0 && f <= 1.0;
      s_fl2[lane - 32] = p_log2(C.frac_sign[k] > 0 ? f : 1.0 - f);
      cb->e[C.frac_ec[k]] = C.frac_sign[k] > 0 ? 1.0 / f : -1.0 / (1.0 - f);  // d ln F_c / d f
    }
  }
  if (tid < P.ndim) {
    cb->xd[tid] = P.xref[tid];
    cb->xf[tid] = float(P.xref[tid]);
  }
  __syncthreads();
  // stage 2
  if (kind2 >= 0 && prologue_wave(kind2, nw) == w) {
    const FactorPlan& F = P.fac[lane];
    const KOut ko{cb->d + F.cst, cb->f + F.cst};
    ok = factor_constants(F, th, s_tr[lane], ko, cb->e + F.ecst, &s_ln2[lane], P.precision == UML_MIXED) && ok;
  }
  if (w == nw - 1 && lane >= 32 && lane - 32 < npar) cb->theta[lane - 32] = th_copy;
  const bool wave_bad = __ballot(ok ? 0 : 1) != 0;
  if (lane == 0 && w < 16) s_bad[w] = wave_bad ? 1 : 0;
  __syncthreads();
  // stage 3 (unrolled to the maximum counts, with every read unconditional and
  // the unused entries replaced by zero, so the reads go out together)
  if (tid < ncomp) {
    double v[8 + kMaxFacPerComp];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = s_fl2[tid * 8 + k];
#pragma unroll
    for (int j = 0; j < kMaxFacPerComp; ++j) v[8 + j] = s_ln2[c_fac[j]];
    double lk2 = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) lk2 += k < c_nfrac ? v[k] : 0.0;
#pragma unroll
    for (int j = 0; j < kMaxFacPerComp; ++j) lk2 += j < c_nfac ? v[8 + j] : 0.0;
    const float hi = float(lk2);
    cb->d[c_lk2] = lk2;
    cb->d[c_lk2 + 1] = 0.0;
    cb->f[c_lk2] = hi;
    cb->f[c_lk2 + 1] = float(lk2 - double(hi));
  }
  if (tid == 0) {
    int bad = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) bad |= i < nw ? s_bad[i] : 0;
    cb->domain_ok = bad ? 0 : 1;
    cb->valid = 1;
    cb->key = P.key;
  }
}

// Copies a constant block from LDS to global memory, by the whole workgroup.
static __device__ __forceinline__ void store_const_block(ConstBlock* dst, const ConstBlock& src) {
  const int4* s4 = reinterpret_cast<const int4*>(&src);
  int4* d4 = reinterpret_cast<int4*>(dst);
  for (int i = threadIdx.x; i < int(sizeof(ConstBlock) / 16); i += blockDim.x) d4[i] = s4[i];
}

}  // namespace uml
