// Event kernels of libuml for gfx950.
//
// One launch evaluates -sum_i w_i ln P(x_i|theta) (Eq. 1) and every sum the
// gradient needs, for one dataset or for many (one "job" each):
//   * each workgroup owns one fixed-size tile of one job's events; each lane
//     reads its events as 16-byte vectors from the structure-of-arrays columns,
//     computes the mixture in base-2 log space and accumulates the K moment
//     sums in registers (FP32 in mixed mode, FP64 otherwise);
//   * the workgroup reduces its lanes through LDS in a fixed order and writes
//     one FP64 partial per moment and tile (pass 1);
//   * the last workgroup of a job to finish (an integer atomic counter) sums
//     the tile partials in tile order with Neumaier compensation (pass 2) and
//     assembles NLL and gradient in FP64 (epilogue).
// No floating-point atomics: results are bitwise reproducible and independent
// of the grid, because a tile's lanes, its reduction order and the tile size
// depend only on the job's own event count.
//
// The parameter-only terms (normalisation integrals, the combined prefactors
// of Eq. 3, the angular coefficients) are computed once per parameter point by
// the prologue kernel in FP64 and rounded to FP32 for mixed mode.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <type_traits>
#include <utility>

#include "devmath.h"
#include "kernels.h"
#include "prologue.h"
#include "uml_internal.h"

namespace uml {

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------

template <int I, class... Ts>
struct TypeAt;
template <class T, class... Ts>
struct TypeAt<0, T, Ts...> {
  using type = T;
};
template <int I, class T, class... Ts>
struct TypeAt<I, T, Ts...> {
  using type = typename TypeAt<I - 1, Ts...>::type;
};

template <class Fn, int... Is>
__host__ __device__ __forceinline__ void sfor_impl(Fn&& fn, std::integer_sequence<int, Is...>) {
  (fn(std::integral_constant<int, Is>{}), ...);
}
template <int N, class Fn>
__host__ __device__ __forceinline__ void sfor(Fn&& fn) {
  sfor_impl(fn, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// arithmetic of the two precisions
// ---------------------------------------------------------------------------

struct PrecMixed {
  using T = float;
  static constexpr int VW = 4;  // one 16-byte load = 4 events
  __device__ static const float* consts(const ConstBlock* cb) { return cb->f; }
  __device__ static const float* xrefs(const ConstBlock* cb) { return cb->xf; }
};
struct PrecF64 {
  using T = double;
  static constexpr int VW = 2;
  __device__ static const double* consts(const ConstBlock* cb) { return cb->d; }
  __device__ static const double* xrefs(const ConstBlock* cb) { return cb->xd; }
};

// ---------------------------------------------------------------------------
// catalogue factors: per-event value and moments
//   exp-type factors add to the component's base-2 exponent e,
//   polynomial-type factors return their value v;
//   m[] receives the event-dependent factors of the moment sums.
// Kernel constants c[] are written by the prologue (see compute_constants).
// In mixed precision a constant through which every event depends on a
// parameter comes as an FP32 pair (hi, lo), and the lo part enters before
// the rounding of a value that varies from event to event, so its effect is
// not lost to the same rounding at every event.
// ---------------------------------------------------------------------------

template <class T>
constexpr bool kF32 = std::is_same<T, float>::value;

// Gaussian in dimension D.  c = {c0_hi, c1_hi, c1_lo, k2}: the exponent
// -c1 (d - c0_lo)^2 with c1 = log2(e) / (2 sigma^2), d = x' - c0_hi exact and
// k2 = 2 c1 c0_lo (FP32 only; in FP64 c0_hi = mu - xref, c0_lo = 0).
template <int D>
struct Gauss {
  static constexpr int kind = FK_GAUSS, order = 0;
  static constexpr int ncst = fk_ncst(FK_GAUSS, 0), nmom = fk_nmom(FK_GAUSS, 0);
  static constexpr bool expo = true;
  static constexpr int maxdim = D;
  static constexpr unsigned shift_mask = 1u << D;
  static constexpr bool pre = false;  // event-only terms stored as columns
  static std::string sig() { return "G" + std::to_string(D); }
  template <class T>
  __device__ static __forceinline__ void eval(const T* xs, const T* c, T& e, T& v, T* m) {
    const T d = xs[D] - c[0];
    const T d2 = d * d;
    if constexpr (kF32<T>) e = fma(d, fma(-c[2], d, c[3]), e);
    e = fma(-d2, c[1], e);
    m[0] = d;
    m[1] = d2;
    (void)v;
  }
};

// Exponential e^{lambda x} in dimension D.  c = {lambda log2(e)} as a pair.
template <int D>
struct Exp {
  static constexpr int kind = FK_EXP, order = 0;
  static constexpr int ncst = fk_ncst(FK_EXP, 0), nmom = fk_nmom(FK_EXP, 0);
  static constexpr bool expo = true;
  static constexpr int maxdim = D;
  static constexpr unsigned shift_mask = 1u << D;
  static constexpr bool pre = false;  // event-only terms stored as columns
  static std::string sig() { return "E" + std::to_string(D); }
  template <class T>
  __device__ static __forceinline__ void eval(const T* xs, const T* c, T& e, T& v, T* m) {
    if constexpr (kF32<T>) e = fma(xs[D], c[1], e);
    e = fma(xs[D], c[0], e);
    m[0] = xs[D];
    (void)v;
  }
};

// Chebyshev series of order N in dimension D without its norm (which is in
// the component's prefactor): v = sgn (1 + sum c_j T_j(u)), sgn the sign of
// the norm.  c = {s_hi, s_lo, t, sgn, sgn c_1 .. sgn c_N}, u = x s + t.
template <int D, int N>
struct Cheb {
  static constexpr int kind = FK_CHEB, order = N;
  static constexpr int ncst = fk_ncst(FK_CHEB, N), nmom = fk_nmom(FK_CHEB, N);
  static constexpr bool expo = false;
  static constexpr int maxdim = D;
  static constexpr unsigned shift_mask = 0;
  static constexpr bool pre = false;  // event-only terms stored as columns
  static std::string sig() { return "C" + std::to_string(D) + "." + std::to_string(N); }
  template <class T>
  __device__ static __forceinline__ void eval(const T* xs, const T* c, T& e, T& v, T* m) {
    const T u = kF32<T> ? fma(xs[D], c[0], fma(xs[D], c[1], c[2])) : fma(xs[D], c[0], c[2]);
    T tj[N + 1];
    tj[0] = T(1);
    tj[1] = u;
    if constexpr (N >= 2) {
      const T u2 = u + u;
#pragma unroll
      for (int j = 2; j <= N; ++j) tj[j] = fma(u2, tj[j - 1], -tj[j - 2]);
    }
    T val = c[3];
#pragma unroll
    for (int j = 1; j <= N; ++j) {
      val = fma(c[3 + j], tj[j], val);
      m[j - 1] = tj[j];
    }
    v = val;
    (void)e;
  }
};

// The event-only terms of the P-wave density of one event (see PWave):
// u0 and the eight angular terms m.  One function for the kernel that
// recomputes them and for the kernel that stores them, so both give the same
// values.
template <class T>
__device__ __forceinline__ void pwave_terms(T cl, T ck, T ph, T& u0, T (&m)[8]) {
  const T sl2 = fma(-cl, cl, T(1));  // sin^2 theta_l
  const T sk2 = fma(-ck, ck, T(1));  // sin^2 theta_K
  const T skl2 = sk2 * sl2;
  const T skl = k_sqrt(skl2);        // sin theta_K sin theta_l
  T sp, cp;
  k_sincos(ph, sp, cp);
  const T w = ck * skl;              // sin 2K sin l / 2
  const T wc = w * cl;               // sin 2K sin 2l / 4
  u0 = fma(T(-0.5), skl2, sk2);
  m[0] = fma((ck + ck) * ck, sl2, -u0);  // u1 - u0
  m[1] = skl2 * fma(cp + cp, cp, T(-1)); // S3: sin^2K sin^2l cos 2phi
  m[2] = wc * cp;                        // S4 / 4
  m[3] = w * cp;                         // S5 / 2
  m[4] = sk2 * cl;                       // AFB / (4/3)
  m[5] = w * sp;                         // S7 / 2
  m[6] = wc * sp;                        // S8 / 4
  m[7] = skl2 * (sp * cp);               // S9 / 2
}

// v = u0 + sum_k c_k m_k with the coefficients c (8 hi parts, then in FP32
// their 8 lo parts): the lo terms first, then the hi terms, then u0.
template <class T>
__device__ __forceinline__ T pwave_value(const T* c, T u0, const T* m) {
  T val;
  if constexpr (kF32<T>) {
    val = c[8] * m[0];
#pragma unroll
    for (int k = 1; k < 8; ++k) val = fma(c[8 + k], m[k], val);
#pragma unroll
    for (int k = 0; k < 8; ++k) val = fma(c[k], m[k], val);
    val += u0;
  } else {
    val = u0;
#pragma unroll
    for (int k = 0; k < 8; ++k) val = fma(c[k], m[k], val);
  }
  return val;
}

// P-wave angular density (Eq. 4) in dimensions (cos theta_l, cos theta_K, phi),
// without its factor 9/(32 pi) (in the component's prefactor).
// Written as  v = u0 + c0 (u1 - u0) + sum_k c_k b_k  with
//   u0 = sin^2 K (3/4 + cos 2l / 4) = sin^2 K (1 - sin^2 l / 2),
//   u1 = cos^2 K (1 - cos 2l) = 2 cos^2 K sin^2 l,
//   b  = the S3, S4, S5, AFB, S7, S8, S9 terms without their constant
//        factors (1, 4, 2, 4/3, 2, 4, 2), which the prologue folds into
//        c = {FL, S3, 4 S4, 2 S5, 4/3 AFB, 2 S7, 4 S8, 2 S9} (then, in FP32,
//        the lo parts of the same 8: their sum over the terms is taken first,
//        then the hi terms, then u0, so each enters before a rounding of a
//        value that varies from event to event);
// moments m = {u1 - u0, b_S3, .., b_S9}.  sin K sin l = sqrt(sin^2 K sin^2 l)
// needs one square root; 1 - c^2 is one FMA (correctly rounded).
template <int D0, int D1, int D2>
struct PWave {
  static constexpr int kind = FK_PWAVE, order = 0;
  static constexpr int ncst = fk_ncst(FK_PWAVE, 0), nmom = fk_nmom(FK_PWAVE, 0);
  static constexpr bool expo = false;
  static constexpr int maxdim = D0 > D1 ? (D0 > D2 ? D0 : D2) : (D1 > D2 ? D1 : D2);
  static constexpr unsigned shift_mask = 0;
  static constexpr bool pre = false;  // event-only terms stored as columns
  static std::string sig() {
    return "P" + std::to_string(D0) + std::to_string(D1) + std::to_string(D2);
  }
  template <class T>
  __device__ static __forceinline__ void eval(const T* xs, const T* c, T& e, T& v, T* m) {
    T u0, mm[8];
    pwave_terms(xs[D0], xs[D1], xs[D2], u0, mm);
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = mm[k];
    v = pwave_value(c, u0, mm);
    (void)e;
  }
};

// The P-wave density with its event-only terms read from the nine stored
// columns B .. B+8 (u0, then the eight angular terms), computed once per
// dataset (the optimisation of event-dependent terms, Sec. 2.4.2).
template <int B>
struct PWavePre {
  static constexpr int kind = FK_PWAVE, order = 0;
  static constexpr int ncst = fk_ncst(FK_PWAVE, 0), nmom = fk_nmom(FK_PWAVE, 0);
  static constexpr bool expo = false;
  static constexpr int maxdim = B + kPWaveTerms - 1;
  static constexpr unsigned shift_mask = 0;
  static constexpr bool pre = true;  // event-only terms stored as columns
  static std::string sig() { return "Q" + std::to_string(B); }
  template <class T>
  __device__ static __forceinline__ void eval(const T* xs, const T* c, T& e, T& v, T* m) {
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = xs[B + 1 + k];
    v = pwave_value(c, xs[B], m);
    (void)e;
  }
};

template <class... F>
struct Comp {
  static constexpr int nfac = sizeof...(F);
  static constexpr int ncst = kCompCst + (F::ncst + ... + 0);
  static constexpr int nmom = 1 + (F::nmom + ... + 0);
  static constexpr int maxdim = std::max({F::maxdim...});
  static constexpr unsigned shift_mask = (F::shift_mask | ... | 0u);
  static constexpr bool pre = (F::pre || ... || false);
  template <int I>
  using fac = typename TypeAt<I, F...>::type;
  // offsets inside the component's block: constants after log2 K_c (a
  // pair), moments after r_c
  static constexpr int cst_off(int i) {
    constexpr int a[] = {F::ncst...};
    int o = kCompCst;
    for (int k = 0; k < i; ++k) o += a[k];
    return o;
  }
  static constexpr int mom_off(int i) {
    constexpr int a[] = {F::nmom...};
    int o = 1;
    for (int k = 0; k < i; ++k) o += a[k];
    return o;
  }
  static std::string sig() { return (std::string() + ... + F::sig()); }
};

template <class... C>
struct Shape {
  static constexpr int ncomp = sizeof...(C);
  static constexpr int K = 1 + (C::nmom + ...);
  static constexpr int ncst = (C::ncst + ...);
  static constexpr int ndim = std::max({C::maxdim...}) + 1;
  static constexpr unsigned shift_mask = (C::shift_mask | ...);
  static constexpr bool pre = (C::pre || ...);
  template <int I>
  using comp = typename TypeAt<I, C...>::type;
  static constexpr int cst_base(int i) {
    constexpr int a[] = {C::ncst...};
    int o = 0;
    for (int k = 0; k < i; ++k) o += a[k];
    return o;
  }
  static constexpr int mom_base(int i) {  // slot of r_c
    constexpr int a[] = {C::nmom...};
    int o = 1;
    for (int k = 0; k < i; ++k) o += a[k];
    return o;
  }
  static std::string sig() {
    std::string s;
    ((s += (s.empty() ? "" : "|") + C::sig()), ...);
    return s;
  }
};

// ---------------------------------------------------------------------------
// one event
// ---------------------------------------------------------------------------

// Every factor of every component at one event (shifted coordinates xs):
// the base-2 exponent E_c and polynomial product V_c of each component, the
// factor values pv and the event-dependent moment factors mom.
template <class S, class T>
__device__ __forceinline__ void components(const T (&x)[S::ndim], const T (&c)[S::ncst],
                                           const T (&xref)[S::ndim], T (&E)[S::ncomp],
                                           T (&V)[S::ncomp], T (&mom)[S::K],
                                           T (&pv)[S::ncomp][kMaxFacPerComp]) {
  constexpr int NC = S::ncomp;
  T xs[S::ndim];
  sfor<S::ndim>([&](auto Id) {
    constexpr int d = Id;
    if constexpr ((S::shift_mask >> d) & 1u)
      xs[d] = x[d] - xref[d];  // exact in FP32 for x within [xref/2, 2 xref]
    else
      xs[d] = x[d];
  });
  sfor<NC>([&](auto Ic) {
    constexpr int ci = Ic;
    using Cc = typename S::template comp<ci>;
    constexpr int cb = S::cst_base(ci), mb = S::mom_base(ci);
    // log2 K_c: the exponent starts from its lo part and takes the hi part
    // last (FP32), so the lo part is added before the final rounding
    T e = kF32<T> ? c[cb + 1] : c[cb];
    T v = T(1);
    sfor<Cc::nfac>([&](auto If) {
      constexpr int fi = If;
      using Fc = typename Cc::template fac<fi>;
      T pval = T(1);
      Fc::template eval<T>(xs, c + cb + Cc::cst_off(fi), e, pval, mom + mb + Cc::mom_off(fi));
      pv[ci][fi] = pval;
      if constexpr (!Fc::expo) v *= pval;
    });
    E[ci] = kF32<T> ? e + c[cb] : e;
    V[ci] = v;
  });
}

// The mixture in base-2 log space: P = 2^Emax sum, sum = sum_c Sp_c with
// Sp_c = 2^{E_c - Emax} V_c = ec_c V_c.
template <int NC, class T>
__device__ __forceinline__ void combine(const T (&E)[NC], const T (&V)[NC], T (&ec)[NC], T& Emax,
                                        T (&Sp)[NC], T& sum) {
  if constexpr (NC == 1) {
    ec[0] = T(1);
    Emax = E[0];
  } else if constexpr (NC == 2) {
    const T dE = E[0] - E[1];
    const T t = k_exp2(-fabs(dE));
    const bool ge = dE >= T(0);
    ec[0] = ge ? T(1) : t;
    ec[1] = ge ? t : T(1);
    Emax = ge ? E[0] : E[1];
  } else {
    Emax = E[0];
#pragma unroll
    for (int i = 1; i < NC; ++i) Emax = fmax(Emax, E[i]);
#pragma unroll
    for (int i = 0; i < NC; ++i) ec[i] = k_exp2(E[i] - Emax);
  }
  // (the sum starts from the first term: a literal 0 + Sp_0 is an addition the
  // compiler must keep, for the sign of a zero)
#pragma unroll
  for (int i = 0; i < NC; ++i) Sp[i] = ec[i] * V[i];
  sum = Sp[0];
#pragma unroll
  for (int i = 1; i < NC; ++i) sum += Sp[i];
}

// FIRST: the event starts the sums (each acc[k] is set, not added to).
template <class S, class T, bool W, bool FIRST = false>
__device__ __forceinline__ void event(const T (&x)[S::ndim], T w, const T (&c)[S::ncst],
                                      const T (&xref)[S::ndim], T (&acc)[S::K]) {
  constexpr int NC = S::ncomp;
  T E[NC], V[NC], mom[S::K];
  T pv[NC][kMaxFacPerComp];
  components<S, T>(x, c, xref, E, V, mom, pv);
  T ec[NC], Emax, Sp[NC], sum;
  combine<NC, T>(E, V, ec, Emax, Sp, sum);
  const T l2 = Emax + k_log2(sum);  // log2 P
  const T inv = k_rcp(sum);
  const auto add = [&](int k, T v) {
    if constexpr (FIRST)
      acc[k] = v;
    else
      acc[k] += v;
  };
  const auto add_prod = [&](int k, T a, T b) {
    if constexpr (FIRST)
      acc[k] = a * b;
    else
      acc[k] = fma(a, b, acc[k]);
  };
  add(0, W ? w * l2 : l2);
  sfor<NC>([&](auto Ic) {
    constexpr int ci = Ic;
    using Cc = typename S::template comp<ci>;
    constexpr int mb = S::mom_base(ci);
    const T r = Sp[ci] * inv;
    const T wr = W ? w * r : r;
    add(mb, wr);
    const T wq = (W ? w * ec[ci] : ec[ci]) * inv;  // r_c / V_c
    sfor<Cc::nfac>([&](auto If) {
      constexpr int fi = If;
      using Fc = typename Cc::template fac<fi>;
      constexpr int o = mb + Cc::mom_off(fi);
      if constexpr (Fc::expo) {
#pragma unroll
        for (int k = 0; k < Fc::nmom; ++k) add_prod(o + k, wr, mom[o + k]);
      } else {
        T q = wq;  // r_c / v_f = wq * prod of the component's other polynomial factors
        sfor<Cc::nfac>([&](auto Ig) {
          constexpr int gi = Ig;
          using Gc = typename Cc::template fac<gi>;
          if constexpr (gi != fi && !Gc::expo) q *= pv[ci][gi];
        });
#pragma unroll
        for (int k = 0; k < Fc::nmom; ++k) add_prod(o + k, q, mom[o + k]);
      }
    });
  });
}

// ---------------------------------------------------------------------------
// one tile
// ---------------------------------------------------------------------------

template <class T, int VW>
struct Vec;
template <>
struct Vec<float, 4> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec<double, 2> {
  typedef double type __attribute__((ext_vector_type(2)));
};

// Event columns live in device global memory: loads through global-space
// pointers compile to global (not flat) vector loads.
template <class T>
__device__ __forceinline__ T load_global(const T* p) {
  return *(__attribute__((address_space(1))) const T*)(p);
}

template <class T, int VW>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&out)[VW]) {
  using V = typename Vec<T, VW>::type;
  const V v = load_global(reinterpret_cast<const V*>(p));
#pragma unroll
  for (int q = 0; q < VW; ++q) out[q] = v[q];
}

// The first group of a full tile's events (VW per thread), loaded ahead of
// the constant check so that the two latencies overlap.
template <class S, class P>
struct FirstGroup {
  typename P::T x[P::VW][S::ndim];
  typename P::T w[P::VW];
};

template <class S, class P>
__device__ __forceinline__ void load_first_group(const Job& J, int64_t base, FirstGroup<S, P>& f) {
  using T = typename P::T;
  constexpr int VW = P::VW;
  const int64_t e0 = base + int64_t(VW) * threadIdx.x;
#pragma unroll
  for (int d = 0; d < S::ndim; ++d) {
    T tmp[VW];
    load_vec<T, VW>(static_cast<const T*>(J.col[d]) + e0, tmp);
#pragma unroll
    for (int q = 0; q < VW; ++q) f.x[q][d] = tmp[q];
  }
  if (J.w) load_vec<T, VW>(static_cast<const T*>(J.w) + e0, f.w);
}

// The lane's moment sums are FP64.  FP64: in registers (acc).  Mixed
// precision: each group of VW events is summed in FP32 and then added to the
// lane's FP64 sums, which sit in LDS (lds[k * stride], this lane's column of
// the pass-1 buffer; an LDS FP64 add that returns nothing, so they take no
// registers).  An FP32 running sum over many events would drop the events
// whose terms are below half its last place, and responsibilities span many
// orders of magnitude, so those dropped terms would all have the same sign (a
// bias that grows with N).
template <class S, class P, bool W, bool FULL>
__device__ __forceinline__ void process_tile(const Job& J, int64_t base,
                                             const typename P::T (&c)[S::ncst],
                                             const typename P::T (&xref)[S::ndim],
                                             double (&acc)[kF32<typename P::T> ? 1 : S::K], double* lds,
                                             int stride,
                                             const FirstGroup<S, P>& first) {
  using T = typename P::T;
  constexpr int VW = P::VW;
  const int groups = J.events_per_thread / VW;
  const int64_t n = J.n;
  const T* __restrict__ col[S::ndim];
#pragma unroll
  for (int d = 0; d < S::ndim; ++d) col[d] = static_cast<const T*>(J.col[d]);
  const T* __restrict__ wcol = static_cast<const T*>(J.w);
  for (int g = 0; g < groups; ++g) {
    const int64_t e0 = base + int64_t(g) * (VW * kBlock) + int64_t(VW) * threadIdx.x;
    T xv[VW][S::ndim];
    T wv[VW];
    if constexpr (FULL) {
      if (g == 0) {
#pragma unroll
        for (int q = 0; q < VW; ++q) {
#pragma unroll
          for (int d = 0; d < S::ndim; ++d) xv[q][d] = first.x[q][d];
          if constexpr (W) wv[q] = first.w[q];
        }
      } else {
#pragma unroll
        for (int d = 0; d < S::ndim; ++d) {
          T tmp[VW];
          load_vec<T, VW>(col[d] + e0, tmp);
#pragma unroll
          for (int q = 0; q < VW; ++q) xv[q][d] = tmp[q];
        }
        if constexpr (W) load_vec<T, VW>(wcol + e0, wv);
      }
    } else {
#pragma unroll
      for (int q = 0; q < VW; ++q) {
        const bool ok = e0 + q < n;
#pragma unroll
        for (int d = 0; d < S::ndim; ++d) xv[q][d] = ok ? load_global(col[d] + e0 + q) : T(0);
        if constexpr (W) wv[q] = ok ? load_global(wcol + e0 + q) : T(0);
      }
    }
    if constexpr (kF32<T>) {
      T a32[S::K];
      if constexpr (FULL) {  // the group's first event starts its sums
        event<S, T, W, true>(xv[0], W ? wv[0] : T(1), c, xref, a32);
#pragma unroll
        for (int q = 1; q < VW; ++q) event<S, T, W>(xv[q], W ? wv[q] : T(1), c, xref, a32);
      } else {
#pragma unroll
        for (int k = 0; k < S::K; ++k) a32[k] = T(0);
#pragma unroll
        for (int q = 0; q < VW; ++q) {
          if (e0 + q < n) event<S, T, W>(xv[q], W ? wv[q] : T(1), c, xref, a32);
        }
      }
      if (g == 0) {
#pragma unroll
        for (int k = 0; k < S::K; ++k) lds[k * stride] = double(a32[k]);
      } else {
#pragma unroll
        for (int k = 0; k < S::K; ++k)
          __hip_atomic_fetch_add(lds + k * stride, double(a32[k]), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    } else {
#pragma unroll
      for (int q = 0; q < VW; ++q) {
        if (FULL || e0 + q < n) event<S, T, W>(xv[q], W ? wv[q] : T(1), c, xref, acc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// prologue and epilogue (FP64, one lane)
// ---------------------------------------------------------------------------

// NLL and gradient from the K moment sums: the chain rule through the
// mixture reduces to d NLL / d theta_p = -sum over p's terms of
// e[ec] * M[mom] (EpiTerm), one thread per free parameter.
template <class PV, class CV>
__device__ __forceinline__ void epilogue(const PV& P, const CV* cb, const double* __restrict__ tot,
                                         double* __restrict__ out) {
  const int tid = threadIdx.x;
  const double nll = -0.69314718055994530942 * tot[0];  // slot 0 holds sum w log2 P
  const bool bad = !cb->domain_ok || !isfinite(nll);
  if (tid == 0) out[0] = bad ? INFINITY : nll;
  if (tid < P.nfree) {
    const int p = P.free_idx[tid];
    double g = 0.0;
    for (int t = P.term_begin[p]; t < P.term_begin[p + 1]; ++t)
      g -= cb->e[P.term[t].ec] * tot[P.term[t].mom];
    out[1 + tid] = bad ? 0.0 : g;
  }
}

// What the epilogue reads of the plan and of the point's constants, in one
// small block (LDS of the collecting workgroup).
struct EpiView {
  int nfree, domain_ok;
  int free_idx[UML_MAX_PARAMS];
  int term_begin[UML_MAX_PARAMS + 1];
  EpiTerm term[kMaxTerms];
  double e[kMaxECst];
};

// Bulk copy of n bytes (a multiple of 16, both 16-byte aligned) by
// `threads` threads, this one being number `t`: every load is issued before
// any is waited for.
__device__ __forceinline__ void bulk_copy16(void* dst, const void* src, int nbytes, int t = threadIdx.x,
                                            int threads = kBlock) {
  const int4* s4 = static_cast<const int4*>(src);
  int4* d4 = static_cast<int4*>(dst);
  const int n = nbytes / 16;
  for (int i = t; i < n; i += threads) d4[i] = s4[i];
}

// Threads per column of column_sums, and the threads it occupies.
template <int K>
__host__ __device__ constexpr int column_q() {
  int q = 1;
  while (q * 2 * K <= kBlock && q * 2 <= 16) q *= 2;
  return q;
}

// Fixed-order sums of column k (columns col_stride apart) over `count`
// entries spaced `step` apart, split over Q threads per column (thread (k, j)
// takes entries j, j+Q, ..),
// then combined in j order through LDS.  Entries are read device-coherently:
// they were written by other workgroups of this launch.  Every thread of the
// workgroup must call this; out[k] receives the column sums.
template <int K>
__device__ __forceinline__ void column_sums(double* base, int col_stride, int count, int step,
                                            double* lds, double* out) {
  constexpr int Q = column_q<K>();
  const int tid = threadIdx.x;
  if (tid < K * Q) {
    const int k = tid / Q, j = tid % Q;
    double* col = base + int64_t(k) * col_stride;
    double s = 0.0, comp = 0.0;
    int m = j;
    for (; m + 7 * Q < count; m += 8 * Q) {  // eight loads in flight
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        x[u] = __hip_atomic_load(col + int64_t(m + u * Q) * step, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int u = 0; u < 8; ++u) {  // Neumaier, in entry order
        const double t = s + x[u];
        comp += fabs(s) >= fabs(x[u]) ? (s - t) + x[u] : (x[u] - t) + s;
        s = t;
      }
    }
    for (; m < count; m += Q) {
      const double xv =
          __hip_atomic_load(col + int64_t(m) * step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double t = s + xv;
      comp += fabs(s) >= fabs(xv) ? (s - t) + xv : (xv - t) + s;
      s = t;
    }
    lds[k * Q + j] = s + comp;
  }
  __syncthreads();
  if (tid < K) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) s += lds[tid * Q + j];
    out[tid] = s;
  }
  __syncthreads();
}

// Copies of wave-invariant values in scalar registers.
__device__ __forceinline__ float to_sgpr(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double to_sgpr(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(b & 0xffffffffu));
  const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(b >> 32));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// ---------------------------------------------------------------------------
// device-resident BFGS (one step per evaluation)
// ---------------------------------------------------------------------------

// One step of the quasi-Newton minimisation (the Broyden-Fletcher-Goldfarb-
// Shanno variant of the variable-metric method Migrad uses, Sec. 2.1) for the
// fit whose trial point this workgroup just evaluated (fs->out).  FP64; thread
// i < n owns row i of the metric V.  Line search: backtracking from a unit
// step with the Armijo condition; a rise of the NLL below the rounding level
// tol_f_rel |f| is accepted when the slope along p has not turned up (strong
// Wolfe curvature), so mixed-precision rounding cannot stall the search.
// Stops when EDM = 0.5 g^T V g < edm_tol.  Writes the next trial point and
// its constants (the next launch's cache) unless the fit is finished.
__device__ __noinline__ void bfgs_step(const Plan& P, FitState* fs, ConstBlock* cst, ConstBlock* s_cbuf) {
  __shared__ double sv[4][UML_MAX_PARAMS];  // s, y, V y, new gradient
  __shared__ double s_th[UML_MAX_PARAMS];    // the next trial point
  __shared__ double sc[4];
  __shared__ int act, fin;
  const int tid = threadIdx.x, nf = P.nfree;
  if (tid == 0) {
    const double ft = fs->out[0];
    fs->n_eval++;
    int a;
    if (fs->phase == 0) {
      a = isfinite(ft) ? 0 : 3;
    } else {
      const double f = fs->f, gp = fs->gp, al = fs->alpha;
      bool ok = isfinite(ft) && ft <= f + 1e-4 * al * gp + fs->tol_f_rel * fabs(f);
      if (ok && ft > f + 1e-4 * al * gp) {  // accepted on the rounding tolerance only
        double gtp = 0.0;
        for (int k = 0; k < nf; ++k) gtp += fs->out[1 + k] * fs->p[k];
        ok = fabs(gtp) <= 0.9 * fabs(gp);
      }
      a = ok ? 1 : 2;
    }
    act = a;
    fin = 0;
  }
  __syncthreads();
  const int a = act;
  if (a == 3) {  // the start point has P <= 0 somewhere
    if (tid == 0) {
      fs->status = UML_FIT_PDF_NONPOSITIVE;
      fs->done = 1;
    }
    return;
  }
  if (a == 1) {  // accept x + alpha p, update the metric
    if (tid < nf) {
      const double sk = fs->alpha * fs->p[tid];
      sv[0][tid] = sk;
      sv[1][tid] = fs->out[1 + tid] - fs->g[tid];
      sv[3][tid] = fs->out[1 + tid];
    }
    __syncthreads();
    if (tid < nf) {
      double vy = 0.0;
      for (int j = 0; j < nf; ++j) vy += fs->V[tid * UML_MAX_PARAMS + j] * sv[1][j];
      sv[2][tid] = vy;
    }
    __syncthreads();
    if (tid == 0) {
      double sy = 0.0, yvy = 0.0;
      for (int k = 0; k < nf; ++k) {
        sy += sv[0][k] * sv[1][k];
        yvy += sv[1][k] * sv[2][k];
      }
      sc[0] = sy;
      sc[1] = yvy;
    }
    __syncthreads();
    const double sy = sc[0], yvy = sc[1];
    if (tid < nf) {
      if (sy > 0.0 && isfinite(sy) && isfinite(yvy)) {
        const double c1 = (sy + yvy) / (sy * sy);
        for (int j = 0; j < nf; ++j)
          fs->V[tid * UML_MAX_PARAMS + j] +=
              c1 * sv[0][tid] * sv[0][j] - (sv[2][tid] * sv[0][j] + sv[0][tid] * sv[2][j]) / sy;
      }
      fs->x[tid] += sv[0][tid];
      fs->g[tid] = sv[3][tid];
    }
    if (tid == 0) {
      fs->f = fs->out[0];
      fs->n_iter++;
      fs->n_ls = 0;
    }
    __syncthreads();
  } else if (a == 0) {  // the start point
    if (tid < nf) {
      fs->x[tid] = fs->theta[P.free_idx[tid]];
      fs->g[tid] = fs->out[1 + tid];
    }
    if (tid == 0) fs->f = fs->out[0];
    __syncthreads();
  }
  if (a == 0 || a == 1) {  // new direction p = -V g
    for (int attempt = 0; attempt < 2; ++attempt) {
      if (tid < nf) {
        double pk = 0.0;
        for (int j = 0; j < nf; ++j) pk -= fs->V[tid * UML_MAX_PARAMS + j] * fs->g[j];
        fs->p[tid] = pk;
      }
      __syncthreads();
      if (tid == 0) {
        double gp = 0.0;
        for (int k = 0; k < nf; ++k) gp += fs->g[k] * fs->p[k];
        sc[2] = gp;
      }
      __syncthreads();
      if (sc[2] < 0.0 || nf == 0) break;
      if (tid < nf)  // the metric lost positivity: restart from the start metric
        for (int j = 0; j < nf; ++j) fs->V[tid * UML_MAX_PARAMS + j] = fs->V0[tid * UML_MAX_PARAMS + j];
      __syncthreads();
    }
    if (tid == 0) {
      const double gp = sc[2];
      fs->gp = gp;
      fs->edm = -0.5 * gp;
      fs->alpha = 1.0;
      fs->phase = 1;
      if (nf == 0 || fs->edm < fs->edm_tol) {
        fs->status = UML_FIT_CONVERGED;
        fin = 1;
      } else if (!(gp < 0.0)) {
        fs->status = UML_FIT_HESSIAN_NOT_PD;
        fin = 1;
      } else if (fs->n_iter >= fs->max_iter) {
        fs->status = UML_FIT_MAX_ITER;
        fin = 1;
      }
    }
  } else if (tid == 0) {  // a == 2: shorten the step
    const double ft = fs->out[0], f = fs->f, gp = fs->gp, al = fs->alpha;
    double an;
    if (!isfinite(ft)) {
      an = 0.25 * al;
    } else {
      const double q = -gp * al * al / (2.0 * (ft - f - gp * al));
      an = fmin(fmax(q, 0.1 * al), 0.5 * al);
    }
    fs->alpha = an;
    fs->n_ls++;
    if (fs->n_ls > 60 || an < 1e-12) {
      fs->status = fs->edm < 100.0 * fs->edm_tol ? UML_FIT_CONVERGED : UML_FIT_LINESEARCH_FAIL;
      fin = 1;
    }
  }
  __syncthreads();
  if (fin) {
    if (tid < nf) fs->theta[P.free_idx[tid]] = fs->x[tid];
    __syncthreads();
    if (tid == 0) fs->done = 1;
    return;
  }
  if (tid < nf) fs->theta[P.free_idx[tid]] = fs->x[tid] + fs->alpha * fs->p[tid];
  __syncthreads();
  if (tid < P.npar) s_th[tid] = fs->theta[tid];
  __syncthreads();
  compute_constants(lds(&P), lds(s_th), lds(s_cbuf));  // the next launch's cache, built in LDS
  __syncthreads();
  store_const_block(cst, *s_cbuf);
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------

// One workgroup's arrival at a completion counter shared by `members`
// workgroups of this launch; true for the workgroup that completes the count.
// Called by one thread after a workgroup barrier that follows the workgroup's
// partial stores.  Memory model (HIP's scoped model, agent scope):
//   * the increment is an agent-scope release: every store that happens
//     before it (the partials, ordered before it by the barrier) is visible to
//     any agent-scope acquire that reads the incremented value or a later one;
//   * the workgroup that completes the count reads the last value of the
//     counter's release sequence, and its agent-scope acquire fence makes the
//     partials of every member visible to its later loads; the workgroup
//     barrier after this call extends that to its other threads;
//   * the completing workgroup resets the counter for the next launch, which
//     is ordered after this one by the end of the kernel.
// On gfx950 the release writes back this XCD's L2 and waits for the
// workgroup's stores, the acquire invalidates the L2's non-coherent lines.
__device__ __forceinline__ bool arrive(unsigned* cnt, unsigned members) {
  const unsigned p = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  const bool last = p + 1u == members;
  if (last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return last;
}

// Rounds a collecting workgroup waits for one tile's partials before it gives
// up (each round is at least one memory round trip: seconds in all).
constexpr int kSpinLimit = 1 << 22;
#ifndef UML_POLL_BATCH
#define UML_POLL_BATCH 1
#endif
// Tiles a collecting thread polls at once.
constexpr int kPollBatch = UML_POLL_BATCH;

template <int K>
__host__ __device__ constexpr int reduce_parts() {
  int p = 1;
  while (p * 2 * K <= kBlock && p * 2 <= 32) p *= 2;
  return p;
}

// A point that misses the cache: the plan and theta go to LDS (buf, at least
// sizeof(Plan) + UML_MAX_PARAMS doubles; both reads in flight together), then
// the workgroup runs the prologue into cb.  Ends with a workgroup barrier.
__device__ __forceinline__ void miss_prologue(const Plan* __restrict__ plan, const double* __restrict__ th,
                                           int npar, void* buf, ConstBlock* cb) {
  Plan* s_plan = static_cast<Plan*>(buf);
  double* s_th = reinterpret_cast<double*>(static_cast<char*>(buf) + sizeof(Plan));
  bulk_copy16(s_plan, plan, int(sizeof(Plan)));
  if (int(threadIdx.x) < npar) s_th[threadIdx.x] = th[threadIdx.x];
  __syncthreads();
  compute_constants(lds(s_plan), lds(s_th), lds(cb));
  __syncthreads();
}

// Waves per SIMD the kernel is built for.  The mixed-precision kernels keep
// four (at most 128 VGPRs): their FP32 event loops need that latency hiding,
// and the largest of them sits right at the limit.  The FP64 kernels and those
// reading precomputed terms hold more per event and are left unconstrained.
template <class S, class P>
__host__ __device__ constexpr int eval_min_waves() {
  return (P::VW == 4 && !S::pre) ? 4 : 1;
}

// Two kernels per model shape and precision:
//   BATCH = false  one dataset (job j0, tile = workgroup) at the point
//                  theta0, with the job's cached constant block cst0, plan
//                  plan0, model key key0 and parameter count npar0.  These
//                  lead the argument list; the hardware preloads the five
//                  into scalar registers (the library is built that way), so
//                  the loads of the cache check, the check itself and a
//                  missing point's prologue go ahead without waiting for the
//                  rest of the arguments, and the job's fields stay in
//                  scalar registers.
//   BATCH = true   a ragged launch over many jobs (tile map: workgroup ->
//                  (job, tile)), each workgroup taking its job's point, block
//                  and count from the job array; jobs in fit mode take their
//                  BFGS step in the workgroup that completes them.
// Keeping the two apart keeps the BFGS step's registers out of the plain
// evaluation and lets its job descriptor come from the kernel arguments
// alone.
template <class S, class P, bool BATCH>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(eval_min_waves<S, P>()))) void eval_kernel(const double* __restrict__ theta0,
                                                      const ConstBlock* __restrict__ cst0,
                                                      const Plan* __restrict__ plan0, long long key0, int npar0,
                                                      const int2* __restrict__ tmap,
                                                      const Job* __restrict__ jobs,
                                                      double* __restrict__ out_override, const Job j0) {
  using T = typename P::T;
  constexpr int K = S::K;
  const int tid = threadIdx.x, lane = tid & 63;
  int jid = 0, tile = blockIdx.x;
  const double* __restrict__ th = theta0;
  const ConstBlock* __restrict__ gc = cst0;
  int npar = npar0;
  if constexpr (BATCH) {
    const int2 t = tmap[blockIdx.x];
    jid = t.x;
    tile = t.y;
    if (jid < 0) return;
    th = jobs[jid].theta;
    gc = jobs[jid].cst;
    npar = jobs[jid].npar;
  }
  // the cache check's loads, issued before the fit's done flag is known and
  // unconditionally (lanes past the parameter count re-read parameter 0, and
  // every model has at least one), so nothing waits for them until the check
  const int pl = lane < npar ? lane : 0;
  const double th_l = th[pl], gc_l = gc->theta[pl];
  const Job J = BATCH ? jobs[jid] : j0;
  if constexpr (BATCH)
    if (J.fit && J.fit->done) return;  // a finished fit: its tiles do nothing
  const Plan* __restrict__ plan = BATCH ? J.plan : plan0;
  const long long key = BATCH ? J.key : key0;
  // single dataset: the launch count, which picks this launch's partial slots
  unsigned long long epoch = 0;
  if constexpr (!BATCH) epoch = __hip_atomic_load(J.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __shared__ __align__(16) ConstBlock s_cb;

  // Parameter-only constants.  The job keeps the block of the last point it
  // evaluated: when theta matches it bit for bit its constants are used
  // (scalar loads, issued together with the comparison); otherwise the
  // workgroup computes them here in FP64 (the prologue: normalisations,
  // combined prefactors, angular coefficients).
  const int64_t tsize = int64_t(J.events_per_thread) * kBlock;
  const int64_t base = int64_t(tile) * tsize;
  const bool full = base + tsize <= J.n;
  FirstGroup<S, P> first;
  if (full) load_first_group<S, P>(J, base, first);

  // LDS: the pass-1 transpose buffer (also holds the plan while constants
  // are computed, and the pass-2 sums and plan), and the pass-2 partials
  constexpr int STRIDE = kBlock + 8;
  constexpr int PARTS = reduce_parts<K>();
  constexpr int CH = kBlock / PARTS;
  // T-sized transpose buffer, reused afterwards for K + UML_MAX_PARAMS
  // doubles followed by the plan
  constexpr int PASS2_BYTES =
      (K + UML_MAX_PARAMS) * sizeof(double) + sizeof(Plan) + sizeof(ConstBlock) + 16;
  constexpr int LDS_T = (K * STRIDE * sizeof(double) > PASS2_BYTES) ? K * STRIDE
                                                                    : int(PASS2_BYTES / sizeof(double)) + 4;
  __shared__ __align__(16) double red[LDS_T];
  __shared__ double red2[K * (PARTS > 16 ? PARTS : 16)];
  __shared__ int s_flag;

  T c[S::ncst];
#pragma unroll
  for (int i = 0; i < S::ncst; ++i) c[i] = P::consts(gc)[i];
  T xref[S::ndim];  // only shifted dimensions (all below UML_MAX_DIMS) have one
#pragma unroll
  for (int d = 0; d < S::ndim; ++d) xref[d] = ((S::shift_mask >> d) & 1u) ? P::xrefs(gc)[d] : T(0);
  const bool eq = lane >= npar || __double_as_longlong(th_l) == __double_as_longlong(gc_l);
  const bool hit = __all(eq) && gc->valid && gc->key == key;  // the same in every wave
  if (!hit) {
    miss_prologue(plan, th, npar, red, &s_cb);
#pragma unroll
    for (int i = 0; i < S::ncst; ++i) c[i] = to_sgpr(P::consts(&s_cb)[i]);
#pragma unroll
    for (int d = 0; d < S::ndim; ++d)
      xref[d] = ((S::shift_mask >> d) & 1u) ? to_sgpr(P::xrefs(&s_cb)[d]) : T(0);
  }

  double acc[kF32<T> ? 1 : K];  // FP64: the lane sums; mixed: in LDS (red)
#pragma unroll
  for (int k = 0; k < (kF32<T> ? 1 : K); ++k) acc[k] = 0.0;
  double* lsum = red + tid;
  if (J.w) {
    if (full)
      process_tile<S, P, true, true>(J, base, c, xref, acc, lsum, STRIDE, first);
    else
      process_tile<S, P, true, false>(J, base, c, xref, acc, lsum, STRIDE, first);
  } else {
    if (full)
      process_tile<S, P, false, true>(J, base, c, xref, acc, lsum, STRIDE, first);
    else
      process_tile<S, P, false, false>(J, base, c, xref, acc, lsum, STRIDE, first);
  }

  // pass 1: lanes -> tile partial, through LDS in a fixed order (buffers
  // declared above)
  if constexpr (!kF32<T>) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * STRIDE + tid] = acc[k];
  }
  __syncthreads();
  if (tid < K * PARTS) {
    const int k = tid / PARTS, p = tid % PARTS;
    double s = 0.0;
#pragma unroll 8
    for (int i = 0; i < CH; ++i) s += red[k * STRIDE + i * PARTS + p];
    red2[k * PARTS + p] = s;
  }
  __syncthreads();
  const int nt = J.n_tiles;
  double* tot = reinterpret_cast<double*>(red);
  // The epilogue's plan and cached constants live in the pass-1 buffer, after
  // the K + UML_MAX_PARAMS moment sums (16-byte aligned).
  Plan* s_plan = reinterpret_cast<Plan*>(tot + ((K + UML_MAX_PARAMS + 1) & ~1));
  ConstBlock* s_gc = reinterpret_cast<ConstBlock*>(reinterpret_cast<char*>(s_plan) + sizeof(Plan));
  if constexpr (!BATCH) {
    // Single dataset: each tile writes its K partials, every one an FP64
    // value that replaces the sentinel (kSentinel) left in its slot, and is
    // done; workgroup 0 then collects them.  A slot is read until it holds a
    // value (agent-scope atomic loads and stores of naturally aligned 64-bit
    // words: each read returns either the sentinel or the whole value), so
    // no counter, no ordering between the slots and no cache write-back is
    // needed.  Two buffers of slots alternate between launches (the launch
    // count, J.epoch, picks one): the collector first refills the other
    // buffer with sentinels for the next launch, so those stores overlap its
    // wait, and the end of this kernel orders them before the next launch.
    const int64_t kn = int64_t(K) * nt;
    double* __restrict__ sp = J.spart + (epoch & 1ull) * kn;  // [K][nt]
    if (tid < K) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < PARTS; ++p) s += red2[tid * PARTS + p];
      __hip_atomic_store(sp + int64_t(tid) * nt + tile, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tile != 0) return;
    {
      double* nxt = J.spart + ((epoch + 1ull) & 1ull) * kn;
      const double sentinel = __longlong_as_double(static_cast<long long>(kSentinel));
      for (int64_t i = tid; i < kn; i += kBlock)
        __hip_atomic_store(nxt + i, sentinel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the epilogue's share of the plan and of the constants, read while the
    // partials are polled
    __shared__ EpiView s_epi;
    {
      const Plan* __restrict__ gp = plan;
      const ConstBlock* cbs = hit ? gc : &s_cb;
      if (tid < UML_MAX_PARAMS) s_epi.free_idx[tid] = gp->free_idx[tid];
      if (tid <= UML_MAX_PARAMS) s_epi.term_begin[tid] = gp->term_begin[tid];
      if (tid < kMaxTerms) s_epi.term[tid] = gp->term[tid];
      if (tid < kMaxECst) s_epi.e[tid] = cbs->e[tid];
      if (tid == 0) {
        s_epi.nfree = gp->nfree;
        s_epi.domain_ok = cbs->domain_ok;
      }
    }
    // thread t sums the tiles t, t + 256, .. in order (Neumaier), polling PB
    // of them at a time; a wait that exceeds kSpinLimit rounds (seconds)
    // gives up and the result is NaN
    constexpr int PB = kPollBatch;
    double sum[K], cmp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) sum[k] = cmp[k] = 0.0;
    bool lost = false;
    for (int t0 = tid; t0 < nt; t0 += PB * kBlock) {
      double v[PB][K];
      for (int spin = 0;; ++spin) {
        bool ready = true;
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          const int t = t0 + b * kBlock;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            // moment k of tile t at sp[k * nt + t]: a wave's loads are contiguous
            v[b][k] = t < nt ? __hip_atomic_load(sp + int64_t(k) * nt + t, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                             : 0.0;
            ready = ready && static_cast<unsigned long long>(__double_as_longlong(v[b][k])) != kSentinel;
          }
        }
        if (ready) break;
        if (spin >= kSpinLimit) {
          lost = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        if (t0 + b * kBlock < nt) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const double x = v[b][k], u = sum[k] + x;
            cmp[k] += fabs(sum[k]) >= fabs(x) ? (sum[k] - u) + x : (x - u) + sum[k];
            sum[k] = u;
          }
        }
      }
    }
    // the 256 thread sums of each moment through LDS in the fixed order of
    // pass 1
#pragma unroll
    for (int k = 0; k < K; ++k) red[k * STRIDE + tid] = sum[k] + cmp[k];
    const bool any_lost = __syncthreads_or(lost ? 1 : 0) != 0;
    if (tid < K * PARTS) {
      const int k = tid / PARTS, p = tid % PARTS;
      double x = 0.0;
#pragma unroll 8
      for (int i = 0; i < CH; ++i) x += red[k * STRIDE + i * PARTS + p];
      red2[k * PARTS + p] = x;
    }
    __syncthreads();
    if (tid < K) {
      double x = 0.0;
#pragma unroll
      for (int p = 0; p < PARTS; ++p) x += red2[tid * PARTS + p];
      tot[tid] = any_lost ? NAN : x;
    }
    if (tid == 0) __hip_atomic_store(J.epoch, epoch + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the new point's constants, for the cache: written only now that every
    // tile has passed its own cache check (a workgroup that started later
    // could otherwise match the new point against a partly written block)
    if (!hit) bulk_copy16(J.cst, &s_cb, int(sizeof(ConstBlock)));
    __syncthreads();
    epilogue(s_epi, &s_epi, tot, out_override ? out_override : J.out);
  } else {
    double* gpart = J.partials + int64_t(K) * nt;  // [K][kGroups]
    // With at most kGroups tiles each tile is its own group: its partial goes
    // straight to the group partials and the group level is skipped.
    const bool single = nt <= kGroups;
    if (tid < K) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < PARTS; ++p) s += red2[tid * PARTS + p];
      // device-coherent store: written through to the point where every XCD's
      // loads of the same address meet, so no L2 write-back is needed
      double* dst = single ? gpart + int64_t(tid) * kGroups + tile : J.partials + int64_t(tid) * nt + tile;
      __hip_atomic_store(dst, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // Completion, in two levels (see kGroups), each a release/acquire counter
    // step (arrive) after a barrier that orders this workgroup's stores.
    const int ng = nt < kGroups ? nt : kGroups;
    const int g = tile % ng;
    __syncthreads();
    if (!single) {
      if (tid == 0)
        s_flag = arrive(J.counter + g * kCounterStride, unsigned((nt - 1 - g) / ng + 1)) ? 1 : 0;
      __syncthreads();
      if (!s_flag) return;
      // the last tile of group g sums the group's tiles g, g + ng, .. in order
      {
        const int members = (nt - 1 - g) / ng + 1;
        column_sums<K>(J.partials + g, nt, members, ng, red2, tot);
      }
      if (tid < K)
        __hip_atomic_store(gpart + int64_t(tid) * kGroups + g, tot[tid], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
    }
    if (tid == 0) s_flag = arrive(J.counter + kGroups * kCounterStride, unsigned(ng)) ? 1 : 0;
    __syncthreads();
    if (!s_flag) return;
    // The last group: the sum over groups, the plan and the constants.  The
    // threads the column sums leave idle fetch the plan (and the cached
    // constants) meanwhile, so the three reads cost one round trip.
    constexpr int QS = K * column_q<K>();
    constexpr bool spare = kBlock - QS >= 64;
    if (spare ? tid >= QS : true) {
      const int t = spare ? tid - QS : tid, nt2 = spare ? kBlock - QS : kBlock;
      bulk_copy16(s_plan, J.plan, int(sizeof(Plan)), t, nt2);
      if (hit) bulk_copy16(s_gc, gc, int(sizeof(ConstBlock)), t, nt2);
    }
    if (!hit) bulk_copy16(J.cst, &s_cb, int(sizeof(ConstBlock)));
    if (!spare) __syncthreads();
    column_sums<K>(gpart, kGroups, ng, 1, red2, tot);  // ends with a barrier
    epilogue(*s_plan, hit ? s_gc : &s_cb, tot, J.out);
    if (J.fit) {
      __syncthreads();
      bfgs_step(*s_plan, J.fit, J.cst, s_gc);  // s_gc is free once the epilogue is done
    }
  }
}

// The events of one tile per workgroup at which P <= 0 or P is not finite
// (outside the domain of Eq. 1's logarithm), added to *count; every event
// counts when the point is outside the model's domain.  The same per-event
// arithmetic as eval_kernel, so it counts exactly the events that make an
// evaluation +inf.  Not on the evaluation path: the library runs it only
// after an evaluation returned +inf.
template <class S, class P>
__global__ __launch_bounds__(kBlock) void count_kernel(const double* __restrict__ th, const Job J,
                                                       unsigned long long* __restrict__ count) {
  using T = typename P::T;
  constexpr int NC = S::ncomp;
  __shared__ __align__(16) char buf[sizeof(Plan) + UML_MAX_PARAMS * sizeof(double)];
  __shared__ __align__(16) ConstBlock s_cb;
  miss_prologue(J.plan, th, J.npar, buf, &s_cb);
  T c[S::ncst], xref[S::ndim];
#pragma unroll
  for (int i = 0; i < S::ncst; ++i) c[i] = P::consts(&s_cb)[i];
#pragma unroll
  for (int d = 0; d < S::ndim; ++d) xref[d] = ((S::shift_mask >> d) & 1u) ? P::xrefs(&s_cb)[d] : T(0);
  const bool dom = s_cb.domain_ok != 0;
  const int64_t tsize = int64_t(J.events_per_thread) * kBlock;
  const int64_t base = int64_t(blockIdx.x) * tsize;
  const int64_t end = base + tsize < J.n ? base + tsize : J.n;
  unsigned long long bad = 0;
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    if (!dom) {
      ++bad;
      continue;
    }
    T x[S::ndim];
#pragma unroll
    for (int d = 0; d < S::ndim; ++d) x[d] = load_global(static_cast<const T*>(J.col[d]) + i);
    T E[NC], V[NC], mom[S::K], pv[NC][kMaxFacPerComp];
    components<S, T>(x, c, xref, E, V, mom, pv);
    T ec[NC], Emax, Sp[NC], sum;
    combine<NC, T>(E, V, ec, Emax, Sp, sum);
    const T l2 = Emax + k_log2(sum);
    if (!(sum > T(0)) || !isfinite(l2)) ++bad;
  }
  if (bad) atomicAdd(count, bad);
}

template <class S>
void launch_count(const LaunchArgs& a, unsigned long long* d_count) {
  if (a.precision == UML_MIXED)
    hipLaunchKernelGGL((count_kernel<S, PrecMixed>), dim3(a.grid), dim3(kBlock), 0, a.stream, a.theta, a.job0,
                       d_count);
  else
    hipLaunchKernelGGL((count_kernel<S, PrecF64>), dim3(a.grid), dim3(kBlock), 0, a.stream, a.theta, a.job0,
                       d_count);
}

template <class S>
void launch_eval(const LaunchArgs& a) {
  const double* th0 = a.theta ? a.theta : a.job0.theta;
  if (a.tmap) {
    if (a.precision == UML_MIXED)
      hipLaunchKernelGGL((eval_kernel<S, PrecMixed, true>), dim3(a.grid), dim3(kBlock), 0, a.stream, th0,
                         a.job0.cst, a.job0.plan, a.job0.key, a.job0.npar, a.tmap, a.jobs, a.out, a.job0);
    else
      hipLaunchKernelGGL((eval_kernel<S, PrecF64, true>), dim3(a.grid), dim3(kBlock), 0, a.stream, th0,
                         a.job0.cst, a.job0.plan, a.job0.key, a.job0.npar, a.tmap, a.jobs, a.out, a.job0);
  } else {
    if (a.precision == UML_MIXED)
      hipLaunchKernelGGL((eval_kernel<S, PrecMixed, false>), dim3(a.grid), dim3(kBlock), 0, a.stream, th0,
                         a.job0.cst, a.job0.plan, a.job0.key, a.job0.npar, a.tmap, a.jobs, a.out, a.job0);
    else
      hipLaunchKernelGGL((eval_kernel<S, PrecF64, false>), dim3(a.grid), dim3(kBlock), 0, a.stream, th0,
                         a.job0.cst, a.job0.plan, a.job0.key, a.job0.npar, a.tmap, a.jobs, a.out, a.job0);
  }
}

template <class S>
Family make_family() {
  return Family{S::sig(), S::K, S::ncst, &launch_eval<S>, nullptr, &launch_count<S>};
}

// The compiled catalogue of model shapes.  Components are ordered by their
// factor kinds, factors by (kind, dimension); dimensions are numbered
// Gaussian/exponential first, then the P-wave's own order, then the rest.
static const Family* families() {
  static const Family table[] = {
      make_family<Shape<Comp<Gauss<0>>>>(),                                  // Gauss
      make_family<Shape<Comp<Exp<0>>>>(),                                    // exponential
      make_family<Shape<Comp<Cheb<0, 1>>>>(),                                // Chebyshev
      make_family<Shape<Comp<Cheb<0, 2>>>>(),
      make_family<Shape<Comp<Cheb<0, 3>>>>(),
      make_family<Shape<Comp<Cheb<0, 4>>>>(),
      make_family<Shape<Comp<PWave<0, 1, 2>>>>(),                            // angular fit
      make_family<Shape<Comp<Exp<0>>, Comp<Gauss<0>>>>(),                    // mass fit
      make_family<Shape<Comp<Exp<0>>, Comp<Gauss<0>>, Comp<Gauss<0>>>>(),    // two peaks + background
      make_family<Shape<Comp<Cheb<0, 1>>, Comp<Exp<0>>, Comp<Gauss<0>>, Comp<Gauss<0>>>>(),
      make_family<Shape<Comp<Gauss<0>, PWave<1, 2, 3>>>>(),                  // 4-D signal
      make_family<Shape<Comp<Exp<0>, Cheb<1, 2>, Cheb<2, 2>, Cheb<3, 2>>,  // 4-D model
                        Comp<Gauss<0>, PWave<1, 2, 3>>>>(),
      // the same with the P-wave's event-only terms precomputed
      make_family<Shape<Comp<PWavePre<3>>>>(),
      make_family<Shape<Comp<Gauss<0>, PWavePre<4>>>>(),
      make_family<Shape<Comp<Exp<0>, Cheb<1, 2>, Cheb<2, 2>, Cheb<3, 2>>, Comp<Gauss<0>, PWavePre<4>>>>(),
      Family{"", 0, 0, nullptr, nullptr, nullptr},
  };
  return table;
}

// The stored P-wave terms of a dataset, one event per thread.
template <class T>
__global__ __launch_bounds__(kBlock) void pwave_terms_kernel(const PrecomputeArgs a) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const T cl = load_global(static_cast<const T*>(a.in[0]) + i);
  const T ck = load_global(static_cast<const T*>(a.in[1]) + i);
  const T ph = load_global(static_cast<const T*>(a.in[2]) + i);
  T u0, m[8];
  pwave_terms(cl, ck, ph, u0, m);
  static_cast<T*>(a.out[0])[i] = u0;
#pragma unroll
  for (int k = 0; k < 8; ++k) static_cast<T*>(a.out[1 + k])[i] = m[k];
}

__global__ __launch_bounds__(kBlock) void fill_sentinel_kernel(double* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = __longlong_as_double(static_cast<long long>(kSentinel));
}

void launch_fill_sentinel(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_sentinel_kernel, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, p, n);
}

void launch_pwave_terms(const PrecomputeArgs& a, int precision, hipStream_t s) {
  const unsigned blocks = unsigned((a.n + kBlock - 1) / kBlock);
  if (precision == UML_MIXED)
    hipLaunchKernelGGL(pwave_terms_kernel<float>, dim3(blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(pwave_terms_kernel<double>, dim3(blocks), dim3(kBlock), 0, s, a);
}

const Family* find_family(const std::string& sig) {
  for (const Family* f = families(); f->eval; ++f)
    if (f->sig == sig) return f;
  return nullptr;
}

std::string family_list() {
  std::string s;
  for (const Family* f = families(); f->eval; ++f) s += (s.empty() ? "" : ", ") + f->sig;
  return s;
}

}  // namespace uml
