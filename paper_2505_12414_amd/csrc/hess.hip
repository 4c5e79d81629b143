// Hessian of the NLL on gfx950: H = sum_i w_i (s_i s_i^T - d2P_i / P_i)
// (the second derivatives of Sec. 2.2, used for the covariance the HESSE
// step reports), together with the NLL, its gradient and, for weighted
// fits, W2 = sum_i w_i^2 s_i s_i^T (the middle of the sandwich covariance).
//
// With P = sum_c S_c, S_c = F_c prod_f p_f, responsibilities r_c = S_c / P
// and component log-derivatives l_c = d ln S_c / d theta:
//     s = sum_c r_c l_c,     d2P / P = sum_c r_c (d2 S_c / S_c),
// and (d2 S_c / S_c)_ab is l_ca l_cb when a and b belong to different units
// of the component (different factors, or a fraction and a factor), and the
// unit's own d2p/p when they belong to the same one (zero for a fraction and
// for the P-wave density, which are linear in their parameters).
//
// One workgroup per tile of events.  The tile is processed in chunks: each
// lane of the first wave evaluates one event by walking the plan and stages
// (w, log2 P, s, r, l, d2p/p) in LDS; then each thread owns a few of the
// M = 1 + nfree + 2 npairs sums and accumulates them in FP64 over the chunk in
// event order.  Tile sums go to [M][n_tiles]; a second kernel adds the tiles
// in tile order.  Every order is fixed: the results are reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "devmath.h"
#include "hess.h"
#include "prologue.h"
#include "uml_internal.h"

namespace uml {

// Second derivatives that the gradient does not need, for one factor: d2 ln D
// of the Gaussian normalisation D = Phi(zb) - Phi(za) in (mu, sigma), and
// -Var[x] of the truncated exponential (d2 ln p / d lambda^2).
static __device__ __forceinline__ void hess_factor_constants(const FactorPlan& F, const double* __restrict__ th,
                                                             double* h) {
  const double kInvSqrt2Pi = 0.39894228040143267794;
  h[0] = h[1] = h[2] = h[3] = 0.0;
  const double a = F.lo[0], b = F.hi[0];
  if (F.kind == FK_GAUSS) {
    const double mu = th[F.par[0]], sg = th[F.par[1]];
    const double za = (a - mu) / sg, zb = (b - mu) / sg;
    const double D = d_phi_diff(za, zb);
    const double pa = p_exp(-0.5 * za * za) * kInvSqrt2Pi, pb = p_exp(-0.5 * zb * zb) * kInvSqrt2Pi;
    const double s2 = sg * sg;
    const double Dm = (pa - pb) / sg, Ds = (za * pa - zb * pb) / sg;
    const double Dmm = (za * pa - zb * pb) / s2;
    const double Dms = (-(pa - pb) + za * za * pa - zb * zb * pb) / s2;
    const double Dss = (-2.0 * za * pa + za * za * za * pa + 2.0 * zb * pb - zb * zb * zb * pb) / s2;
    h[0] = Dmm / D - Dm * Dm / (D * D);
    h[1] = Dms / D - Dm * Ds / (D * D);
    h[2] = Dss / D - Ds * Ds / (D * D);
  } else if (F.kind == FK_EXP) {
    const double lam = th[F.par[0]], L = b - a, z = lam * L;
    double hp;  // h'(z), h(z) = 1/(1 - e^{-z}) - 1/z; Var[x] = L^2 h'(lambda L)
    if (fabs(z) < 0.05) {
      const double z2 = z * z;
      hp = 1.0 / 12.0 + z2 * (-1.0 / 240.0 + z2 * (1.0 / 6048.0 - z2 / 172800.0));
    } else {
      const double em = p_expm1(-z);
      hp = 1.0 / (z * z) - p_exp(-z) / (em * em);
    }
    h[0] = -L * L * hp;
  }
}

// Both prologues of a Hessian pass, by the whole workgroup (256 threads): the
// plan and theta go to LDS first, then compute_constants, then lane f of the
// wave of its kind computes factor f's second-derivative constants.
__device__ __forceinline__ void prologue_from_lds(const Plan* __restrict__ plan, const double* theta,
                                                  ConstBlock* cb, double* hc) {
  __shared__ __align__(16) Plan sp;
  __shared__ __align__(16) ConstBlock scb;
  __shared__ double sth[UML_MAX_PARAMS];
  const int4* src = reinterpret_cast<const int4*>(plan);
  int4* dst = reinterpret_cast<int4*>(&sp);
  for (int k = threadIdx.x; k < int(sizeof(Plan) / 16); k += blockDim.x) dst[k] = src[k];
  __syncthreads();
  for (int k = threadIdx.x; k < sp.npar; k += blockDim.x) sth[k] = theta[k];
  __syncthreads();
  compute_constants(lds(&sp), lds(sth), lds(&scb));
  const int lane = threadIdx.x & 63;
  if (lane < sp.nfac && prologue_wave(sp.fac[lane].kind, blockDim.x >> 6) == int(threadIdx.x >> 6))
    hess_factor_constants(sp.fac[lane], sth, hc + 4 * lane);
  __syncthreads();
  store_const_block(cb, scb);
}

__global__ __launch_bounds__(256) void hess_prologue_kernel(const Plan* __restrict__ plan,
                                                           const double* __restrict__ theta,
                                                           ConstBlock* cb, double* hc) {
  prologue_from_lds(plan, theta, cb, hc);
}

// The same for a batch: workgroup j prepares job j.
__global__ __launch_bounds__(256) void hess_prologue_batch_kernel(const HessJob* __restrict__ jobs) {
  const HessJob& J = jobs[blockIdx.x];
  prologue_from_lds(J.A.plan, J.theta, const_cast<ConstBlock*>(J.A.cb), const_cast<double*>(J.A.hc));
}

template <class T>
__device__ __forceinline__ T ld(const void* col, int64_t i) {
  return static_cast<const T*>(col)[i];
}

// The kernel constants of the event arithmetic's precision (the FP32 set,
// with its pairs, for mixed precision).
__device__ __forceinline__ const float* kconsts(const ConstBlock& cb, float) { return cb.f; }
__device__ __forceinline__ const double* kconsts(const ConstBlock& cb, double) { return cb.d; }
template <class T>
constexpr bool kHessF32 = std::is_same<T, float>::value;

// Evaluates one event and writes its staged row.  A parameter belongs to at
// most one unit of a component (the Hessian plan refuses models where it does
// not), so each entry of l_c is written once after the zeroing: plain stores,
// no read-modify-write chains through LDS.
template <class T>
__device__ void hess_event(const Plan& P, const ConstBlock& cb, const double* hc, const HessPlan& H,
                           T* row) {
  const int nf = P.nfree, nc = P.ncomp;
  T* s = row + 2;
  T* r = s + nf;
  T* lv = r + nc;
  T* q = lv + nc * nf;
  const T* xs = q + H.nq;  // the event's coordinates, staged with the chunk
  for (int k = 0; k < nc * nf; ++k) lv[k] = T(0);
  T E[kMaxComp], V[kMaxComp];
  for (int c = 0; c < nc; ++c) {
    const CompPlan& C = P.comp[c];
    T* l = lv + c * nf;
    const T* kcomp = kconsts(cb, T(0)) + C.cst_lk2;
    T e = kHessF32<T> ? kcomp[1] : kcomp[0];  // log2 K_c: lo part first (see eval.hip)
    T v = T(1);
    for (int k = 0; k < C.nfrac; ++k) {
      const int fp = P.free_pos[C.frac_par[k]];
      if (fp >= 0) l[fp] = T(cb.e[C.frac_ec[k]]);
    }
    for (int j = 0; j < C.nfac; ++j) {
      const int fi = C.fac[j];
      const FactorPlan& F = P.fac[fi];
      const T* kc = kconsts(cb, T(0)) + F.cst;
      const double* ec = cb.e + F.ecst;
      T* qf = q + H.q_off[fi];
      switch (F.kind) {
        case FK_GAUSS: {
          const T x = xs[F.dim[0]] - T(F.xref);
          const T d = x - kc[0];
          if constexpr (kHessF32<T>) e = fma(d, fma(-kc[2], d, kc[3]), e);
          e = fma(-d * d, kc[1], e);
          const T lm = fma(d, T(ec[0]), T(ec[1]));
          const T ls = fma(d * d, T(ec[2]), fma(d, T(ec[4]), T(ec[3])));
          const int pm = P.free_pos[F.par[0]], ps = P.free_pos[F.par[1]];
          if (pm >= 0) l[pm] = lm;
          if (ps >= 0) l[ps] = ls;
          const T is2 = T(ec[0]), is3 = T(ec[2]);
          // the centre's remainder c0_lo = k2 / (2 c1) (zero in FP64)
          const T dt = kHessF32<T> ? d - kc[3] / (T(2) * (kc[1] + kc[2])) : d;
          qf[0] = lm * lm - is2 - T(hc[4 * fi + 0]);
          qf[1] = lm * ls - T(2) * dt * is3 - T(hc[4 * fi + 1]);
          qf[2] = ls * ls - T(3) * dt * dt * is2 * is2 + is2 - T(hc[4 * fi + 2]);
          break;
        }
        case FK_EXP: {
          const T x = xs[F.dim[0]] - T(F.xref);
          if constexpr (kHessF32<T>) e = fma(x, kc[1], e);
          e = fma(x, kc[0], e);
          const T lx = x + T(ec[1]);
          const int p = P.free_pos[F.par[0]];
          if (p >= 0) l[p] = lx;
          qf[0] = lx * lx + T(hc[4 * fi + 0]);
          break;
        }
        case FK_CHEB: {
          const int k = F.order;
          const T x = xs[F.dim[0]] - T(F.xref);
          const T u = kHessF32<T> ? fma(x, kc[0], fma(x, kc[1], kc[2])) : fma(x, kc[0], kc[2]);
          T tj[kMaxCheb + 1];
          tj[0] = T(1);
          tj[1] = u;
          for (int jj = 2; jj <= k; ++jj) tj[jj] = T(2) * u * tj[jj - 1] - tj[jj - 2];
          T val = kc[3];
          for (int jj = 1; jj <= k; ++jj) val = fma(kc[3 + jj], tj[jj], val);
          v *= val;
          const T iv = T(1) / val;
          for (int jj = 0; jj < k; ++jj) {
            const int p = P.free_pos[F.par[jj]];
            if (p >= 0) l[p] = fma(T(ec[jj]) * tj[jj + 1], iv, T(ec[k + jj]));
          }
          int t = 0;
          for (int a = 0; a < k; ++a)
            for (int b = a; b < k; ++b, ++t)
              qf[t] = T(ec[0]) * iv * (tj[a + 1] * T(ec[k + b]) + tj[b + 1] * T(ec[k + a])) +
                      T(2) * T(ec[k + a]) * T(ec[k + b]);
          break;
        }
        case FK_PWAVE: {
          const T cl = xs[F.dim[0]], ck = xs[F.dim[1]], ph = xs[F.dim[2]];
          const T sl2 = fma(-cl, cl, T(1)), sk2 = fma(-ck, ck, T(1));
          const T skl2 = sk2 * sl2, skl = k_sqrt(skl2);
          T sp, cp;
          k_sincos(ph, sp, cp);
          const T w = ck * skl, wc = w * cl;
          const T u0 = fma(T(-0.5), skl2, sk2);
          T m[8];
          m[0] = fma((ck + ck) * ck, sl2, -u0);
          m[1] = skl2 * fma(cp + cp, cp, T(-1));
          m[2] = wc * cp;
          m[3] = w * cp;
          m[4] = sk2 * cl;
          m[5] = w * sp;
          m[6] = wc * sp;
          m[7] = skl2 * (sp * cp);
          T val = T(0);  // the coefficients' lo parts first (zero in FP64), then hi, then u0
          if constexpr (kHessF32<T>)
            for (int kk = 0; kk < 8; ++kk) val = fma(kc[8 + kk], m[kk], val);
          for (int kk = 0; kk < 8; ++kk) val = fma(kc[kk], m[kk], val);
          val += u0;
          v *= val;
          const T iv = T(1) / val;
          for (int kk = 0; kk < 8; ++kk) {
            const int p = P.free_pos[F.par[kk]];
            if (p >= 0) l[p] = T(ec[kk]) * m[kk] * iv;
          }
          break;
        }
      }
    }
    E[c] = kHessF32<T> ? e + kcomp[0] : e;
    V[c] = v;
  }
  T Emax = E[0];
  for (int c = 1; c < nc; ++c) Emax = fmax(Emax, E[c]);
  T Sp[kMaxComp], sum = T(0);
  for (int c = 0; c < nc; ++c) {
    Sp[c] = k_exp2(E[c] - Emax) * V[c];
    sum += Sp[c];
  }
  const T inv = T(1) / sum;
  row[1] = Emax + k_log2(sum);
  for (int c = 0; c < nc; ++c) r[c] = Sp[c] * inv;
  // s = sum_c r_c l_c, four parameters per step: every load of a step is
  // issued before its stores (s and l_c are disjoint parts of the row)
  const T* __restrict__ lr = lv;
  T* __restrict__ sw = s;
  for (int a0 = 0; a0 < nf; a0 += 4) {
    T sa[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c < nc) {
        T lv4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) lv4[u] = a0 + u < nf ? lr[c * nf + a0 + u] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) sa[u] = fma(r[c], lv4[u], sa[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (a0 + u < nf) sw[a0 + u] = sa[u];
  }
}

typedef double hess_d4 __attribute__((ext_vector_type(4)));

// The matrix sums of a tile, over the free parameters padded to 16 or 32:
//   product 0: sum w s s^T,  product 1: sum w^2 s s^T,
//   product 2 + c: sum w r_c l_c l_c^T (component c),
// each as 1 or 2 x 2 blocks of 16 x 16 (block b: rows 16 (b >> 1), columns
// 16 (b & 1); block 2, below the diagonal, is never formed, since the sums
// are symmetric).  Product p belongs to wave p % 4.
static_assert(kBlock == 256, "the Hessian tile assigns its matrix products to four waves");
constexpr int kHessProdPerWave = (2 + kMaxComp + 3) / 4;

// One tile of one dataset: its M sums go to A.part[j * A.n_tiles + tile].
// Per chunk, the staged rows feed
//   * the vector sums (one thread each): sum w log2 P, sum w s_a, and
//     sum w r_c q_k for every second-derivative entry k of a factor of c;
//   * the matrix sums on the FP64 matrix cores (v_mfma_f64_16x16x4f64: four
//     events per instruction; lane l supplies row l % 16 of the left operand
//     and column l % 16 of the right one for event l / 16, and holds outputs
//     (l / 16 + 4 i, l % 16), i < 4).
// At the end of the tile the pairs are assembled from them:
//   H_ab  = (sum w s s^T)_ab - sum_c [l_a l_b of c if a and b are in different
//           units of c; sum w r_c q of their unit if in the same one; else 0],
//   W2_ab = (sum w^2 s s^T)_ab.
template <class T>
__device__ __forceinline__ void hess_tile(const HessArgs& A, int tile) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Plan* sP = reinterpret_cast<Plan*>(lds_raw);
  ConstBlock* sC = reinterpret_cast<ConstBlock*>(lds_raw + sizeof(Plan));
  HessPlan* sH = reinterpret_cast<HessPlan*>(lds_raw + sizeof(Plan) + sizeof(ConstBlock));
  double* sh = reinterpret_cast<double*>(lds_raw + sizeof(Plan) + sizeof(ConstBlock) + sizeof(HessPlan));
  T* stage = reinterpret_cast<T*>(sh + 4 * kMaxFac);
  const int tid = threadIdx.x;
  {
    const int4* src = reinterpret_cast<const int4*>(A.plan);
    int4* dst = reinterpret_cast<int4*>(sP);
    for (int k = tid; k < int(sizeof(Plan) / 16); k += kBlock) dst[k] = src[k];
    src = reinterpret_cast<const int4*>(A.cb);
    dst = reinterpret_cast<int4*>(sC);
    for (int k = tid; k < int(sizeof(ConstBlock) / 16); k += kBlock) dst[k] = src[k];
    src = reinterpret_cast<const int4*>(A.hplan);
    dst = reinterpret_cast<int4*>(sH);
    for (int k = tid; k < int(sizeof(HessPlan) / 16); k += kBlock) dst[k] = src[k];
    for (int k = tid; k < 4 * kMaxFac; k += kBlock) sh[k] = A.hc[k];
  }
  __syncthreads();
  const Plan& P = *sP;
  const HessPlan& H = *sH;
  const int nf = P.nfree, nc = P.ncomp, V = A.row_len, M = A.n_sums;
  const int lane = tid & 63;
  const int nb = nf > 16 ? 2 : 1;
  const int nvec = 1 + nf + H.nq;
  const int r_off = 2 + nf, l_off = 2 + nf + nc, q_off = 2 + nf + nc + nc * nf;
  const int x_off = q_off + H.nq, nd = P.ndim;
  // this thread's vector sum: the staged value it weights, and the
  // responsibility it is multiplied by (-1: none)
  int voff = -1, vr = -1;
  // Each vector sum is split over vrep threads: thread t takes sum t % nvec
  // over the tile's events t / nvec, t / nvec + vrep, .. in order, in one
  // running FP64 sum (so the result does not depend on the chunk size); the
  // vrep partials meet in vbuf at the end of the tile and are added in a
  // fixed order.
  __shared__ double vbuf[kBlock];
  const int vrep = nvec < kBlock ? kBlock / nvec : 1;
  const int vj = tid % nvec, vk = tid / nvec;
  const bool vact = vk < vrep;
  if (!vact) {
  } else if (vj == 0) {
    voff = 1;
  } else if (vj <= nf) {
    voff = 2 + vj - 1;
  } else {
    const int k = vj - 1 - nf;
    int fi = 0;  // the factor of entry k: the last with q_off <= k
    while (fi + 1 < P.nfac && H.q_off[fi + 1] <= k) ++fi;
    int comp = 0;
    for (int c = 0; c < nc; ++c)
      for (int j = 0; j < P.comp[c].nfac; ++j)
        if (P.comp[c].fac[j] == fi) comp = c;
    voff = q_off + k;
    vr = r_off + comp;
  }
  double vpart = 0.0;  // this thread's share of its vector sum
  // this wave's products (wave w takes products w and w + 4), each with its
  // nb x nb accumulator blocks; the wave index is made uniform explicitly so
  // the choice of operands is a scalar branch
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nprod = 2 + nc;
  const int kq = lane >> 4, iq = lane & 15;
  const bool o0 = iq < nf, o1 = iq + 16 < nf;
  const int i0 = o0 ? iq : 0, i1 = o1 ? iq + 16 : 0;
  hess_d4 macc[kHessProdPerWave][4];
#pragma unroll
  for (int u = 0; u < kHessProdPerWave; ++u)
#pragma unroll
    for (int b = 0; b < 4; ++b) macc[u][b] = hess_d4{0.0, 0.0, 0.0, 0.0};
  const int64_t t0 = int64_t(tile) * A.tile_events;
  const int64_t t1 = t0 + A.tile_events < A.n ? t0 + A.tile_events : A.n;
  for (int64_t c0 = t0; c0 < t1; c0 += A.chunk) {
    const int cnt = int((t1 - c0) < A.chunk ? (t1 - c0) : A.chunk);
    // the chunk's weights and coordinates into the rows, column by column
    // (every load of the chunk in flight at once, each column's coalesced)
    for (int k = tid; k < (nd + 1) * cnt; k += kBlock) {
      const int d = k / cnt, e = k - d * cnt;
      T* row = stage + int64_t(e) * V;
      if (d == 0)
        row[0] = A.w ? ld<T>(A.w, c0 + e) : T(1);
      else
        row[x_off + d - 1] = ld<T>(A.col[d - 1], c0 + e);
    }
    __syncthreads();
    if (tid < cnt) hess_event<T>(P, *sC, sh, H, stage + int64_t(tid) * V);
    __syncthreads();
    if (vact) {
      const int vo = vr >= 0 ? vr : 0;
      const int lc0 = int(c0 - t0);  // the chunk's first event within the tile
      for (int e = (vk - lc0 % vrep + vrep) % vrep; e < cnt; e += vrep) {
        const T* r0 = stage + e * V;
        const double v0 = double(r0[0]) * double(r0[voff]);
        vpart += vr >= 0 ? v0 * double(r0[vo]) : v0;
      }
    }
    // matrix sums: per step every lane loads the staged values of its event
    // that this wave's products use (at parameters iq and iq + 16)
    for (int e0 = 0; e0 < cnt; e0 += 4) {
      const int e = e0 + kq;
      const bool ev = e < cnt;
      const T* row = stage + (ev ? e : 0) * V;
      const double w = ev ? double(row[0]) : 0.0;
#pragma unroll
      for (int u = 0; u < kHessProdPerWave; ++u) {
        const int pr = wv + 4 * u;
        if (pr < nprod) {  // uniform
          double x0, x1, sc;
          if (pr < 2) {
            x0 = (ev && o0) ? double(row[2 + i0]) : 0.0;
            x1 = (ev && o1) ? double(row[2 + i1]) : 0.0;
            sc = pr == 0 ? w : w * w;
          } else {
            const int c = pr - 2;
            const T* l = row + l_off + c * nf;
            x0 = (ev && o0) ? double(l[i0]) : 0.0;
            x1 = (ev && o1) ? double(l[i1]) : 0.0;
            sc = w * double(row[r_off + c]);
          }
          const double a0 = x0 * sc;
          macc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x0, macc[u][0], 0, 0, 0);
          if (nb == 2) {
            const double a1 = x1 * sc;
            // block 2 (rows 16-31, columns 0-15) lies below the diagonal: every
            // pair read at the end has a <= b, so it is not formed
            macc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, x1, macc[u][1], 0, 0, 0);
            macc[u][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, x1, macc[u][3], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  if (vact) vbuf[tid] = vpart;
  __syncthreads();
  double vacc = 0.0;
  if (tid < nvec)  // the vrep partials of sum tid, in replica order
    for (int r = 0; r < vrep; ++r) vacc += vbuf[r * nvec + tid];
  // the tile's sums to LDS (over the staging rows): [2 + nc][nf][nf], then the
  // vector sums
  double* mats = reinterpret_cast<double*>(stage);
  double* vs = mats + (2 + nc) * nf * nf;
#pragma unroll
  for (int u = 0; u < kHessProdPerWave; ++u) {
    const int pr = wv + 4 * u;
    if (pr < nprod) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (b >= nb * nb) break;
        const int col = (b & 1) * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rw = (b >> 1) * 16 + (lane >> 4) + 4 * i;
          if (rw < nf && col < nf) mats[(pr * nf + rw) * nf + col] = macc[u][b][i];
        }
      }
    }
  }
  if (tid < nvec) vs[tid] = vacc;
  __syncthreads();
  for (int j = tid; j < M; j += kBlock) {
    double o;
    if (j <= nf) {
      o = vs[j];
    } else {
      const int pr = (j - 1 - nf) % H.npairs;
      const bool w2 = (j - 1 - nf) >= H.npairs;
      const int a = H.pa[pr], b = H.pb[pr];
      if (w2) {
        o = mats[(nf + a) * nf + b];
      } else {
        double d2 = 0.0;  // sum_c of w r_c (d2 S_c / S_c)_ab
        for (int c = 0; c < nc; ++c) {
          const int rc = H.rel[pr * kMaxComp + c];
          if (rc == kRelProduct)
            d2 += mats[((2 + c) * nf + a) * nf + b];
          else if (rc >= 0)
            d2 += vs[1 + nf + rc];
        }
        o = mats[a * nf + b] - d2;
      }
    }
    A.part[int64_t(j) * A.n_tiles + tile] = o;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void hess_kernel(const HessArgs A) {
  hess_tile<T>(A, blockIdx.x);
}

// A batch: the ragged map names (job, tile) for each workgroup; entries with
// a negative job are padding.
template <class T>
__global__ __launch_bounds__(kBlock) void hess_batch_kernel(const HessJob* __restrict__ jobs,
                                                            const int2* __restrict__ tmap) {
  const int2 t = tmap[blockIdx.x];
  if (t.x < 0) return;
  const HessArgs& A = jobs[t.x].A;  // read in place: the column table is indexed at run time
  hess_tile<T>(A, t.y);
}

// Sum j of every tile, by one wave: lane l adds tiles l, l + 64, .. in order
// (Neumaier), then the 64 lane sums are added in a fixed tree.  The order
// depends only on the tile count, so the result is reproducible.
__device__ __forceinline__ void hess_reduce(const double* __restrict__ part, int n_tiles, int j,
                                            double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double* col = part + int64_t(j) * n_tiles;
  double s = 0.0, comp = 0.0;
  for (int t = lane; t < n_tiles; t += 64) {
    const double x = col[t];
    const double u = s + x;
    comp += fabs(s) >= fabs(x) ? (s - u) + x : (x - u) + s;
    s = u;
  }
  double v = s + comp;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if (lane == 0) out[j] = v;
}

// Four sums per workgroup (one per wave).
constexpr int kReduceSumsPerBlock = kBlock / 64;

__global__ __launch_bounds__(kBlock) void hess_reduce_kernel(const double* __restrict__ part, int n_tiles,
                                                             int M, double* __restrict__ out) {
  const int j = blockIdx.x * kReduceSumsPerBlock + int(threadIdx.x >> 6);
  if (j < M) hess_reduce(part, n_tiles, j, out);
}

// A batch: blockIdx.y is the job.
__global__ __launch_bounds__(kBlock) void hess_reduce_batch_kernel(const HessJob* __restrict__ jobs) {
  const HessJob& J = jobs[blockIdx.y];
  const int j = blockIdx.x * kReduceSumsPerBlock + int(threadIdx.x >> 6);
  if (j < J.A.n_sums) hess_reduce(J.A.part, J.A.n_tiles, j, J.out);
}

size_t hess_lds_bytes(int row_len, int chunk, int precision, int mat_bytes) {
  const size_t stage = size_t(row_len) * chunk * (precision == UML_MIXED ? 4 : 8);
  return sizeof(Plan) + sizeof(ConstBlock) + sizeof(HessPlan) + sizeof(double) * 4 * kMaxFac +
         (stage > size_t(mat_bytes) ? stage : size_t(mat_bytes));
}

int hess_mat_bytes(const Plan& P, const HessPlan& H) {
  return int(sizeof(double)) * ((2 + P.ncomp) * P.nfree * P.nfree + 1 + P.nfree + H.nq);
}

void launch_hessian(const HessArgs& A, const double* d_theta, ConstBlock* d_cb, double* d_hc,
                    double* d_out, int precision, hipStream_t s) {
  hipLaunchKernelGGL(hess_prologue_kernel, dim3(1), dim3(256), 0, s, A.plan, d_theta, d_cb, d_hc);
  const size_t lds = hess_lds_bytes(A.row_len, A.chunk, precision, A.mat_bytes);
  if (precision == UML_MIXED)
    hipLaunchKernelGGL(hess_kernel<float>, dim3(A.n_tiles), dim3(kBlock), lds, s, A);
  else
    hipLaunchKernelGGL(hess_kernel<double>, dim3(A.n_tiles), dim3(kBlock), lds, s, A);
  hipLaunchKernelGGL(hess_reduce_kernel, dim3((A.n_sums + kReduceSumsPerBlock - 1) / kReduceSumsPerBlock),
                     dim3(kBlock), 0, s, A.part, A.n_tiles, A.n_sums, d_out);
}

void launch_hessian_batch(const HessJob* d_jobs, int n_jobs, const int2* d_map, int n_map, int row_len,
                          int chunk, int mat_bytes, int n_sums, int precision, hipStream_t s) {
  if (n_jobs <= 0) return;
  hipLaunchKernelGGL(hess_prologue_batch_kernel, dim3(n_jobs), dim3(256), 0, s, d_jobs);
  const size_t lds = hess_lds_bytes(row_len, chunk, precision, mat_bytes);
  if (precision == UML_MIXED)
    hipLaunchKernelGGL(hess_batch_kernel<float>, dim3(n_map), dim3(kBlock), lds, s, d_jobs, d_map);
  else
    hipLaunchKernelGGL(hess_batch_kernel<double>, dim3(n_map), dim3(kBlock), lds, s, d_jobs, d_map);
  hipLaunchKernelGGL(hess_reduce_batch_kernel,
                     dim3((n_sums + kReduceSumsPerBlock - 1) / kReduceSumsPerBlock, n_jobs), dim3(kBlock), 0, s,
                     d_jobs);
}

}  // namespace uml
