// Pseudo-experiment generation on the device (the toy studies of Sec. 2.5):
// events drawn from a model at a parameter point, written straight into a
// dataset's event columns, so a toy fit needs no upload.
//
// Each event is drawn from its own uniform stream: Philox4x64 with 10 rounds
// (the counter-based generator of Salmon, Moraes, Dror and Shaw, SC11) at
// counters (b, event, 0, 0), b = 0, 1, .., key (seed, 0); each 64-bit word
// gives u = (top 53 bits + 1/2) / 2^53.  An event depends only on (seed,
// index), never on the launch or the lane that draws it.  The model tree is
// walked depth first: a sum picks its first child when u < f, a product draws
// every child in order, and the leaves draw their dimensions:
//   Gaussian     Box-Muller, rejected outside the range;
//   exponential  inverse distribution function;
//   Chebyshev    accept-reject under 1 + sum |c_j|;
//   P-wave       accept-reject of uniform angles under the sum of the
//                absolute coefficients times the maxima of their terms.
// Every accept-reject loop stops after kGenCap attempts (the event is then
// counted as failed), so every lane finishes.
//
// Arithmetic is FP64 without contraction of multiplies and adds.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "gen.h"

#pragma clang fp contract(off)

namespace uml {
namespace {

__device__ __forceinline__ void philox4x64(uint64_t x[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, x[0]), lo0 = M0 * x[0];
    const uint64_t hi1 = __umul64hi(M1, x[2]), lo1 = M1 * x[2];
    const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

constexpr double kPi = 3.14159265358979323846;

// The bracket of the P-wave decay rate (Eq. 4) times 9 / (32 pi).
__device__ __noinline__ double pwave_value(double ctl, double ctk, double phi, const double* c) {
  const double FL = c[0], S3 = c[1], S4 = c[2], S5 = c[3], AFB = c[4], S7 = c[5], S8 = c[6], S9 = c[7];
  const double sl2 = 1.0 - ctl * ctl, sk2 = 1.0 - ctk * ctk;
  const double sl = sqrt(sl2), sk = sqrt(sk2);
  const double c2l = 2.0 * ctl * ctl - 1.0;
  const double s2l = 2.0 * sl * ctl, s2k = 2.0 * sk * ctk;
  const double cp = cos(phi), sp = sin(phi), c2p = cos(2.0 * phi), s2p = sin(2.0 * phi);
  const double v = (1.0 - FL) * (0.75 * sk2) + FL * (ctk * ctk) + (1.0 - FL) * (0.25 * sk2 * c2l) -
                   FL * (ctk * ctk * c2l) + S3 * (sk2 * sl2 * c2p) + S4 * (s2k * s2l * cp) +
                   S5 * (s2k * sl * cp) + AFB * (4.0 / 3.0 * sk2 * ctl) + S7 * (s2k * sl * sp) +
                   S8 * (s2k * s2l * sp) + S9 * (sk2 * sl2 * s2p);
  return 9.0 / (32.0 * kPi) * v;
}

// The same bracket in FP32 with the hardware sine and cosine, for a quick
// accept-reject decision: sin^2 from (1 - c)(1 + c) formed in FP64, so each
// basis term carries a relative error of a few FP32 ulps and the sine and
// cosine an absolute one of about 1e-7; the value is within about 2e-6 times
// the envelope of the FP64 one.
__device__ float pwave_value_f32(double ctl, double ctk, double phi, const float* c) {
  const float FL = c[0], S3 = c[1], S4 = c[2], S5 = c[3], AFB = c[4], S7 = c[5], S8 = c[6], S9 = c[7];
  const float cl = float(ctl), ck = float(ctk);
  const float sl2 = float(1.0 - ctl) * float(1.0 + ctl), sk2 = float(1.0 - ctk) * float(1.0 + ctk);
  const float sl = sqrtf(sl2), sk = sqrtf(sk2);
  const float c2l = 2.0f * cl * cl - 1.0f;
  const float s2l = 2.0f * sl * cl, s2k = 2.0f * sk * ck;
  const float ph = float(phi);
  const float cp = __cosf(ph), sp = __sinf(ph), c2p = __cosf(2.0f * ph), s2p = __sinf(2.0f * ph);
  const float v = (1.0f - FL) * (0.75f * sk2) + FL * (ck * ck) + (1.0f - FL) * (0.25f * sk2 * c2l) -
                  FL * (ck * ck * c2l) + S3 * (sk2 * sl2 * c2p) + S4 * (s2k * s2l * cp) +
                  S5 * (s2k * sl * cp) + AFB * (4.0f / 3.0f * sk2 * cl) + S7 * (s2k * sl * sp) +
                  S8 * (s2k * s2l * sp) + S9 * (sk2 * sl2 * s2p);
  return float(9.0 / (32.0 * kPi)) * v;
}

// Waves per SIMD the generation kernels are built for (a register budget of
// 512 / kGenWaves per lane).
constexpr int kGenWaves = 4;

// Per workgroup: the step program, each node's constants at the point, and
// where each user dimension is stored.
constexpr int kGenNodeK = 12;
struct GenShared {
  GenStep step[kMaxGenSteps];
  double k[UML_MAX_NODES][kGenNodeK];
  float kf[UML_MAX_NODES][8];  // P-wave: the coefficients in FP32
  int dim[UML_MAX_NODES][3];   // leaves: user dimensions
  int order[UML_MAX_NODES];    // Chebyshev: number of coefficients
  void* col[UML_MAX_DIMS];
  double lo[UML_MAX_DIMS], hi[UML_MAX_DIMS];
};

// A node's parameter-only constants (the same values each draw used to form
// for itself):
//   sum          {f}
//   Gaussian     {mu, sigma, lo, hi}
//   exponential  {lambda, lo, hi, L = hi - lo, expm1(lambda L)}
//   Chebyshev    {lo, hi, L, envelope 1 + sum |c_j|, c_1 .. c_k}
//   P-wave       {c_0 .. c_7, envelope}, and the coefficients in FP32
__device__ void node_constants(const GenPlan& G, const GenNode& nd, const double* __restrict__ th, double* K,
                               float* KF) {
  switch (nd.kind) {
    case UML_SUM:
      K[0] = th[nd.par[0]];
      break;
    case UML_GAUSS: {
      const int d = nd.dim[0];
      K[0] = th[nd.par[0]];
      K[1] = th[nd.par[1]];
      K[2] = G.lo[d];
      K[3] = G.hi[d];
      break;
    }
    case UML_EXP: {
      const int d = nd.dim[0];
      const double lo = G.lo[d], hi = G.hi[d], lam = th[nd.par[0]], L = hi - lo;
      K[0] = lam;
      K[1] = lo;
      K[2] = hi;
      K[3] = L;
      K[4] = expm1(lam * L);
      break;
    }
    case UML_CHEB: {
      const int d = nd.dim[0];
      const double lo = G.lo[d], hi = G.hi[d];
      double env = 1.0;
      for (int j = 0; j < nd.npar; ++j) {
        env += fabs(th[nd.par[j]]);
        K[4 + j] = th[nd.par[j]];
      }
      K[0] = lo;
      K[1] = hi;
      K[2] = hi - lo;
      K[3] = env;
      break;
    }
    case UML_PWAVE: {
      double c[8];
      for (int k = 0; k < 8; ++k) c[k] = th[nd.par[k]];
      double env = 0.75 * fabs(1.0 - c[0]) + fabs(c[0]) + 0.25 * fabs(1.0 - c[0]) + fabs(c[0]) +
                   4.0 / 3.0 * fabs(c[4]);
      for (int k = 1; k < 8; ++k)
        if (k != 4) env += fabs(c[k]);
      for (int k = 0; k < 8; ++k) {
        K[k] = c[k];
        KF[k] = float(c[k]);
      }
      K[8] = env * (9.0 / (32.0 * kPi));
      break;
    }
  }
}

// Lane t: step t, node t and user dimension t of the workgroup's tables.
__device__ void gen_setup(GenShared& S, const GenPlan& G, const double* __restrict__ theta, const GenOut& out) {
  const int t = threadIdx.x;
  if (t < G.nstep) S.step[t] = G.step[t];
  if (t < G.nnode) {
    const GenNode& nd = G.node[t];
    node_constants(G, nd, theta, S.k[t], S.kf[t]);
    for (int k = 0; k < 3; ++k) S.dim[t][k] = nd.dim[k];
    S.order[t] = nd.npar;
  }
  if (t < G.ndim) {
    S.col[t] = out.col[G.col_of_user[t]];
    S.lo[t] = G.lo[t];
    S.hi[t] = G.hi[t];
  }
}

template <class T>
__device__ __forceinline__ T to_storage(double v, double lo, double hi);
template <>
__device__ __forceinline__ double to_storage<double>(double v, double, double) {
  return v;
}
// Nearest FP32 value, moved one step inwards if rounding left the range.
template <>
__device__ __forceinline__ float to_storage<float>(double v, double lo, double hi) {
  float f = __double2float_rn(v);
  if (double(f) > hi) f = nextafterf(f, -INFINITY);
  if (double(f) < lo) f = nextafterf(f, INFINITY);
  return f;
}

template <class T>
__device__ __forceinline__ void store(const GenShared& S, int d, int64_t i, double v) {
  static_cast<T*>(S.col[d])[i] = to_storage<T>(v, S.lo[d], S.hi[d]);
}

__device__ __forceinline__ double unit(uint64_t r) {
  return (double(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// Word idx (0..7) of the two-block window w, by selects (no indexed
// registers).
__device__ __forceinline__ uint64_t pick(const uint64_t (&w)[8], int idx) {
  uint64_t r = w[0];
#pragma unroll
  for (int t = 1; t < 8; ++t) r = idx == t ? w[t] : r;
  return r;
}

// Events [b0, b1) of pseudo-experiment `seed`, drawn by one wave.  A lane
// advances its event by one step per pass: a sum's choice or one attempt
// of a leaf.  The stream words the step needs are taken from a window of
// two Philox blocks, the next block drawn at the top of the pass when the
// window runs short, so every lane that needs one computes it together.  A
// lane whose event is complete takes the next event of the range, so lanes
// stay busy until the range runs out whatever their accept-reject luck.
// Each event still reads only its own stream in its own order.
template <class T>
__device__ __forceinline__ void gen_range(const GenShared& S, int root, uint64_t seed, int64_t b0, int64_t b1,
                          unsigned int* bad) {
  const int lane = threadIdx.x & 63;
  int64_t pool = b0;  // the next event not yet taken (the same in every lane)
  int64_t i = 0;
  int st = -1, a = 0, pos = 0, nb = 0;
  bool ok = true;
  uint64_t blk = 0;
  uint64_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  while (true) {
    const bool want = st < 0;
    const uint64_t m = __ballot(want);
    if (want) {
      const int64_t j = pool + __popcll(m & ((1ull << lane) - 1));
      if (j < b1) {
        i = j;
        st = root;
        a = 0;
        ok = true;
        blk = 0;
        nb = 0;
        pos = 0;
      }
    }
    pool += __popcll(m);
    if (!__any(st >= 0)) break;
    if (st < 0) continue;
    const GenStep P = S.step[st];
    const double* K = S.k[P.node];
    const int need = P.kind == UML_PWAVE ? 4 : (P.kind == UML_GAUSS || P.kind == UML_CHEB) ? 2 : 1;
    if (4 * nb - pos < need) {  // the event's next block: counters (block, event, 0, 0), key (seed, 0)
      uint64_t x[4] = {blk, uint64_t(i), 0, 0};
      philox4x64(x, seed, 0);
      ++blk;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        w[t] = nb == 0 ? x[t] : w[t];
        w[4 + t] = nb == 0 ? w[4 + t] : x[t];
      }
      ++nb;
    }
    double u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) u[t] = unit(pick(w, pos + t));
    pos += need;
    if (pos >= 4) {
#pragma unroll
      for (int t = 0; t < 4; ++t) w[t] = w[4 + t];
      pos -= 4;
      --nb;
    }
    if (P.kind == UML_SUM) {
      st = u[0] < K[0] ? P.child[0] : P.child[1];
      continue;
    }
    const int* D = S.dim[P.node];
    bool drawn = false;  // the leaf has its value
    if (P.kind == UML_GAUSS) {  // Box-Muller, rejected outside the range
      const double v = K[0] + K[1] * (sqrt(-2.0 * log(u[0])) * cos(2.0 * kPi * u[1]));
      drawn = v >= K[2] && v <= K[3];
      if (drawn) store<T>(S, D[0], i, v);
    } else if (P.kind == UML_EXP) {  // inverse distribution function
      const double lam = K[0], lo = K[1], hi = K[2], L = K[3];
      const double v = lam == 0.0 ? lo + u[0] * L : lo + log1p(u[0] * K[4]) / lam;
      store<T>(S, D[0], i, v < lo ? lo : (v > hi ? hi : v));
      drawn = true;
    } else if (P.kind == UML_CHEB) {  // accept-reject under 1 + sum |c_j|
      const double lo = K[0], hi = K[1], L = K[2];
      const double v = lo + u[0] * L;
      const double t = (2.0 * v - lo - hi) / L;
      double tm = 1.0, tj = t, val = 1.0;
      const int k = S.order[P.node];
      for (int j = 1; j <= k; ++j) {
        val += K[3 + j] * tj;
        const double tn = 2.0 * t * tj - tm;
        tm = tj;
        tj = tn;
      }
      drawn = u[1] * K[3] <= val;
      if (drawn) store<T>(S, D[0], i, v);
    } else {  // P-wave: accept-reject of uniform angles
      // The decision u4 env <= value is taken from the FP32 value when the two
      // sides differ by more than 1e-4 env (fifty times its error bound), and
      // from the FP64 value otherwise, so it is always the FP64 decision.
      const double env = K[8];
      const float margin = float(1e-4 * env);
      const double ctl = 2.0 * u[0] - 1.0, ctk = 2.0 * u[1] - 1.0, phi = kPi * (2.0 * u[2] - 1.0);
      const double lhs = u[3] * env;
      const float gap = float(lhs) - pwave_value_f32(ctl, ctk, phi, S.kf[P.node]);
      drawn = gap > margin ? false : gap < -margin ? true : lhs <= pwave_value(ctl, ctk, phi, K);
      if (drawn) {
        store<T>(S, D[0], i, ctl);
        store<T>(S, D[1], i, ctk);
        store<T>(S, D[2], i, phi);
      }
    }
    if (!drawn && ++a == kGenCap) {  // the attempt cap: the leaf's dimensions at their lower ends
      const int nd = P.kind == UML_PWAVE ? 3 : 1;
      for (int k = 0; k < nd; ++k) store<T>(S, D[k], i, S.lo[D[k]]);
      ok = false;
      drawn = true;
    }
    if (drawn) {
      st = P.next;
      a = 0;
      if (st < 0 && !ok) atomicAdd(bad, 1u);
    }
  }
}

template <class T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kGenWaves))) void generate_kernel(const GenPlan* __restrict__ plan,
                                                      const double* __restrict__ theta, uint64_t seed,
                                                      const GenOut out, int64_t block) {
  __shared__ GenShared S;
  gen_setup(S, *plan, theta, out);
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * block;
  const int64_t b1 = b0 + block < out.n ? b0 + block : out.n;
  gen_range<T>(S, plan->root_step, seed, b0, b1, out.bad);
}

// Many pseudo-experiments at once: the map names (job, block of `block`
// events) for each workgroup.
template <class T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kGenWaves))) void generate_batch_kernel(const GenPlan* __restrict__ plan,
                                                            const GenJob* __restrict__ jobs,
                                                            const int2* __restrict__ map, int64_t block) {
  __shared__ GenShared S;
  const int2 t = map[blockIdx.x];
  const GenJob& J = jobs[t.x];
  gen_setup(S, *plan, J.theta, J.out);
  __syncthreads();
  const int64_t b0 = int64_t(t.y) * block;
  const int64_t b1 = b0 + block < J.out.n ? b0 + block : J.out.n;
  gen_range<T>(S, plan->root_step, J.seed, b0, b1, J.out.bad);
}

}  // namespace

void launch_generate_batch(const GenPlan* d_plan, const GenJob* d_jobs, const int2* d_map, int n_map,
                           int64_t block, int precision, hipStream_t s) {
  if (n_map <= 0) return;
  if (precision == UML_MIXED)
    hipLaunchKernelGGL(generate_batch_kernel<float>, dim3(n_map), dim3(64), 0, s, d_plan, d_jobs, d_map, block);
  else
    hipLaunchKernelGGL(generate_batch_kernel<double>, dim3(n_map), dim3(64), 0, s, d_plan, d_jobs, d_map,
                       block);
}

void launch_generate(const GenPlan* d_plan, const double* d_theta, uint64_t seed, const GenOut& out,
                     int precision, hipStream_t s) {
  if (out.n <= 0) return;
  const int64_t block = gen_block_events(out.n);
  const unsigned blocks = unsigned((out.n + block - 1) / block);
  if (precision == UML_MIXED)
    hipLaunchKernelGGL(generate_kernel<float>, dim3(blocks), dim3(64), 0, s, d_plan, d_theta, seed, out, block);
  else
    hipLaunchKernelGGL(generate_kernel<double>, dim3(blocks), dim3(64), 0, s, d_plan, d_theta, seed, out, block);
}

}  // namespace uml
