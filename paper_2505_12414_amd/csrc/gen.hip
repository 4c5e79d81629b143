// Pseudo-experiment generation on the device (the toy studies of Sec. 2.5):
// events drawn from a model at a parameter point, written straight into a
// dataset's event columns, so a toy fit needs no upload.
//
// Each event is drawn by one thread from its own uniform stream: Philox4x64
// with 10 rounds (the counter-based generator of Salmon, Moraes, Dror and
// Shaw, SC11) at counters (b, event, 0, 0), b = 0, 1, .., key (seed, 0); each
// 64-bit word gives u = (top 53 bits + 1/2) / 2^53.  An event depends only on
// (seed, index), never on the launch.  The model tree is walked depth first:
// a sum picks its first child when u < f, a product draws every child in
// order, and the leaves draw their dimensions:
//   Gaussian     Box-Muller, rejected outside the range;
//   exponential  inverse distribution function;
//   Chebyshev    accept-reject under 1 + sum |c_j|;
//   P-wave       accept-reject of uniform angles under the sum of the
//                absolute coefficients times the maxima of their terms.
// Every accept-reject loop stops after kGenCap attempts (the event is then
// counted as failed), so every thread finishes.
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

struct Stream {
  uint64_t seed, event, block;
  uint64_t buf[4];
  int pos;
  __device__ double next() {
    if (pos == 4) {
      buf[0] = block;
      buf[1] = event;
      buf[2] = 0;
      buf[3] = 0;
      philox4x64(buf, seed, 0);
      ++block;
      pos = 0;
    }
    const uint64_t r = buf[pos++];
    return (double(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  }
};

constexpr double kPi = 3.14159265358979323846;

// The bracket of the P-wave decay rate (Eq. 4) times 9 / (32 pi).
__device__ double pwave_value(double ctl, double ctk, double phi, const double* c) {
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

// Draws the dimensions of one leaf into x (user order); false if the draw
// hit the attempt cap.
__device__ bool draw_leaf(const GenPlan& G, const GenNode& nd, const double* th, Stream& s, double* x) {
  switch (nd.kind) {
    case UML_GAUSS: {
      const int d = nd.dim[0];
      const double lo = G.lo[d], hi = G.hi[d], mu = th[nd.par[0]], sg = th[nd.par[1]];
      for (int a = 0; a < kGenCap; ++a) {
        const double u1 = s.next(), u2 = s.next();
        const double v = mu + sg * (sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2));
        if (v >= lo && v <= hi) {
          x[d] = v;
          return true;
        }
      }
      x[d] = lo;
      return false;
    }
    case UML_EXP: {
      const int d = nd.dim[0];
      const double lo = G.lo[d], hi = G.hi[d], lam = th[nd.par[0]], L = hi - lo;
      const double u = s.next();
      const double v = lam == 0.0 ? lo + u * L : lo + log1p(u * expm1(lam * L)) / lam;
      x[d] = v < lo ? lo : (v > hi ? hi : v);
      return true;
    }
    case UML_CHEB: {
      const int d = nd.dim[0], k = nd.npar;
      const double lo = G.lo[d], hi = G.hi[d], L = hi - lo;
      double env = 1.0;
      for (int j = 0; j < k; ++j) env += fabs(th[nd.par[j]]);
      for (int a = 0; a < kGenCap; ++a) {
        const double u1 = s.next(), u2 = s.next();
        const double v = lo + u1 * L;
        const double t = (2.0 * v - lo - hi) / L;
        double tm = 1.0, tj = t, val = 1.0;
        for (int j = 1; j <= k; ++j) {
          val += th[nd.par[j - 1]] * tj;
          const double tn = 2.0 * t * tj - tm;
          tm = tj;
          tj = tn;
        }
        if (u2 * env <= val) {
          x[d] = v;
          return true;
        }
      }
      x[d] = lo;
      return false;
    }
    case UML_PWAVE: {
      double c[8];
      for (int k = 0; k < 8; ++k) c[k] = th[nd.par[k]];
      double env = 0.75 * fabs(1.0 - c[0]) + fabs(c[0]) + 0.25 * fabs(1.0 - c[0]) + fabs(c[0]) +
                   4.0 / 3.0 * fabs(c[4]);
      for (int k = 1; k < 8; ++k)
        if (k != 4) env += fabs(c[k]);
      env *= 9.0 / (32.0 * kPi);
      // The decision u4 env <= value is taken from the FP32 value when the two
      // sides differ by more than 1e-4 env (fifty times its error bound), and
      // from the FP64 value otherwise, so it is always the FP64 decision.
      float cf[8];
      for (int k = 0; k < 8; ++k) cf[k] = float(c[k]);
      const float margin = float(1e-4 * env);
      for (int a = 0; a < kGenCap; ++a) {
        const double u1 = s.next(), u2 = s.next(), u3 = s.next(), u4 = s.next();
        const double ctl = 2.0 * u1 - 1.0, ctk = 2.0 * u2 - 1.0, phi = kPi * (2.0 * u3 - 1.0);
        const double lhs = u4 * env;
        const float gap = float(lhs) - pwave_value_f32(ctl, ctk, phi, cf);
        const bool accept = gap > margin ? false : gap < -margin ? true : lhs <= pwave_value(ctl, ctk, phi, c);
        if (accept) {
          x[nd.dim[0]] = ctl;
          x[nd.dim[1]] = ctk;
          x[nd.dim[2]] = phi;
          return true;
        }
      }
      for (int k = 0; k < 3; ++k) x[nd.dim[k]] = G.lo[nd.dim[k]];
      return false;
    }
  }
  return false;
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

// Event i of pseudo-experiment `seed` at theta, stored into out.
template <class T>
__device__ void draw_event(const GenPlan& G, const double* __restrict__ theta, uint64_t seed, int64_t i,
                           const GenOut& out) {
  double th[UML_MAX_PARAMS];
  for (int k = 0; k < G.npar; ++k) th[k] = theta[k];
  double x[UML_MAX_DIMS];
  for (int d = 0; d < G.ndim; ++d) x[d] = G.lo[d];
  Stream s{seed, uint64_t(i), 0, {0, 0, 0, 0}, 4};
  // depth-first walk with an explicit stack (children pushed in reverse,
  // so they are drawn in order)
  int stack[UML_MAX_NODES];
  int top = 0;
  stack[top++] = G.root;
  bool ok = true;
  while (top > 0) {
    const GenNode& nd = G.node[stack[--top]];
    if (nd.kind == UML_SUM) {
      const double u = s.next();
      stack[top++] = nd.child[u < th[nd.par[0]] ? 0 : 1];
    } else if (nd.kind == UML_PROD) {
      for (int c = nd.nchild - 1; c >= 0; --c) stack[top++] = nd.child[c];
    } else {
      ok &= draw_leaf(G, nd, th, s, x);
    }
  }
  if (!ok) atomicAdd(out.bad, 1u);
  for (int d = 0; d < G.ndim; ++d)
    static_cast<T*>(out.col[G.col_of_user[d]])[i] = to_storage<T>(x[d], G.lo[d], G.hi[d]);
}

template <class T>
__global__ __launch_bounds__(256) void generate_kernel(const GenPlan* __restrict__ plan,
                                                       const double* __restrict__ theta, uint64_t seed,
                                                       const GenOut out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < out.n) draw_event<T>(*plan, theta, seed, i, out);
}

// Many pseudo-experiments at once: the map names (job, block of 256 events)
// for each workgroup.
template <class T>
__global__ __launch_bounds__(256) void generate_batch_kernel(const GenPlan* __restrict__ plan,
                                                             const GenJob* __restrict__ jobs,
                                                             const int2* __restrict__ map) {
  const int2 t = map[blockIdx.x];
  const GenJob& J = jobs[t.x];
  const int64_t i = int64_t(t.y) * 256 + threadIdx.x;
  if (i < J.out.n) draw_event<T>(*plan, J.theta, J.seed, i, J.out);
}

}  // namespace

void launch_generate_batch(const GenPlan* d_plan, const GenJob* d_jobs, const int2* d_map, int n_map,
                           int precision, hipStream_t s) {
  if (n_map <= 0) return;
  if (precision == UML_MIXED)
    hipLaunchKernelGGL(generate_batch_kernel<float>, dim3(n_map), dim3(256), 0, s, d_plan, d_jobs, d_map);
  else
    hipLaunchKernelGGL(generate_batch_kernel<double>, dim3(n_map), dim3(256), 0, s, d_plan, d_jobs, d_map);
}

void launch_generate(const GenPlan* d_plan, const double* d_theta, uint64_t seed, const GenOut& out,
                     int precision, hipStream_t s) {
  if (out.n <= 0) return;
  const unsigned blocks = unsigned((out.n + 255) / 256);
  if (precision == UML_MIXED)
    hipLaunchKernelGGL(generate_kernel<float>, dim3(blocks), dim3(256), 0, s, d_plan, d_theta, seed, out);
  else
    hipLaunchKernelGGL(generate_kernel<double>, dim3(blocks), dim3(256), 0, s, d_plan, d_theta, seed, out);
}

}  // namespace uml
