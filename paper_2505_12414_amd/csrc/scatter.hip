// Placement kernels of the packed transfers (see scatter.h).
#include <hip/hip_runtime.h>

#include "scatter.h"

namespace uml {
namespace {

__global__ __launch_bounds__(256) void scatter_kernel(const PackRec* __restrict__ recs,
                                                      const uint64_t* __restrict__ staging) {
  const PackRec r = recs[blockIdx.x];
  uint64_t* dst = static_cast<uint64_t*>(r.ptr);
  const int64_t n = r.nbytes / 8;
  if (r.off < 0) {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = 0;
  } else {
    const uint64_t* src = staging + r.off / 8;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  }
}

__global__ __launch_bounds__(256) void gather_kernel(const PackRec* __restrict__ recs,
                                                     uint64_t* __restrict__ staging) {
  const PackRec r = recs[blockIdx.x];
  const uint64_t* src = static_cast<const uint64_t*>(r.ptr);
  uint64_t* dst = staging + r.off / 8;
  const int64_t n = r.nbytes / 8;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void collect_ints_kernel(const char* __restrict__ base, int64_t stride, int n,
                                                           int* __restrict__ out) {
  for (int i = int(blockIdx.x) * 256 + threadIdx.x; i < n; i += int(gridDim.x) * 256)
    out[i] = *reinterpret_cast<const int*>(base + stride * i);
}

template <class T>
__global__ __launch_bounds__(256) void check_events_kernel(const CheckArgs a) {
  unsigned int bad = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * 256) {
    for (int d = 0; d < a.ndim; ++d) {
      const double v = double(static_cast<const T*>(a.col[d])[i]);
      if (!(v >= a.lo[d] && v <= a.hi[d])) ++bad;  // also catches NaN
    }
    if (a.w) {
      const double v = double(static_cast<const T*>(a.w)[i]);
      if (!isfinite(v)) ++bad;
    }
  }
  if (bad) atomicAdd(a.bad, bad);
}

}  // namespace

void launch_check_events(const CheckArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  const int64_t want = (a.n + 255) / 256;
  const unsigned blocks = unsigned(want < 4096 ? want : 4096);
  if (a.fp64)
    hipLaunchKernelGGL(check_events_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(check_events_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
}

void launch_scatter(const PackRec* d_recs, int n, const void* d_staging, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scatter_kernel, dim3(n), dim3(256), 0, s, d_recs, static_cast<const uint64_t*>(d_staging));
}

void launch_collect_ints(const void* base, int64_t stride, int n, int* out, hipStream_t s) {
  if (n <= 0) return;
  const int blocks = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
  hipLaunchKernelGGL(collect_ints_kernel, dim3(blocks), dim3(256), 0, s, static_cast<const char*>(base), stride,
                     n, out);
}

void launch_gather(const PackRec* d_recs, int n, void* d_staging, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_kernel, dim3(n), dim3(256), 0, s, d_recs, static_cast<uint64_t*>(d_staging));
}

}  // namespace uml
