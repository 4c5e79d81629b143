// The allocation-free evaluation entry point: NLL and gradient over the
// caller's device columns, with the launch's scratch memory (the constant
// cache and the tile partials of the event kernel)
// in a fixed-size array of this library's device code instead of a
// dataset's work area.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "host.h"
#include "uml.h"

namespace uml {
namespace {

constexpr size_t kAlign = 256;
constexpr size_t up256(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// scratch layout: constant cache | launch count | tile partials (the
// single-dataset event kernel's two alternating buffers of K per tile, each
// slot the sentinel until written)
constexpr size_t kScrCst = 0;
constexpr size_t kScrEpoch = up256(kScrCst + sizeof(ConstBlock));
constexpr size_t kScrPart = up256(kScrEpoch + sizeof(unsigned long long));
constexpr size_t kScrPartDoubles = (size_t(UML_NOALLOC_SCRATCH_BYTES) - kScrPart) / sizeof(double);
static_assert(UML_NOALLOC_SCRATCH_BYTES % kAlign == 0 && kScrPart < UML_NOALLOC_SCRATCH_BYTES,
              "scratch layout");

// One copy per GPU the library runs on, held until the process ends.  Host
// code never uses this name as an address: it uses the device address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[UML_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};
// per device: the extent (K * tiles) of the last call's buffers; a call of
// another extent refills both buffers first, since each call restores only
// the slots of its own layout
int64_t g_extent[kMaxDevices] = {};

__global__ void clear_words(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// The device address of this device's scratch array, looked up on the first
// call on the device (with the device current); the constant cache and the
// launch count are cleared then.  Every call of a new extent (K * tiles)
// fills both partial buffers with the sentinel over the larger of the two
// extents, on the caller's stream; a call of the same extent finds them
// ready (each launch refills the buffer the next one uses).  The cache is
// keyed by model and point.
int scratch_for_current_device(hipStream_t s, int64_t extent, unsigned char** out, const char* fn) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(UML_E_HIP, std::string(fn) + ": hipGetDevice: " + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(UML_E_HIP, std::string(fn) + ": device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(UML_E_HIP, std::string(fn) + ": hipGetSymbolAddress: " + hipGetErrorString(e));
    const int words = int(kScrPart / sizeof(unsigned));
    hipLaunchKernelGGL(clear_words, dim3((words + 255) / 256), dim3(256), 0, s, static_cast<unsigned*>(p), words);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(UML_E_HIP, std::string(fn) + ": " + hipGetErrorString(e));
    g_scratch[dev] = static_cast<unsigned char*>(p);
    g_extent[dev] = -1;
  }
  if (extent != g_extent[dev]) {
    const int64_t fill = 2 * (extent > g_extent[dev] ? extent : g_extent[dev]);
    launch_fill_sentinel(reinterpret_cast<double*>(g_scratch[dev] + kScrPart), fill, s);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(UML_E_HIP, std::string(fn) + ": " + hipGetErrorString(e));
    g_extent[dev] = extent;
  }
  *out = g_scratch[dev];
  return UML_OK;
}

}  // namespace
}  // namespace uml

using namespace uml;

extern "C" int uml_eval_nll_grad_noalloc(const uml_model* m, int64_t n, const void* const* d_cols,
                                         const void* d_w, const double* d_theta_all, double* d_out,
                                         void* stream) {
  const char* fn = "uml_eval_nll_grad_noalloc";
  if (!m) return set_error(UML_E_INVALID, std::string(fn) + ": null model");
  const Plan& P = m->plan;
  if (!d_theta_all || !d_out) return set_error(UML_E_INVALID, std::string(fn) + ": null device pointer");
  if (n < 0) return set_error(UML_E_INVALID, std::string(fn) + ": negative event count");
  if (P.pre_fac >= 0)
    return set_error(UML_E_UNSUPPORTED, std::string(fn) + ": a model with precomputed terms needs a dataset");
  if (n > 0 && !d_cols) return set_error(UML_E_INVALID, std::string(fn) + ": cols is NULL");
  for (int ud = 0; n > 0 && ud < P.ndim; ++ud)
    if (!d_cols[ud] || reinterpret_cast<uintptr_t>(d_cols[ud]) % 16)
      return set_error(UML_E_INVALID, std::string(fn) + ": every column must be a 16-byte aligned device pointer");
  if (d_w && reinterpret_cast<uintptr_t>(d_w) % 16)
    return set_error(UML_E_INVALID, std::string(fn) + ": the weights must be 16-byte aligned");
  const DataLayout L = data_layout(P, n, d_w != nullptr);
  const size_t need = 2 * size_t(P.K) * size_t(L.n_tiles);
  if (need > kScrPartDoubles)
    return set_error(UML_E_INVALID, std::string(fn) + ": " + std::to_string(n) +
                                        " events need " + std::to_string(need * sizeof(double)) +
                                        " bytes of tile partials; the fixed scratch holds " +
                                        std::to_string(kScrPartDoubles * sizeof(double)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* base = nullptr;
  int rc = scratch_for_current_device(s, int64_t(P.K) * L.n_tiles, &base, fn);
  if (rc) return rc;
  Job J{};
  for (int kd = 0; kd < P.ndim; ++kd) J.col[kd] = n > 0 ? d_cols[P.user_of_dim[kd]] : nullptr;
  J.w = d_w;
  J.n = n;
  J.n_tiles = L.n_tiles;
  J.events_per_thread = L.E;
  J.cst = reinterpret_cast<ConstBlock*>(base + kScrCst);
  J.counter = nullptr;   // the single-dataset kernel counts nothing
  J.partials = nullptr;
  J.spart = reinterpret_cast<double*>(base + kScrPart);
  J.epoch = reinterpret_cast<unsigned long long*>(base + kScrEpoch);
  J.out = d_out;
  J.plan = m->d_plan;
  J.fit = nullptr;
  J.theta = d_theta_all;
  J.npar = P.npar;
  J.key = P.key;
  LaunchArgs a{};
  a.job0 = J;
  a.jobs = nullptr;
  a.tmap = nullptr;
  a.grid = L.n_tiles;
  a.out = d_out;
  a.theta = d_theta_all;
  a.precision = P.precision;
  a.stream = s;
  m->family->eval(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(UML_E_HIP, std::string(fn) + ": " + hipGetErrorString(e));
  return UML_OK;
}
