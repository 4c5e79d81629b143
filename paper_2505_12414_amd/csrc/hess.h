// Hessian pass: layout shared by the host runtime and hess.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "uml_internal.h"

namespace uml {

constexpr int kMaxPairs = UML_MAX_PARAMS * (UML_MAX_PARAMS + 1) / 2;

// Relation of a parameter pair (a, b) within one component (HessPlan::rel):
// index >= 0 of the unit's own d2p/p entry, or one of these.
constexpr signed char kRelAbsent = -1;   // a or b not in the component
constexpr signed char kRelProduct = -2;  // different units: l_a l_b
constexpr signed char kRelZero = -3;     // same fraction or P-wave: linear

// Static structure of the Hessian for one plan (free parameters only).
struct HessPlan {
  int nq;                           // d2p/p entries per event
  int q_off[kMaxFac];               // first entry of each factor
  int npairs;                       // a <= b over free parameters
  short pa[kMaxPairs], pb[kMaxPairs];
  signed char rel[kMaxPairs * kMaxComp];
  int pad_[2];
};
static_assert(sizeof(HessPlan) % 16 == 0, "HessPlan is copied in 16-byte units");

struct HessArgs {
  const void* col[UML_MAX_DIMS];  // kernel-dimension order
  const void* w;
  int64_t n;
  const Plan* plan;
  const ConstBlock* cb;
  const double* hc;        // 4 per factor
  const HessPlan* hplan;
  double* part;            // [n_sums][n_tiles]
  int n_tiles;
  int64_t tile_events;
  int chunk;               // events staged at once
  int row_len;             // staged values per event
  int n_sums;              // 1 + nfree + 2 npairs
  int mat_bytes;           // LDS for a tile's matrix and vector sums
};

// One dataset of a batched Hessian pass: its arguments, its parameter vector
// (device) and where its M sums go (device).
struct HessJob {
  HessArgs A;
  const double* theta;
  double* out;
};

// Builds the Hessian structure; returns false (with a message) when a
// parameter appears in two units of one component.
bool build_hess_plan(const Plan& P, HessPlan& H, std::string& err);
int hess_row_len(const Plan& P, const HessPlan& H);
size_t hess_lds_bytes(int row_len, int chunk, int precision, int mat_bytes);
int hess_mat_bytes(const Plan& P, const HessPlan& H);
void launch_hessian(const HessArgs& A, const double* d_theta, ConstBlock* d_cb, double* d_hc,
                    double* d_out, int precision, hipStream_t s);
// Batched pass over n_jobs datasets of one model: d_map holds n_map (job,
// tile) entries (job < 0: padding); row_len, chunk and n_sums are the
// model's.
void launch_hessian_batch(const HessJob* d_jobs, int n_jobs, const int2* d_map, int n_map, int row_len,
                          int chunk, int mat_bytes, int n_sums, int precision, hipStream_t s);

}  // namespace uml
