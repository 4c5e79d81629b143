// Pseudo-experiment generation on the device: the model tree in the form the
// generation kernel walks (host runtime and gen.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "uml_internal.h"

namespace uml {

struct GenNode {
  int kind;  // UML_GAUSS .. UML_SUM
  int dim[3];
  int npar;
  int par[8];
  int nchild;
  int child[4];
};

struct GenPlan {
  int nnode, root, ndim, npar;
  GenNode node[UML_MAX_NODES];
  double lo[UML_MAX_DIMS], hi[UML_MAX_DIMS];  // user dimension order
  int col_of_user[UML_MAX_DIMS];              // kernel column of each user dimension
};

// Output of one generation: the event columns (kernel order, storage type)
// and a counter of events whose sampling hit the attempt cap.
struct GenOut {
  void* col[UML_MAX_DIMS];
  int64_t n;
  unsigned int* bad;
};

// One pseudo-experiment of a batch: its output, parameters (device) and seed.
struct GenJob {
  GenOut out;
  const double* theta;
  uint64_t seed;
};

constexpr int kGenCap = 65536;  // accept-reject attempts per draw

// Queues the generation of events [0, n) of pseudo-experiment `seed` from the
// plan at the device parameter vector d_theta.
void launch_generate(const GenPlan* d_plan, const double* d_theta, uint64_t seed, const GenOut& out,
                     int precision, hipStream_t s);
// A batch of pseudo-experiments: d_map holds n_map (job, block of 256 events)
// entries.
void launch_generate_batch(const GenPlan* d_plan, const GenJob* d_jobs, const int2* d_map, int n_map,
                           int precision, hipStream_t s);

}  // namespace uml
