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

// The tree unfolded for a walk without a stack: a sum step picks one of its
// two child steps, a leaf step draws its dimensions and names the step that
// follows it (-1: the event is complete).  Products become these links when
// the plan is built, their children chained in order.
struct GenStep {
  int kind;      // UML_SUM or a leaf kind
  int node;      // the node it visits
  int next;      // leaf: the following step, -1 at the end of the event
  int child[2];  // sum: the entry steps of its two children
};
constexpr int kMaxGenSteps = 64;

struct GenPlan {
  int nnode, root, ndim, npar;
  GenNode node[UML_MAX_NODES];
  int nstep;      // steps of the unfolded tree; -1 if they exceed kMaxGenSteps
  int root_step;  // entry step of the root
  GenStep step[kMaxGenSteps];
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
// Events per workgroup (one wave of 64 lanes) of a generation launch over
// n_total events: 64 times 1, 2, 4 or 8 events per lane, the fewest that
// still make the launch about kGenTargetWaves waves (enough to fill the
// chip), so a lane that draws several events keeps the others busy while
// small launches keep their parallelism.
constexpr int64_t kGenTargetWaves = 4096;
inline int64_t gen_block_events(int64_t n_total) {
  int64_t e = 1;
  while (e < 8 && n_total > 64 * kGenTargetWaves * e) e *= 2;
  return 64 * e;
}

// Queues the generation of events [0, n) of pseudo-experiment `seed` from the
// plan at the device parameter vector d_theta.
void launch_generate(const GenPlan* d_plan, const double* d_theta, uint64_t seed, const GenOut& out,
                     int precision, hipStream_t s);
// A batch of pseudo-experiments: d_map holds n_map (job, block) entries,
// each block `block` events (gen_block_events of the batch's total).
void launch_generate_batch(const GenPlan* d_plan, const GenJob* d_jobs, const int2* d_map, int n_map,
                           int64_t block, int precision, hipStream_t s);

}  // namespace uml
