// Host-side entry points of the device code (kernel launchers and the table
// of compiled model shapes).
#pragma once

#include <string>

#include "uml_internal.h"

namespace uml {

struct LaunchArgs {
  Job job0;              // the job of a single-dataset launch (by value)
  const Job* jobs;       // device array of jobs (batched launches)
  const int2* tmap;      // workgroup -> (job, tile), or nullptr: job 0, tile = workgroup
  int grid;              // workgroups
  double* out;           // overrides jobs[0].out when not nullptr
  const double* theta;   // overrides jobs[0].theta when not nullptr
  int precision;
  hipStream_t stream;
};

// One compiled model shape: its signature (see plan_signature) and launchers.
// The precomputed P-wave terms of a dataset: angle columns in, nine columns
// out (u0 and the eight angular terms), in the storage type.
struct PrecomputeArgs {
  const void* in[3];
  void* out[kPWaveTerms];
  int64_t n;
};
void launch_pwave_terms(const PrecomputeArgs& a, int precision, hipStream_t s);
// Fills n 64-bit words at p with the tile-partial sentinel (kSentinel).
void launch_fill_sentinel(double* p, int64_t n, hipStream_t s);

struct Family {
  std::string sig;
  int K;       // accumulators per event
  int ncst;    // kernel constants
  void (*eval)(const LaunchArgs&);
  void (*hess)(const LaunchArgs&, double* hpart, int nfree);
  // events with P <= 0 or not finite at a.theta, added to *d_count
  void (*count)(const LaunchArgs&, unsigned long long* d_count);
};

// Returns the compiled family for a signature, or nullptr.
const Family* find_family(const std::string& sig);
// All compiled signatures, for error messages.
std::string family_list();


}  // namespace uml
