// Packed host<->device transfers for the serving loop (and the device-side
// domain check of borrowed event columns): many small pieces for
// many destinations travel in one copy and are placed (or collected) by one
// kernel, instead of one copy each.  Every copy is a separate stream
// operation with a fixed cost of its own, which dominated admitting and
// retiring fits one small copy at a time.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "uml.h"

namespace uml {

// One piece: nbytes (a multiple of 8, 8-byte aligned at both ends) between
// the device address `ptr` and offset `off` of a staging buffer.  For an
// upload, off < 0 writes zeros instead.
struct PackRec {
  void* ptr;
  int64_t off;
  int64_t nbytes;
};

// staging -> pieces; one workgroup per record
void launch_scatter(const PackRec* d_recs, int n, const void* d_staging, hipStream_t s);
// pieces -> staging; one workgroup per record
void launch_gather(const PackRec* d_recs, int n, void* d_staging, hipStream_t s);
// out[i] = the int at base + i * stride, i < n; out may be mapped pinned host
// memory (its device address), so small results reach the host without a copy.
void launch_collect_ints(const void* base, int64_t stride, int n, int* out, hipStream_t s);

// The domain check of borrowed event columns: every value of kernel dimension
// d in [lo[d], hi[d]] and every weight finite; bad counts the violations.
struct CheckArgs {
  const void* col[UML_MAX_DIMS];
  const void* w;
  int ndim;
  int fp64;
  int64_t n;
  double lo[UML_MAX_DIMS], hi[UML_MAX_DIMS];
  unsigned int* bad;
};
void launch_check_events(const CheckArgs& a, hipStream_t s);

}  // namespace uml
