// Allocation-free evaluation of the source field at query points: the fixed
// per-GPU scratch area and its layout (device code in noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sa {

// at most this many query points per call, and the source history is split
// into at most this many chunks (their partials live in the scratch area)
constexpr int64_t kNoAllocMaxPoints = 4096;
constexpr int kNoAllocMaxChunks = 64;
// chunk partials (64 x 5 x 4096 doubles, 10 MiB), the centred points in FP64
// and FP32, the gradient and density outputs the caller does not take, roles
constexpr size_t kNoAllocScratchBytes = (size_t)11 << 20;

struct NoAllocLayout {
  int64_t stride;             // points rounded up to 64
  double *part;               // [n_chunks][5][stride]
  double *px, *py, *pz, *pq2;
  float *fx, *fy, *fz, *fq2;
  double *G;                  // [3][stride] gradient when the caller passes none
  double *ld;                 // [stride] densities (zero for query points)
  int8_t *role;               // [stride]
  size_t bytes;               // bytes of the area used
};

// device address of the scratch area on `device` (the current device),
// taken once per device; nullptr if it cannot be had
void *noalloc_scratch(int device);
// the sub-arrays of the area for n points and n_chunks chunks (host arithmetic
// only; base NULL gives the bytes alone)
NoAllocLayout noalloc_layout(void *base, int64_t n, int n_chunks);
// centred coordinates (FP64, FP32), |x|^2 and roles of x [n][3] (device)
void launch_noalloc_points(hipStream_t st, int64_t n, const double *x, const double center[3],
                           const NoAllocLayout &L);

}  // namespace sa
