// Fixed device scratch area of the allocation-free source-field evaluation
// (sa_iga_eval_source_field_noalloc) and its point-preparation kernel.
//
// The area is one file-scope device array per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel or a copy: its
// device address is taken once per device with hipGetSymbolAddress (at the
// set-up of the first object on that device) and that address is used.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "noalloc.h"

namespace sa {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// centred point coordinates and |x|^2 in FP64 and FP32, roles (the query
// points take no flux or Dirichlet density)
__global__ void k_noalloc_points(int64_t n, const double *__restrict__ x, double cx, double cy, double cz,
                                 NoAllocLayout L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[3 * i] - cx, b = x[3 * i + 1] - cy, c = x[3 * i + 2] - cz;
  const double q2 = a * a + b * b + c * c;
  L.px[i] = a;
  L.py[i] = b;
  L.pz[i] = c;
  L.pq2[i] = q2;
  L.fx[i] = (float)a;
  L.fy[i] = (float)b;
  L.fz[i] = (float)c;
  L.fq2[i] = (float)q2;
  L.role[i] = (int8_t)2;
}

}  // namespace

// device address of this device's scratch area (nullptr on failure); the
// device must be current
void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_ptr[device] = p;
  }
  return g_ptr[device];
}

NoAllocLayout noalloc_layout(void *base, int64_t n, int n_chunks) {
  NoAllocLayout L{};
  // address arithmetic on integers: a null base gives the sizes alone
  const uintptr_t b0 = (uintptr_t)base;
  uintptr_t b = b0;
  const int64_t s = (n + 63) / 64 * 64;
  auto take = [&](size_t bytes) {
    void *p = (void *)b;
    b += (bytes + 255) / 256 * 256;
    return p;
  };
  L.stride = s;
  L.part = (double *)take((size_t)n_chunks * 5 * s * sizeof(double));
  L.px = (double *)take(s * sizeof(double));
  L.py = (double *)take(s * sizeof(double));
  L.pz = (double *)take(s * sizeof(double));
  L.pq2 = (double *)take(s * sizeof(double));
  L.fx = (float *)take(s * sizeof(float));
  L.fy = (float *)take(s * sizeof(float));
  L.fz = (float *)take(s * sizeof(float));
  L.fq2 = (float *)take(s * sizeof(float));
  L.G = (double *)take(3 * s * sizeof(double));
  L.ld = (double *)take(s * sizeof(double));
  L.role = (int8_t *)take(s);
  L.bytes = (size_t)(b - b0);
  return L;
}

void launch_noalloc_points(hipStream_t st, int64_t n, const double *x, const double center[3],
                           const NoAllocLayout &L) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_noalloc_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, center[0],
                     center[1], center[2], L);
}

}  // namespace sa
