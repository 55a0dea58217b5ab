// Element-wise kernels of the multi-patch theta-step (the operators and the
// conjugate gradient pieces are the CSR kernels of kernels.hip).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "multipatch.h"

namespace sa {

namespace {

constexpr int kThreads = 256;

// right-hand side of the theta-step on the free unknowns (Eq. 20 with the
// Dirichlet columns moved over) and the first iterate
__global__ void k_mp_rhs(int64_t nI, const int64_t *__restrict__ I, const double *__restrict__ Bw,
                         const double *__restrict__ F1, const double *__restrict__ F0, double theta,
                         const double *__restrict__ AIDvD, const double *__restrict__ w, double *__restrict__ bI,
                         double *__restrict__ xI) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nI) return;
  const int64_t g = I[i];
  double b = Bw[g] + theta * F1[g] + (1.0 - theta) * F0[g];
  if (AIDvD) b -= AIDvD[i];
  bI[i] = b;
  xI[i] = w[g];
}

__global__ void k_mp_commit(int64_t nI, const int64_t *__restrict__ I, const double *__restrict__ xI, int64_t nD,
                            const int64_t *__restrict__ D, const double *__restrict__ vD, double *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nI) w[I[i]] = xI[i];
  else if (i < nI + nD) w[D[i - nI]] = vD[i - nI];
}

__global__ void k_mp_as_gather(int64_t n, const int64_t *__restrict__ gidx, const double *__restrict__ r,
                               double *__restrict__ rp, const PcgScalars *sc) {
  if (sc && sc->done) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t g = gidx[k];
  rp[k] = g >= 0 ? r[g] : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_mp_as_combine(int64_t n, const int64_t *__restrict__ rowptr,
                                                            const int64_t *__restrict__ pos,
                                                            const double *__restrict__ zp,
                                                            const double *__restrict__ r, double *__restrict__ z,
                                                            double *__restrict__ part, const PcgScalars *sc) {
  if (sc && sc->done) return;
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) v += zp[pos[e]];
    z[i] = v;
    acc = fma(r[i], v, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

void launch_mp_rhs(hipStream_t st, int64_t nI, const int64_t *I, const double *Bw, const double *F1, const double *F0,
                   double theta, const double *AIDvD, const double *w, double *bI, double *xI) {
  if (nI <= 0) return;
  hipLaunchKernelGGL(k_mp_rhs, dim3(blocks(nI)), dim3(kThreads), 0, st, nI, I, Bw, F1, F0, theta, AIDvD, w, bI, xI);
}

void launch_mp_commit(hipStream_t st, int64_t nI, const int64_t *I, const double *xI, int64_t nD, const int64_t *D,
                      const double *vD, double *w) {
  if (nI + nD <= 0) return;
  hipLaunchKernelGGL(k_mp_commit, dim3(blocks(nI + nD)), dim3(kThreads), 0, st, nI, I, xI, nD, D, vD, w);
}

void launch_mp_as_gather(hipStream_t st, int64_t n, const int64_t *gidx, const double *r, double *rp,
                         const PcgScalars *sc) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mp_as_gather, dim3(blocks(n)), dim3(kThreads), 0, st, n, gidx, r, rp, sc);
}

void launch_mp_as_combine(hipStream_t st, int64_t n, const int64_t *rowptr, const int64_t *pos, const double *zp,
                          const double *r, double *z, double *part, const PcgScalars *sc) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mp_as_combine, dim3((unsigned)parts_for(n)), dim3(kThreads), 0, st, n, rowptr, pos, zp, r, z,
                     part, sc);
}

}  // namespace sa
