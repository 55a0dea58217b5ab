// Element-wise kernels of the multi-patch theta-step (multipatch_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sa {

// bI[i] = Bw[I[i]] + theta F1[I[i]] + (1 - theta) F0[I[i]] - AIDvD[i]
// (AIDvD may be NULL) and xI[i] = w[I[i]], for i < nI
void launch_mp_rhs(hipStream_t st, int64_t nI, const int64_t *I, const double *Bw, const double *F1, const double *F0,
                   double theta, const double *AIDvD, const double *w, double *bI, double *xI);

// w[I[i]] = xI[i] (i < nI), w[D[j]] = vD[j] (j < nD)
void launch_mp_commit(hipStream_t st, int64_t nI, const int64_t *I, const double *xI, int64_t nD, const int64_t *D,
                      const double *vD, double *w);

struct PcgScalars;

// additive Schwarz over the patches, the two ends (the local solves run in
// between: launch_fd_batch, whose in-LDS form reads r through gidx itself
// and needs no gather, or launch_fd on each patch's vector):
//   gather:  rp[k] = r[gidx[k]] (gidx[k] >= 0), else 0, over the patches'
//            concatenated vectors (n entries)
//   combine: z[i] = sum of zp[pos[e]] over e in [rowptr[i], rowptr[i+1])
//            (the patches holding unknown i, in patch order), and partials of
//            r . z in parts_for(n) blocks
void launch_mp_as_gather(hipStream_t st, int64_t n, const int64_t *gidx, const double *r, double *rp,
                         const PcgScalars *sc);
void launch_mp_as_combine(hipStream_t st, int64_t n, const int64_t *rowptr, const int64_t *pos, const double *zp,
                          const double *r, double *z, double *part, const PcgScalars *sc);

}  // namespace sa
