// Launch wrappers of the gfx950 kernels (device code in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sa {

// per-source coefficient record (FP64: 8 doubles, FP32: 8 floats); the
// exponent of source i at a point x (centred coordinates, q2 = |x|^2) is
//   arg_i(x) = c_i q2 + u_i . x + K_i,   c_i = -1/(4 alpha D_i),
//   u_i = -2 c_i x_i,  K_i = c_i |x_i|^2 + ln(s E_i / (rho c_p (4 pi alpha D_i)^{3/2}))
// (in base 2 for the FP32 record), so that T~_i(x) = exp(arg_i) and
// grad T~_i(x) = exp(arg_i) (2 c_i x + u_i).
constexpr int kCoefStride = 8;
// FP32 far-field tile: the sources summed in FP32 before folding into FP64,
// and the aligned block whose first source is the origin of its FP32 records.
// Far-field chunks start at multiples of it.
constexpr int kTile32 = 128;
// far-chunk lengths: multiples of the sources the matrix-core far kernel
// stages at a time (512), so that only a slot's last chunk ends in a part
// block
constexpr int kFarChunkQuantum = 512;
static_assert(kFarChunkQuantum % kTile32 == 0, "far chunks start on FP32 record blocks");

// Paths advanced by one launch (by value in the kernel arguments).  Slot s
// holds path `path[s]`, whose sources start at row src0[s] of the global
// source arrays; its first n_act[s] sources are switched on and the first
// n_far[s] of those are summed in FP32.  now[s] = (n+1) * sources_per_step is
// the tick count at the end of the slot's step, so slots may sit at
// different steps.
constexpr int kMaxBatch = 64;
struct PathTab {
  int count;
  int32_t path[kMaxBatch];
  int64_t src0[kMaxBatch];
  int32_t n_act[kMaxBatch];
  int32_t n_far[kMaxBatch];
  int64_t now[kMaxBatch];
  uint8_t mode[kMaxBatch];   // 1: the far sources are supplied by the network (not summed here)
};

struct CoeffParams {
  double delta;           // dt / sources_per_step
  double shift;           // r^2 / (8 alpha)
  double alpha;
  double rc;              // rho c_p
  double scale;           // kernel scale s
};

// coefficient records of the switched-on sources of every slot (written at
// the sources' global rows); max_act = max over slots of n_act
void launch_coeff(hipStream_t st, const PathTab &tab, int64_t max_act, const int64_t *tick, const double *sx,
                  const double *sy, const double *sz, const double *E, const CoeffParams &cp,
                  double *c64, float *c32);

struct SumPlan {
  int points_per_lane;    // 1, 2 or 4
  int waves;              // waves per workgroup
  int n_chunks_far, chunk_far;     // FP32 chunks over [0, n_far) of each path
  int n_chunks_near, chunk_near;   // FP64 chunks over [n_far, n_act)
  int64_t nq, part_stride;
};

// partials part[(slot * n_chunks + chunk) * 5 + k][part_stride]; chunks past a
// path's own range write zeros.  With qidx, the kernel sums pl.nq points
// whose indices (into the point arrays and the partials) are qidx[0..nq).
void launch_sum(hipStream_t st, const SumPlan &pl, const PathTab &tab, const double *px, const double *py,
                const double *pz, const double *pq2, const float *fx, const float *fy, const float *fz,
                const float *fq2, const double *c64, const float *c32, double *part,
                const int32_t *qidx = nullptr);

// A planar face whose points form the grid x[ax_a] = sa[a], x[ax_b] = sb[b],
// x[ax_n] = sn (centred coordinates), point index off + b * na + a.
struct TFace {
  int na, nb, ax_a, ax_b, ax_n;
  int64_t off;
  double sn;
  const double *sa, *sb;
};
// 32 x 32 point tiles of the tensor faces: {face, b0, a0, 0}
struct TensorArgs {
  const TFace *faces;
  const int4 *tiles;
  int n_tiles;
  const double *sx, *sy, *sz;    // centred source positions (all paths)
  const double *c64;             // coefficient records (c, ..., ln A at [5])
  // or, where age_c is set, the coefficients from the source's age a = now -
  // tick (an integer number of source intervals): c = age_c[a],
  // ln A = src_le[i] + age_l[a] (no coefficient records needed)
  const int64_t *tick;
  const double *age_c, *age_l, *src_le;
  double *part;
  int64_t stride;
  int max_groups;                // workgroups of a launch of one to three paths (0: one per work item)
  int max_groups_batch;          // ... of four paths or more, where the sum dominates the step
  int lds_pad;                   // extra LDS bytes per workgroup: fewer groups per compute unit, room
                                 // for the kernels that run beside the sum
};
// allow lds_pad bytes of dynamic LDS for the tensor sum
bool sum_tensor_prepare(int lds_pad);
constexpr int kTensorTile = 32;
// the kernel sum at the points of the tensor faces as matrix products over
// the sources (matrix cores): FP32 for the far chunks, FP64 for the near
// chunks, the same chunks and partial layout as launch_sum
void launch_sum_tensor(hipStream_t st, const SumPlan &pl, const PathTab &tab, const TensorArgs &a);

// reduce chunk partials; T, grad; per-point load density:
//   NEUMANN: -k (grad . n) w dS,  DIRICHLET: -T~ w dS,  else 0
// outputs of slot s go to index o = (by_slot ? s : path[s]): T + o*ostride,
// grad + o*3*ostride (component-major), ld + o*ostride.  Slots with mode 1
// add the network's far field net[(s*4 + c) * net_stride + q] (c = 0: T,
// 1..3: gradient) before the densities are formed.
void launch_finalize(hipStream_t st, const PathTab &tab, bool by_slot, int64_t nq, int n_chunks,
                     int64_t part_stride, const double *part, const double *px, const double *py,
                     const double *pz, const double *nx, const double *ny, const double *nz, const double *wdS,
                     const int8_t *role, double kcond, int64_t ostride, double *T, double *g, double *ld,
                     const double *net, int64_t net_stride);

// net heat-loss rate at n edge points: grad T^ = sum_e (gx, gy, gz)[e] u[col[e]]
// over the CSR row of each point, q~ = -k G . n (G [3][gstride], the source
// field's gradient), q^ = -k grad T^ . n (nrm [n][3]); qt, qh [n]; the
// integrands |q~ + q^| ds and |q~| ds in fnet, ftil [n] and their sums, in a
// fixed order, in integrals [2]
void launch_heat_loss(hipStream_t st, int64_t n, const int64_t *rowptr, const int32_t *col, const double *gx,
                      const double *gy, const double *gz, const double *u, const double *G, int64_t gstride,
                      const double *nrm, const double *ds, double kcond, double *qt, double *qh, double *fnet,
                      double *ftil, double *integrals);

// out[r] = sum_e val[e] * in[col[e]] over rows [0, nrow) of a CSR
void launch_gather(hipStream_t st, int64_t nrow, const int64_t *rowptr, const int32_t *col,
                   const double *val, const double *in, double *out);

// ---- solver --------------------------------------------------------------
struct PcgScalars {
  double bnorm2;          // |b_free|^2
  double rz;              // r . z
  double rr;              // r . r (latest)
  double alpha, beta;
  int32_t iter;
  int32_t done;           // 1 = converged, 2 = breakdown
  double rtol2;           // rtol^2
  int32_t pad[2];
};

struct StencilOp {
  int n[3];
  int hw[3];
  int n_off;
  int64_t nrow;
  const double *A;        // [n_off][nrow]
  const uint8_t *free_mask;  // 1 = unknown row (NULL: all free)
};

struct CsrOp {
  int64_t nrow;
  const int64_t *rowptr;
  const int32_t *col;
  const double *val;
};

struct FdOp {
  int n[3], lo[3], m[3];
  const double *U[3];
  const double *inv_diag;
  double *t1, *t2;        // scratch [m0 m1 m2]
};

// theta-scheme initial residual:
//   rhs = B v + theta F1 + (1-theta) F0 on free rows; x = v with fixed rows
//   replaced by vD (scattered from dir_val over dir_dofs); r = rhs - A x on
//   free rows, 0 on fixed rows; partials of |rhs_free|^2.
void launch_theta_init(hipStream_t st, const StencilOp &A, const double *Bval, const double *v,
                       const double *F1, const double *F0, double theta, double *x, double *r,
                       double *part);
void launch_scatter_dirichlet(hipStream_t st, int64_t nD, const int64_t *dofs, const double *vals,
                              double *x);

// generic PCG pieces (operator is either a stencil or a CSR)
void launch_csr_init(hipStream_t st, const CsrOp &A, const double *b, const double *x, double *r,
                     double *part);
void launch_jacobi(hipStream_t st, int64_t n, const double *inv_diag, const double *r, double *z,
                   double *part, PcgScalars *sc);
void launch_fd(hipStream_t st, const FdOp &F, int64_t n, const double *r, double *z, double *part,
               PcgScalars *sc);
// several FD solves in the same launches: solve b reads the full vector
// r + off[b] (its grid n[0] n[1] n[2]) and writes the entries of its box in
// z + off[b]; the other entries of z are not written (the caller zeroes them
// once).  With gidx set (only where fd_batch_in_lds holds), solve b reads
// entry k of its grid as r[gidx[off[b] + k]] (0 where that is negative)
// instead: r is then the vector of the whole system, gathered on the fly.
constexpr int kFdBatchMax = 8;
struct FdBatch {
  int count;
  FdOp f[kFdBatchMax];
  int64_t off[kFdBatchMax];
  const int64_t *gidx;
};
bool fd_batch_in_lds(const FdBatch &B);
void launch_fd_batch(hipStream_t st, const FdBatch &B, const double *r, double *z, const PcgScalars *sc);
void launch_pcg_start(hipStream_t st, int64_t n, int n_part_b, const double *part_b, int n_part_rz,
                      const double *part_rz, const double *z, double *p, PcgScalars *sc, double rtol);
void launch_stencil_apply_dot(hipStream_t st, const StencilOp &A, const double *p, double *q, double *part,
                              PcgScalars *sc);
void launch_csr_apply_dot(hipStream_t st, const CsrOp &A, const double *p, double *q, double *part,
                          PcgScalars *sc);
// alpha = rz / sum(part_pq); x += alpha p; r -= alpha q; partials of r.r
// (rz = sum(part_rz), the partials of the last preconditioning, n_part_rz of
// them; stored in sc for the direction update that follows)
void launch_pcg_update(hipStream_t st, int64_t n, int n_part, const double *part_pq, int n_part_rz,
                       const double *part_rz, const double *p, const double *q, double *x, double *r,
                       double *part_rr, PcgScalars *sc);
// convergence check on sum(part_rr); beta = sum(part_rz)/rz; p = z + beta p
void launch_pcg_direction(hipStream_t st, int64_t n, int n_part_rr, int n_part_rz, const double *part_rr,
                          const double *part_rz, const double *z, double *p, PcgScalars *sc);

int parts_for(int64_t n);      // number of partials produced by a vector kernel over n rows

// point evaluation: out[i] = sum_e val[e] * u[col[e]] + add
void launch_csr_eval(hipStream_t st, int64_t nrow, const int64_t *rowptr, const int32_t *col,
                     const double *val, const double *u, double *out);

}  // namespace sa
