// Fused solver kernels (device code in solver.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace sa {

// per-solve record written by the device (read back lazily by the host)
struct SolveStatus {
  int32_t iter;
  int32_t done;      // 1 converged, 2 breakdown, 0 not converged within budget
  double relres2;    // |r|^2 / |b|^2 at exit
};

// load-vector gather over the non-empty rows of the transpose CSR
struct GatherRows {
  int64_t nrows;
  const int32_t *rows;       // DOF of each non-empty row
  const int64_t *rowptr;
  const int32_t *col;        // boundary point
  const double *val;         // R_A(x_q)
};
void launch_gather_rows(hipStream_t st, const GatherRows &g, const double *ld, double *F, int64_t ncopy,
                        const double *v, double *x);

// Dirichlet projection solved by one workgroup
struct DirArgs {
  int nD;
  const double *b;                            // projection right-hand side (gathered)
  int u_in_lds;                               // stage Ua, Ub in LDS
  const int64_t *mrow;  const int32_t *mcol;  const double *mval;   // trace mass matrix
  int fd;                                     // 1: Kronecker FD, 0: Jacobi
  int na, nb;
  const double *Ua, *Ub, *inv, *jacobi;
  double *vD;                                 // in: warm start, out: values
  const int64_t *dofs;                        // DOF of each Dirichlet value
  double *xfull;                              // theta-step iterate: receives the values
  double rtol2;
  int max_iter;
  SolveStatus *status;
};
bool dirichlet_fits(int64_t nD);
size_t dirichlet_lds(const DirArgs &a);
void launch_dirichlet(hipStream_t st, const DirArgs &a);

// banded stencil product (theta-step residual or A p)
struct SlArgs {
  int64_t nrow;
  int n0, n1, hw1, hw2;
  const double *A, *B;
  const uint8_t *mask;
  const double *x;        // iterate (theta) or p (apply)
  const double *v;        // u^n (theta)
  const double *F1, *F0;
  double theta;
  double *out;            // r (theta) or q (apply)
  double *part;           // |rhs|^2 (theta) or p.q (apply), one per block
  const PcgScalars *sc;   // apply: skip when done
  PcgScalars *sc_w;       // theta: resets the done flag
};
int stencil_blocks(int64_t nrow);
void launch_stencil_sl(hipStream_t st, const SlArgs &a, int hw0, bool theta);

// fused PCG with the fast-diagonalisation preconditioner on the free box
struct FusedPcg {
  int n[3], lo[3], m[3];
  const double *U0, *U1, *U2, *inv;
  double *x, *r, *z, *p, *q, *t;
  double *part_rz;        // [2][np_rz]
  double *part_rr;        // [np_rz]
  const double *part_pq;  int np_pq;
  const double *part_b;   int np_b;
  int np_rz;              // = m[1] m[2] (one partial per x-fiber)
  double rtol2;
  PcgScalars *sc;
  SolveStatus *status;
  const int64_t *scatter_idx;   // optional: scatter_out[scatter_idx[g]] = z[g]
  double *scatter_out;
};
bool fused_fits(const int m[3]);
void launch_fd_pass(hipStream_t st, const FusedPcg &f, int k, bool first, bool update);
void launch_pcg_dir(hipStream_t st, const FusedPcg &f, int k);

}  // namespace sa
