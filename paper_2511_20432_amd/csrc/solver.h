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

// paths of one batched launch: slot s works on path path[s]
struct SlotMap {
  int count;
  int32_t path[kMaxBatch];
};

// load-vector gather over the non-empty rows of the transpose CSR
struct GatherRows {
  int64_t nrows;
  const int32_t *rows;       // DOF of each non-empty row
  const int64_t *rowptr;
  const int32_t *col;        // boundary point
  const double *val;         // R_A(x_q)
};
// per slot (path p): F[p*fs + rows[r]] = sum val * ld[p*ls + col]; x[p*fs + i] = v[p*fs + i], i < ncopy
void launch_gather_rows(hipStream_t st, const SlotMap &sm, const GatherRows &g, const double *ld, int64_t ls,
                        double *F, int64_t fs, int64_t ncopy, const double *v, double *x);

// two gathers of the same densities in one launch: F1 from g1, F2 from g2
void launch_gather_rows2(hipStream_t st, const SlotMap &sm, const GatherRows &g1, double *F1, int64_t fs1,
                         const GatherRows &g2, double *F2, int64_t fs2, const double *ld, int64_t ls);

// per slot (path p): x[p*n + i] = v[p*n + i] for the free DOFs i (mask[i] != 0);
// the entries of the Dirichlet DOFs of x are left as they are
void launch_copy_free(hipStream_t st, const SlotMap &sm, int64_t n, const uint8_t *mask, const double *v,
                      double *x);

// Dirichlet projection solved by one workgroup
struct DirArgs {
  int nD;
  const double *b;                            // projection right-hand side (gathered)
  int u_in_lds;                               // stage Ua, Ub in LDS
  const int64_t *mrow;  const int32_t *mcol;  const double *mval;   // trace mass matrix
  int fd;                                     // 1: Kronecker FD, 0: Jacobi
  int na, nb;
  const double *Ua, *Ub, *inv, *jacobi;
  double *vD;                                 // in: warm start, out: values (stride nD per path)
  const int64_t *dofs;                        // DOF of each Dirichlet value
  double *xfull;                              // theta-step iterates: receive the values
  int64_t xs;                                 // stride of xfull per path
  double rtol2;
  int max_iter;
  SolveStatus *status;
};
bool dirichlet_fits(int64_t nD);
size_t dirichlet_lds(const DirArgs &a);
void launch_dirichlet(hipStream_t st, const SlotMap &sm, const DirArgs &a);

// banded stencil product (theta-step residual or A p)
struct SlArgs {
  int64_t nrow;
  int64_t vs;             // stride per path of x, v, F1, F0, out
  int np;                 // partials per path (= stencil_blocks(nrow))
  int n0, n1, hw1, hw2;
  const double *A, *B;
  const uint8_t *mask;
  const double *x;        // iterate (theta) or p (apply)
  const double *v;        // u^n (theta)
  const double *F1, *F0;
  double theta;
  double *out;            // r (theta) or q (apply)
  double *part;           // |rhs|^2 (theta) or p.q (apply), one per block
  const PcgScalars *sc;   // apply: skip when done (one per path)
  PcgScalars *sc_w;       // theta: resets the done flags (one per path)
};
int stencil_blocks(int64_t nrow);
void launch_stencil_sl(hipStream_t st, const SlotMap &sm, const SlArgs &a, int hw0, bool theta);

// Matrix-free theta-scheme operators on an affine axis-aligned patch, where
//   A = cM (M2 x M1 x M0) + sum_d cA[d] K_d-term,  B = cM (M2 x M1 x M0) + sum_d cB[d] K_d-term,
//   K_0-term = M2 x M1 x K0, K_1-term = M2 x K1 x M0, K_2-term = K2 x M1 x M0
// with banded 1-D factors (band[d][i][k] = factor[i][i - p_d + k]).  Applied in
// three passes (x, y, z), each a banded product along one axis, through the
// scratch t (8 vectors per path, 10 with the residual check).  Same outputs
// and partials as launch_stencil_sl (theta: r = B v + theta F1 + (1-theta) F0 - A x on the
// free rows, partial sums of rhs^2; apply: q = A p, partial sums of p.q; one
// partial per 64 rows).
struct KronOp {
  int n[3], p[3];
  const double *Mb[3], *Kb[3];
  double cM, cA[3], cB[3];
};
struct KronArgs {
  KronOp op;
  int64_t nrow, vs;       // stride per path of x, v, F1, F0, out
  int np;                 // partials per path
  const uint8_t *mask;
  const double *x, *v, *F1, *F0;
  double theta;
  double *t;  int64_t ts; // scratch, stride per path (>= 8 nrow; 10 nrow with check)
  double *out, *part;
  const PcgScalars *sc;   // apply: skip when done
  PcgScalars *sc_w;       // theta: resets the done flags
  int init_x;             // theta: form the first iterate x = v on the free DOFs (mask) in the x pass
  double *x_init;         // ... writable alias of x
  // theta, checked update: also r_prev = bprev - A v on the free rows (the
  // residual of the step that produced v = u^n, whose right-hand side bprev
  // holds), with partials of |r_prev|^2, |bprev|^2, |v|^2 in
  // part_chk[(p * 3 + c) * np + wave]; then bprev <- this step's right-hand side.
  // check_only: those partials alone (no other output).  t needs 10 nrow.
  int check, check_only;
  double *bprev;          // [paths][vs]
  double *part_chk;       // [paths][3][np]
  // theta: F1 / F0 of launch slot s at F1 + s * f1s (f1_slot) instead of at
  // F1 + path * vs; the same for F0
  int f1_slot, f0_slot;
  int64_t f1s, f0s;
  // theta with init_x: the Dirichlet values of u^{n+1} taken from dv (slot s
  // at dv + s * dvs, value didx[i] for DOF i) into x in the x pass
  const double *dv;
  int64_t dvs;
  const int32_t *didx;
};
void launch_kron(hipStream_t st, const SlotMap &sm, const KronArgs &a, bool theta);
// status records from the check partials of KronArgs (check_only pass): one
// block per slot, record at status + slot
void launch_check_status(hipStream_t st, const SlotMap &sm, const double *part_chk, int np, double rtol2,
                         double bw2, SolveStatus *status);

// fused PCG with the fast-diagonalisation preconditioner on the free box
// Per-path data of path p: x, r, z, p, q at + p*vs; t at + p*ts; partials
// part_rz at + p*2*np_rz, part_rr at + p*np_rz, part_pq at + p*np_pq,
// part_b at + p*np_b; sc at + p; status at + slot; scatter_out at + p*sos.
struct FusedPcg {
  int n[3], lo[3], m[3];
  const double *U0, *U1, *U2, *inv;
  const double *U0T;      // optional: U0 transposed (coalesced back transform; same sums)
  double *x, *r, *z, *p, *q, *t;
  int64_t vs, ts;
  double *part_rz;        // [2][np_rz] per path
  double *part_rr;        // [np_rz] per path
  double *part_xx;        // [np_rz] per path: |x|^2 on the box (attainable-accuracy test)
  const double *part_pq;  int np_pq;
  const double *part_b;   int np_b;
  int np_rz;              // = m[1] m[2] (one partial per x-fiber)
  double rtol2;
  double bw2;             // (64 eps |A|_inf)^2: also converged when |r|^2 <= bw2 |x|^2
  PcgScalars *sc;
  SolveStatus *status;
  const int64_t *scatter_idx;   // optional: scatter_out[scatter_idx[g]] = z[g]
  double *scatter_out;
  int64_t sos;
  // checked update (one FD application, x += P r): k_fd_xbwd adds z to x on
  // the box instead of writing z and p; k_fd_xfwd's first block of a path
  // writes the status record of the previous step's check when bit s of
  // check_mask is set (slot s), else a record that there was none
  int update_x;
  uint64_t check_mask;
  const double *part_chk; int np_chk;   // as in KronArgs, per path
  double chk_rtol2, chk_bw2;
};
bool fused_fits(const int m[3]);
// Checked update of a theta-step on a Kronecker operator with the exact FD
// solve (u^{n+1} = x0 + P r0), in two launches sequences:
//   rhs:   the x and y passes of the right-hand side (a: theta arguments with
//          check), the z pass fused with the first FD transform into f.t (r
//          is not stored; the residual-check partials, zx_blocks(op) per kind
//          and path, go to a.part_chk)
//   solve: the plane transforms, whose first block writes the status record
//          of the previous step's residual check (f.update_x, check_mask,
//          part_chk, np_chk = zx_blocks(op)), and the last transform, which
//          adds P r0 to x
bool zx_fits(int n0);
int zx_blocks(const KronOp &op);
void launch_theta_checked_rhs(hipStream_t st, const SlotMap &sm, const KronArgs &a, const FusedPcg &f,
                              bool with_x = true);
void launch_theta_checked_solve(hipStream_t st, const SlotMap &sm, const FusedPcg &f, bool with_xbwd = true);
// the last FD transform of a checked step n (f: x = u^{n+1} being formed) and
// the x pass of step n+1's right-hand side (a: its theta arguments with
// init_x; v = u^{n+1}), fused per x-row: what launch_theta_checked_solve's
// last launch and launch_theta_checked_rhs's first do, with the same sums
void launch_xbwd_x(hipStream_t st, const SlotMap &sm, const FusedPcg &f, const KronArgs &a);
// LDS bytes of the plane pass of the FD solve (two planes, the y and z eigenvectors)
size_t fd_plane_lds(const int m[3]);
void launch_fd_pass(hipStream_t st, const SlotMap &sm, const FusedPcg &f, int k, bool first, bool update);
// convergence test and p = z + beta p; `last` (the final iteration of a fixed
// budget) records the status without updating p
void launch_pcg_dir(hipStream_t st, const SlotMap &sm, const FusedPcg &f, int k, bool last);
// the final iteration's x, r update and |r|^2 partials, without the
// preconditioned residual (nothing uses it)
void launch_pcg_last_update(hipStream_t st, const SlotMap &sm, const FusedPcg &f, int k);

// Dirichlet projection solved exactly: vD = inv_area (Ib x Ia) b with the dense
// inverses of the two 1-D trace mass factors, one workgroup per path; the
// values are also scattered into the theta-step iterate (xfull[dofs[i]])
struct DirDirect {
  int na, nb;
  const double *Ia, *Ib;   // na x na, nb x nb (symmetric)
  double inv_area;
  const double *b;         // gathered right-hand side, stride vs per path
  double *vD;              // values, stride vs per path
  int64_t vs;
  const int64_t *dofs;
  double *xfull;
  int64_t xs;
  double *tmp;             // optional [path][na nb] scratch: two passes over many workgroups
};
size_t dir_direct_lds(int na, int nb);
// (xfull == nullptr: the values are not scattered)
bool dir_direct_prepare(size_t lds);   // allow that much dynamic LDS for the kernel
void launch_dir_direct(hipStream_t st, const SlotMap &sm, const DirDirect &a);

// per slot s (path p = path[s]) and job j: dst[p * ds + i] = src[s * ss + i], i < n
struct CopyJob {
  const double *src;
  double *dst;
  int64_t n, ss, ds;
};
void launch_copy_jobs(hipStream_t st, const SlotMap &sm, const CopyJob *jobs, int njobs);

}  // namespace sa
