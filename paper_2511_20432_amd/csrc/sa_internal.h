// Internal declarations of the sa_iga library (host side).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "sa_iga.h"

namespace sa {

constexpr int kMaxDeg = 6;
constexpr int kMaxLocal = (kMaxDeg + 1) * (kMaxDeg + 1) * (kMaxDeg + 1);

struct SaError {
  int code;
  std::string msg;
};

// One knot vector with its non-empty intervals (elements).
struct Basis1D {
  int p = 0, n = 0;
  std::vector<double> t;
  std::vector<int> span;           // per element: index s of [t_s, t_{s+1})
  int n_el() const { return (int)span.size(); }
  // values N[0..p] and first derivatives dN[0..p] of the functions s-p..s at xi
  void eval(int s, double xi, double *N, double *dN) const;
  int find_span(double xi) const;  // span index holding xi (closed at the right end)
};

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);  // on [-1, 1]

struct PatchData {
  Basis1D b[3];
  int n[3] = {0, 0, 0};
  int64_t ndof = 0;
  std::vector<double> ctrl;        // [n2][n1][n0][4]
  int role[6];
  int qv[3], qf;
  double center[3];                // bounding-box centre of the control net (m)
};

// Basis, geometry and Jacobian at one parametric point.
struct PointEval {
  int L = 0;
  int64_t idx[kMaxLocal];
  int loc[kMaxLocal][3];
  double R[kMaxLocal];
  double dR[kMaxLocal][3];
  double x[3];
  double J[3][3];                  // J[i][j] = dx_i / dxi_j
};

void eval_point(const PatchData &P, const double xi[3], const int span[3], PointEval &out);

// inverse of the geometry map: the parametric point xi of the physical point
// x, from the nearest element centre by Newton steps kept in [0,1]^3, to
// |x - x(xi)| <= tol; false if x is not reached (outside the patch)
bool locate_point(const PatchData &P, const std::vector<double> &centres, const std::vector<double> &cxi,
                  const double x[3], double tol, double xi[3]);
void element_centres(const PatchData &P, std::vector<double> &centres, std::vector<double> &cxi);
double locate_tolerance(const PatchData &P);   // 1e-13 of the control net's extent
// Gauss points (quad per element) of the edge where parametric face `face`
// meets face `edge_face`: parametric points xi [n][3], the outward unit
// normals of `face` [n][3], arc-length weights ds [n]; returns n
int64_t edge_points(const PatchData &P, int face, int edge_face, int quad, std::vector<double> &xi,
                    std::vector<double> &nrm, std::vector<double> &ds);

// Banded matrix on the control-point grid: row A, offset o <-> (d0, d1, d2)
// in [-hw0, hw0] x [-hw1, hw1] x [-hw2, hw2], value val[o * nrow + A].
struct Stencil {
  int n[3] = {0, 0, 0};
  int hw[3] = {0, 0, 0};
  int n_off = 0;
  int64_t nrow = 0;
  std::vector<double> val;
  void init(const int n_[3], const int hw_[3]);
  int off_index(int d0, int d1, int d2) const {
    return (d0 + hw[0]) + (2 * hw[0] + 1) * ((d1 + hw[1]) + (2 * hw[1] + 1) * (d2 + hw[2]));
  }
  void apply(const double *x, double *y) const;   // host y = S x
};

struct Csr {
  int64_t nrow = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

struct BoundaryTables {
  int64_t nq = 0;
  int64_t face_off[7];
  std::vector<double> x, nrm;      // [nq][3]
  std::vector<double> wdS;         // [nq]
  std::vector<int8_t> role;        // face role of each point
  // non-zero functions of every point (the face layer), CSR by point
  std::vector<int64_t> fptr;
  std::vector<int64_t> fidx;
  std::vector<double> fval;
};

// Fast-diagonalisation data of a Kronecker operator
//   P = cM (M2 x M1 x M0) + c0 (M2 x M1 x K0) + c1 (M2 x K1 x M0) + c2 (K2 x M1 x M0)
// on the box of free indices [lo_d, lo_d + m_d) of an n0 x n1 x n2 grid.
struct FdData {
  int n[3] = {1, 1, 1};
  int lo[3] = {0, 0, 0};
  int m[3] = {1, 1, 1};
  std::vector<double> U[3];        // m_d x m_d, row-major U[k * m + j]
  std::vector<double> inv_diag;    // [m2][m1][m0]
};

struct Model {
  PatchData P;
  sa_material mat;
  sa_solver_options opt;
  double dt = 0;
  Stencil M, K;                    // Eqs. 16-17
  double mean_detJ = 0, mean_metric[3] = {0, 0, 0};
  BoundaryTables bt;
  Csr load;                        // rows = DOFs, cols = NEUMANN points, val = R_A(x_q)
  std::vector<int64_t> dir_dofs;   // sorted
  std::vector<uint8_t> free_mask;  // 1 = unknown, 0 = Dirichlet
  Csr dproj;                       // rows = Dirichlet DOFs, cols = DIRICHLET points, val = R_A(x_q)
  Csr mass_dir;                    // trace mass matrix on the Dirichlet DOFs
  FdData fd_main, fd_dir;
  std::vector<double> M1[3], K1[3];  // 1-D parametric mass / stiffness (volume rule), n_d x n_d
  bool fd_dir_ok = false;
  int free_box_ok = 0;             // Dirichlet set is a union of end layers (box of free DOFs)
};

// interfaces: SA_FACE_INTERFACE is a valid face role (patches of a multi-patch model)
void validate_inputs(const sa_patch *patch, const sa_material *mat, const sa_scan_path *scan,
                     const sa_solver_options &opt, bool interfaces = false);
void load_patch(const sa_patch *patch, PatchData &P);
void assemble_volume(Model &m);
void build_boundary(Model &m);       // faces with role SA_FACE_INTERFACE get no points
void build_transfer(const BoundaryTables &bt, int64_t nd, const std::vector<uint8_t> &free_mask, Csr &load,
                    std::vector<int64_t> &dir_dofs, Csr &dproj, Csr &mass_dir);
void build_fd(Model &m);
void fd_apply_host(const FdData &F, const double *r, double *z, int64_t n_full);

// chunking of the kernel sum's source history for nq points and count paths
// whose longest far and near histories are max_far and max_near sources
struct SumPlan;
SumPlan plan_sum(const sa_solver_options &o, int64_t nq, int count, int64_t max_far, int64_t max_near);

// parameters of the far-history network (layout in mlp.h)
constexpr int64_t kNetParams = 256 * 70 + 256 + 3 * (256 * 256 + 256) + 4 * 256 + 4;

// message of the last failure on this thread (read by sa_iga_last_error)
void set_last_error(const std::string &msg);
double fd_inverse_defect(const FdData &F, const Stencil &S, const std::vector<double> &Sval,
                         const std::vector<uint8_t> &free_mask);

}  // namespace sa
