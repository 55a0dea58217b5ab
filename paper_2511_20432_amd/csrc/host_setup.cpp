// Host-side set-up of the isogeometric model (paper Sec. 2.3): spline basis,
// Gauss rules, mass and conductivity matrices (Eqs. 16-17) in banded
// stencil form, boundary quadrature tables (Eq. 18), Dirichlet trace data
// (Eq. 11) and the fast-diagonalisation preconditioner.  Runs once per
// object; the mesh is fixed for the whole simulation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <thread>

#include "kernels.h"
#include "sa_internal.h"

namespace sa {

static void fail(int code, const std::string &msg) { throw SaError{code, msg}; }

// ---------------------------------------------------------------------------
// 1-D B-splines: Cox-de Boor recursion on the p+1 functions of one span.
// ---------------------------------------------------------------------------
int Basis1D::find_span(double xi) const {
  // last s with t_s <= xi < t_{s+1}; xi = t_end goes to the last element
  if (xi >= t[n]) return n - 1;
  int lo = p, hi = n;  // t[lo] <= xi < t[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (xi < t[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

void Basis1D::eval(int s, double xi, double *N, double *dN) const {
  double left[kMaxDeg + 2], right[kMaxDeg + 2];
  double Nm1[kMaxDeg + 1];  // degree p-1 values of functions s-p+1 .. s
  N[0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    if (j == p) for (int r = 0; r < p; ++r) Nm1[r] = N[r];
    left[j] = xi - t[s + 1 - j];
    right[j] = t[s + j] - xi;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      double den = right[r + 1] + left[j - r];
      double tmp = den != 0.0 ? N[r] / den : 0.0;
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
  if (p == 0) { dN[0] = 0.0; return; }
  // dN_{i,p} = p N_{i,p-1}/(t_{i+p}-t_i) - p N_{i+1,p-1}/(t_{i+p+1}-t_{i+1}), i = s-p+r
  for (int r = 0; r <= p; ++r) {
    int i = s - p + r;
    double a = 0.0, b = 0.0;
    if (r >= 1) {
      double den = t[i + p] - t[i];
      if (den != 0.0) a = Nm1[r - 1] / den;
    }
    if (r <= p - 1) {
      double den = t[i + p + 1] - t[i + 1];
      if (den != 0.0) b = Nm1[r] / den;
    }
    dN[r] = p * (a - b);
  }
}

// Gauss-Legendre nodes by Newton's method on P_n (three-term recurrence).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // refresh derivative at the converged node
        p0 = 1.0; p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    x[n - 1 - i] = z;  // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// ---------------------------------------------------------------------------
// validation and patch loading
// ---------------------------------------------------------------------------
void validate_inputs(const sa_patch *patch, const sa_material *mat, const sa_scan_path *scan,
                     const sa_solver_options &opt, bool interfaces) {
  if (!patch || !mat || !scan) fail(SA_EINVAL, "NULL patch, material or scan path");
  for (int d = 0; d < 3; ++d) {
    int p = patch->degree[d], n = patch->n_ctrl[d];
    if (p < 1 || p > kMaxDeg) fail(SA_EINVAL, "degree must be in 1..6");
    if (n < p + 1) fail(SA_EINVAL, "n_ctrl must be >= degree + 1");
    if (!patch->knots[d]) fail(SA_EINVAL, "NULL knot vector");
    const double *t = patch->knots[d];
    int m = n + p + 1;
    for (int i = 0; i + 1 < m; ++i)
      if (!(t[i] <= t[i + 1])) fail(SA_EINVAL, "knot vector must be non-decreasing");
    for (int i = 0; i <= p; ++i)
      if (t[i] != 0.0 || t[m - 1 - i] != 1.0) fail(SA_EINVAL, "knot vector must be open on [0, 1]");
    // interior knots repeat at most p times (continuity C^0 or better)
    for (int i = 1; i + p < m - 1; ++i)
      if (!(t[i + p] > t[i])) fail(SA_EINVAL, "interior knot multiplicity must not exceed the degree");
    if (patch->quad_vol[d] < 1 || patch->quad_vol[d] > 16) fail(SA_EINVAL, "quad_vol in 1..16");
  }
  if (patch->quad_face < 1 || patch->quad_face > 16) fail(SA_EINVAL, "quad_face in 1..16");
  if (!patch->ctrl_xyzw) fail(SA_EINVAL, "NULL control net");
  int64_t nd = (int64_t)patch->n_ctrl[0] * patch->n_ctrl[1] * patch->n_ctrl[2];
  for (int64_t i = 0; i < nd; ++i) {
    double w = patch->ctrl_xyzw[4 * i + 3];
    if (!(w > 0.0) || !std::isfinite(w)) fail(SA_EINVAL, "weights must be positive");
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(patch->ctrl_xyzw[4 * i + c])) fail(SA_EINVAL, "non-finite control point");
  }
  const int max_role = interfaces ? SA_FACE_INTERFACE : SA_FACE_SOURCE_PLANE;
  for (int f = 0; f < 6; ++f)
    if (patch->face_role[f] < 0 || patch->face_role[f] > max_role) fail(SA_EINVAL, "bad face role");
  if (!(mat->k > 0) || !(mat->rho > 0) || !(mat->cp > 0) || !std::isfinite(mat->T0))
    fail(SA_EINVAL, "material constants must be positive and finite");
  if (scan->n_paths < 1) fail(SA_EINVAL, "n_paths must be >= 1");
  if (!scan->src_offset || !scan->n_steps) fail(SA_EINVAL, "NULL src_offset or n_steps");
  if (!(scan->dt > 0) || scan->sources_per_step < 1 || !(scan->spot_radius >= 0))
    fail(SA_EINVAL, "dt > 0, sources_per_step >= 1, spot_radius >= 0 required");
  if (scan->src_offset[0] != 0) fail(SA_EINVAL, "src_offset[0] must be 0");
  for (int p = 0; p < scan->n_paths; ++p) {
    if (scan->src_offset[p + 1] < scan->src_offset[p]) fail(SA_EINVAL, "src_offset must be non-decreasing");
    if (scan->n_steps[p] < 0) fail(SA_EINVAL, "n_steps must be >= 0");
  }
  int64_t N = scan->src_offset[scan->n_paths];
  if (N > 0 && (!scan->xyz || !scan->tick || !scan->energy)) fail(SA_EINVAL, "NULL source arrays");
  for (int p = 0; p < scan->n_paths; ++p) {
    for (int64_t i = scan->src_offset[p]; i < scan->src_offset[p + 1]; ++i) {
      if (scan->tick[i] < 1) fail(SA_EINVAL, "ticks must be >= 1");
      if (i > scan->src_offset[p] && scan->tick[i] < scan->tick[i - 1])
        fail(SA_EINVAL, "ticks must be non-decreasing within a path");
      if (!std::isfinite(scan->energy[i]) || !std::isfinite(scan->xyz[3 * i]) ||
          !std::isfinite(scan->xyz[3 * i + 1]) || !std::isfinite(scan->xyz[3 * i + 2]))
        fail(SA_EINVAL, "non-finite source data");
    }
  }
  if (!(opt.theta >= 0.0 && opt.theta <= 1.0)) fail(SA_EINVAL, "theta must be in [0, 1]");
  if (opt.precision < 0 || opt.precision > 2) fail(SA_EINVAL, "precision must be an sa_precision value");
  if (opt.precision == SA_PREC_SURROGATE) {
    if (!opt.surrogate_weights) fail(SA_EINVAL, "SA_PREC_SURROGATE needs surrogate_weights");
    if (opt.surrogate_len != 3 + kNetParams)
      fail(SA_EINVAL, "surrogate_len must be 3 + sa_mlp_n_params()");
    for (int64_t i = 0; i < opt.surrogate_len; ++i)
      if (!std::isfinite(opt.surrogate_weights[i])) fail(SA_EINVAL, "non-finite surrogate weight");
    if (!(opt.surrogate_weights[0] > 0) || !(opt.surrogate_weights[1] > 0) || !(opt.surrogate_weights[2] > 0))
      fail(SA_EINVAL, "surrogate scales must be positive");
    if (opt.audit_every < 1) fail(SA_EINVAL, "audit_every must be >= 1");
    if (!(opt.audit_frac > 0 && opt.audit_frac <= 1)) fail(SA_EINVAL, "audit_frac must be in (0, 1]");
    if (!(opt.audit_tol >= 0)) fail(SA_EINVAL, "audit_tol must be >= 0");
  }
  if (!(opt.pcg_rtol > 0) || opt.pcg_max_iter < 1) fail(SA_EINVAL, "bad PCG options");
  if (opt.preconditioner < 0 || opt.preconditioner > 1) fail(SA_EINVAL, "bad preconditioner");
  if (!(opt.tau_near >= 0)) fail(SA_EINVAL, "tau_near must be >= 0");
  if (!(opt.kernel_scale >= 0) || !std::isfinite(opt.kernel_scale)) fail(SA_EINVAL, "bad kernel_scale");
  if (opt.points_per_lane != 0 && opt.points_per_lane != 1 && opt.points_per_lane != 2 &&
      opt.points_per_lane != 4)
    fail(SA_EINVAL, "points_per_lane must be 0, 1, 2 or 4");
  if (opt.waves_per_group != 0 && opt.waves_per_group != 1 && opt.waves_per_group != 2 &&
      opt.waves_per_group != 4 && opt.waves_per_group != 8)
    fail(SA_EINVAL, "waves_per_group must be 0, 1, 2, 4 or 8");
  if (opt.chunk_sources < 0) fail(SA_EINVAL, "chunk_sources must be >= 0");
}

void load_patch(const sa_patch *patch, PatchData &P) {
  for (int d = 0; d < 3; ++d) {
    Basis1D &b = P.b[d];
    b.p = patch->degree[d];
    b.n = patch->n_ctrl[d];
    b.t.assign(patch->knots[d], patch->knots[d] + b.n + b.p + 1);
    b.span.clear();
    for (int s = b.p; s < b.n; ++s)
      if (b.t[s + 1] > b.t[s]) b.span.push_back(s);
    P.n[d] = b.n;
    P.qv[d] = patch->quad_vol[d];
  }
  P.qf = patch->quad_face;
  P.ndof = (int64_t)P.n[0] * P.n[1] * P.n[2];
  P.ctrl.assign(patch->ctrl_xyzw, patch->ctrl_xyzw + 4 * P.ndof);
  for (int f = 0; f < 6; ++f) P.role[f] = patch->face_role[f];
  for (int c = 0; c < 3; ++c) {
    double lo = 1e300, hi = -1e300;
    for (int64_t i = 0; i < P.ndof; ++i) {
      lo = std::min(lo, P.ctrl[4 * i + c]);
      hi = std::max(hi, P.ctrl[4 * i + c]);
    }
    P.center[c] = 0.5 * (lo + hi);
  }
}

// ---------------------------------------------------------------------------
// NURBS basis, geometry and Jacobian at one point (isoparametric map, Eq. 14)
// ---------------------------------------------------------------------------
void eval_point(const PatchData &P, const double xi[3], const int span[3], PointEval &o) {
  double N[3][kMaxDeg + 1], dN[3][kMaxDeg + 1];
  for (int d = 0; d < 3; ++d) P.b[d].eval(span[d], xi[d], N[d], dN[d]);
  const int p0 = P.b[0].p, p1 = P.b[1].p, p2 = P.b[2].p;
  const int n0 = P.n[0], n1 = P.n[1];
  int L = 0;
  double W = 0.0, dW[3] = {0, 0, 0};
  double B[kMaxLocal], dB[kMaxLocal][3], w[kMaxLocal];
  for (int l2 = 0; l2 <= p2; ++l2)
    for (int l1 = 0; l1 <= p1; ++l1)
      for (int l0 = 0; l0 <= p0; ++l0) {
        int a0 = span[0] - p0 + l0, a1 = span[1] - p1 + l1, a2 = span[2] - p2 + l2;
        int64_t A = a0 + (int64_t)n0 * (a1 + (int64_t)n1 * a2);
        o.idx[L] = A;
        o.loc[L][0] = l0; o.loc[L][1] = l1; o.loc[L][2] = l2;
        w[L] = P.ctrl[4 * A + 3];
        B[L] = N[0][l0] * N[1][l1] * N[2][l2];
        dB[L][0] = dN[0][l0] * N[1][l1] * N[2][l2];
        dB[L][1] = N[0][l0] * dN[1][l1] * N[2][l2];
        dB[L][2] = N[0][l0] * N[1][l1] * dN[2][l2];
        W += w[L] * B[L];
        for (int j = 0; j < 3; ++j) dW[j] += w[L] * dB[L][j];
        ++L;
      }
  o.L = L;
  for (int i = 0; i < 3; ++i) {
    o.x[i] = 0.0;
    for (int j = 0; j < 3; ++j) o.J[i][j] = 0.0;
  }
  const double iW = 1.0 / W, iW2 = iW * iW;
  for (int l = 0; l < L; ++l) {
    o.R[l] = w[l] * B[l] * iW;
    for (int j = 0; j < 3; ++j) o.dR[l][j] = w[l] * (dB[l][j] * W - B[l] * dW[j]) * iW2;
    const double *Pc = &P.ctrl[4 * o.idx[l]];
    for (int i = 0; i < 3; ++i) {
      o.x[i] += o.R[l] * Pc[i];
      for (int j = 0; j < 3; ++j) o.J[i][j] += o.dR[l][j] * Pc[i];
    }
  }
}

static double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

static void inv3(const double J[3][3], double det, double Ji[3][3]) {
  double id = 1.0 / det;
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
}

// ---------------------------------------------------------------------------
// stencil matrices
// ---------------------------------------------------------------------------
void Stencil::init(const int n_[3], const int hw_[3]) {
  for (int d = 0; d < 3; ++d) { n[d] = n_[d]; hw[d] = hw_[d]; }
  n_off = (2 * hw[0] + 1) * (2 * hw[1] + 1) * (2 * hw[2] + 1);
  nrow = (int64_t)n[0] * n[1] * n[2];
  val.assign((size_t)n_off * nrow, 0.0);
}

void Stencil::apply(const double *x, double *y) const {
  for (int64_t A = 0; A < nrow; ++A) {
    int a0 = (int)(A % n[0]), a1 = (int)((A / n[0]) % n[1]), a2 = (int)(A / ((int64_t)n[0] * n[1]));
    double s = 0.0;
    for (int d2 = -hw[2]; d2 <= hw[2]; ++d2) {
      int b2 = a2 + d2;
      if (b2 < 0 || b2 >= n[2]) continue;
      for (int d1 = -hw[1]; d1 <= hw[1]; ++d1) {
        int b1 = a1 + d1;
        if (b1 < 0 || b1 >= n[1]) continue;
        for (int d0 = -hw[0]; d0 <= hw[0]; ++d0) {
          int b0 = a0 + d0;
          if (b0 < 0 || b0 >= n[0]) continue;
          int64_t B = b0 + (int64_t)n[0] * (b1 + (int64_t)n[1] * b2);
          s += val[(size_t)off_index(d0, d1, d2) * nrow + A] * x[B];
        }
      }
    }
    y[A] = s;
  }
}

// ---------------------------------------------------------------------------
// volume matrices (Eqs. 16-17): elements coloured by z-slab so that threads
// never write the same row
// ---------------------------------------------------------------------------
void assemble_volume(Model &m) {
  PatchData &P = m.P;
  const int hw[3] = {P.b[0].p, P.b[1].p, P.b[2].p};
  m.M.init(P.n, hw);
  m.K.init(P.n, hw);
  const double rc = m.mat.rho * m.mat.cp, kc = m.mat.k;
  std::vector<double> gx[3], gw[3];
  for (int d = 0; d < 3; ++d) gauss_legendre(P.qv[d], gx[d], gw[d]);
  const int ne0 = P.b[0].n_el(), ne1 = P.b[1].n_el(), ne2 = P.b[2].n_el();
  const int ncol = P.b[2].p + 1;
  unsigned nthr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<double> acc_det(nthr, 0.0), acc_met(3 * nthr, 0.0);

  auto work_slab = [&](int e2, int tid) {
    std::vector<double> Me(kMaxLocal * kMaxLocal), Ke(kMaxLocal * kMaxLocal);
    PointEval pe;
    for (int e1 = 0; e1 < ne1; ++e1)
      for (int e0 = 0; e0 < ne0; ++e0) {
        const int e[3] = {e0, e1, e2};
        int span[3];
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
          span[d] = P.b[d].span[e[d]];
          lo[d] = P.b[d].t[span[d]];
          hi[d] = P.b[d].t[span[d] + 1];
        }
        int L = 0;
        std::fill(Me.begin(), Me.end(), 0.0);
        std::fill(Ke.begin(), Ke.end(), 0.0);
        for (int q2 = 0; q2 < P.qv[2]; ++q2)
          for (int q1 = 0; q1 < P.qv[1]; ++q1)
            for (int q0 = 0; q0 < P.qv[0]; ++q0) {
              const int q[3] = {q0, q1, q2};
              double xi[3], wq = 1.0;
              for (int d = 0; d < 3; ++d) {
                xi[d] = lo[d] + (hi[d] - lo[d]) * 0.5 * (gx[d][q[d]] + 1.0);
                wq *= gw[d][q[d]] * 0.5 * (hi[d] - lo[d]);
              }
              eval_point(P, xi, span, pe);
              L = pe.L;
              double det = det3(pe.J);
              double Ji[3][3];
              inv3(pe.J, det, Ji);
              double dv = wq * std::fabs(det);
              acc_det[tid] += dv;
              for (int d = 0; d < 3; ++d) {
                double g = 0.0;  // (J^-1 J^-T)_dd
                for (int i = 0; i < 3; ++i) g += Ji[d][i] * Ji[d][i];
                acc_met[3 * tid + d] += dv * g;
              }
              double g[kMaxLocal][3];
              for (int l = 0; l < L; ++l)
                for (int i = 0; i < 3; ++i)
                  g[l][i] = pe.dR[l][0] * Ji[0][i] + pe.dR[l][1] * Ji[1][i] + pe.dR[l][2] * Ji[2][i];
              for (int a = 0; a < L; ++a) {
                const double ra = rc * dv * pe.R[a];
                const double ga0 = kc * dv * g[a][0], ga1 = kc * dv * g[a][1], ga2 = kc * dv * g[a][2];
                double *mrow = &Me[a * L], *krow = &Ke[a * L];
                for (int b = a; b < L; ++b) {
                  mrow[b] += ra * pe.R[b];
                  krow[b] += ga0 * g[b][0] + ga1 * g[b][1] + ga2 * g[b][2];
                }
              }
            }
        // scatter (symmetric)
        for (int a = 0; a < L; ++a)
          for (int b = 0; b < L; ++b) {
            int lo_ = std::min(a, b), hi_ = std::max(a, b);
            double mv = Me[lo_ * L + hi_], kv = Ke[lo_ * L + hi_];
            int d0 = pe.loc[b][0] - pe.loc[a][0], d1 = pe.loc[b][1] - pe.loc[a][1],
                d2 = pe.loc[b][2] - pe.loc[a][2];
            size_t o = (size_t)m.M.off_index(d0, d1, d2) * m.M.nrow + pe.idx[a];
            m.M.val[o] += mv;
            m.K.val[o] += kv;
          }
      }
  };

  for (int color = 0; color < ncol; ++color) {
    std::vector<int> slabs;
    for (int e2 = color; e2 < ne2; e2 += ncol) slabs.push_back(e2);
    std::vector<std::thread> th;
    unsigned nt = std::min<unsigned>(nthr, (unsigned)slabs.size());
    for (unsigned t = 0; t < nt; ++t)
      th.emplace_back([&, t]() {
        for (size_t i = t; i < slabs.size(); i += nt) work_slab(slabs[i], (int)t);
      });
    for (auto &x : th) x.join();
  }
  double det = 0.0, met[3] = {0, 0, 0};
  for (unsigned t = 0; t < nthr; ++t) {
    det += acc_det[t];
    for (int d = 0; d < 3; ++d) met[d] += acc_met[3 * t + d];
  }
  m.mean_detJ = det;  // parametric domain has unit measure: the mean equals the volume
  for (int d = 0; d < 3; ++d) m.mean_metric[d] = met[d];
}

// ---------------------------------------------------------------------------
// boundary tables (Eq. 18) and Dirichlet trace data (Eq. 11)
// ---------------------------------------------------------------------------
// Load gather (rows = DOFs, columns = NEUMANN points), the Dirichlet DOFs
// (free_mask 0, ascending), the projection right-hand side gather (rows =
// Dirichlet DOFs, columns = DIRICHLET points) and the trace mass matrix on
// the Dirichlet DOFs, from the boundary tables of nd DOFs.
void build_transfer(const BoundaryTables &bt, int64_t nd, const std::vector<uint8_t> &free_mask, Csr &L,
                    std::vector<int64_t> &dir_dofs, Csr &Dp, Csr &Md) {
  const int64_t q = bt.nq;
  // load gather: F_A = sum over NEUMANN points of R_A(x_q) * flux density_q
  L.nrow = nd;
  L.rowptr.assign(nd + 1, 0);
  for (int64_t i = 0; i < q; ++i)
    if (bt.role[i] == SA_FACE_NEUMANN)
      for (int64_t e = bt.fptr[i]; e < bt.fptr[i + 1]; ++e) L.rowptr[bt.fidx[e] + 1]++;
  for (int64_t A = 0; A < nd; ++A) L.rowptr[A + 1] += L.rowptr[A];
  L.col.assign(L.rowptr[nd], 0);
  L.val.assign(L.rowptr[nd], 0.0);
  {
    std::vector<int64_t> pos(L.rowptr.begin(), L.rowptr.end() - 1);
    for (int64_t i = 0; i < q; ++i)
      if (bt.role[i] == SA_FACE_NEUMANN)
        for (int64_t e = bt.fptr[i]; e < bt.fptr[i + 1]; ++e) {
          int64_t A = bt.fidx[e];
          L.col[pos[A]] = (int32_t)i;
          L.val[pos[A]] = bt.fval[e];
          pos[A]++;
        }
  }
  dir_dofs.clear();
  std::vector<int64_t> dpos(nd, -1);
  for (int64_t A = 0; A < nd; ++A)
    if (!free_mask[A]) {
      dpos[A] = (int64_t)dir_dofs.size();
      dir_dofs.push_back(A);
    }
  const int64_t nD = (int64_t)dir_dofs.size();
  // projection right-hand side gather and trace mass matrix
  Dp.nrow = nD;
  Dp.rowptr.assign(nD + 1, 0);
  std::vector<std::map<int64_t, double>> mrows(nD);
  for (int64_t i = 0; i < q; ++i) {
    if (bt.role[i] != SA_FACE_DIRICHLET) continue;
    for (int64_t e = bt.fptr[i]; e < bt.fptr[i + 1]; ++e) {
      int64_t j = dpos[bt.fidx[e]];
      if (j < 0) continue;
      Dp.rowptr[j + 1]++;
      for (int64_t e2 = bt.fptr[i]; e2 < bt.fptr[i + 1]; ++e2) {
        int64_t k = dpos[bt.fidx[e2]];
        if (k < 0) continue;
        mrows[j][k] += bt.fval[e] * bt.fval[e2] * bt.wdS[i];
      }
    }
  }
  for (int64_t j = 0; j < nD; ++j) Dp.rowptr[j + 1] += Dp.rowptr[j];
  Dp.col.assign(Dp.rowptr[nD], 0);
  Dp.val.assign(Dp.rowptr[nD], 0.0);
  {
    std::vector<int64_t> pos(Dp.rowptr.begin(), Dp.rowptr.end() - 1);
    for (int64_t i = 0; i < q; ++i) {
      if (bt.role[i] != SA_FACE_DIRICHLET) continue;
      for (int64_t e = bt.fptr[i]; e < bt.fptr[i + 1]; ++e) {
        int64_t j = dpos[bt.fidx[e]];
        if (j < 0) continue;
        Dp.col[pos[j]] = (int32_t)i;
        Dp.val[pos[j]] = bt.fval[e];  // the per-point density already carries w dS
        pos[j]++;
      }
    }
  }
  Md.nrow = nD;
  Md.rowptr.assign(nD + 1, 0);
  Md.col.clear();
  Md.val.clear();
  for (int64_t j = 0; j < nD; ++j) {
    for (auto &kv : mrows[j]) {
      Md.col.push_back((int32_t)kv.first);
      Md.val.push_back(kv.second);
    }
    Md.rowptr[j + 1] = (int64_t)Md.col.size();
  }
}

void build_boundary(Model &m) {
  PatchData &P = m.P;
  BoundaryTables &bt = m.bt;
  std::vector<double> gx, gw;
  gauss_legendre(P.qf, gx, gw);
  bt.x.clear(); bt.nrm.clear(); bt.wdS.clear(); bt.role.clear();
  bt.fptr.assign(1, 0); bt.fidx.clear(); bt.fval.clear();
  int64_t q = 0;
  PointEval pe;
  for (int f = 0; f < 6; ++f) {
    bt.face_off[f] = q;
    if (P.role[f] == SA_FACE_INTERFACE) continue;   // glued to another patch: no points
    const int d = f / 2, side = f % 2;
    int a = (d == 0) ? 1 : 0, b = (d == 2) ? 1 : 2;
    const Basis1D &Ba = P.b[a], &Bb = P.b[b];
    for (int eb = 0; eb < Bb.n_el(); ++eb)
      for (int gb = 0; gb < P.qf; ++gb)
        for (int ea = 0; ea < Ba.n_el(); ++ea)
          for (int ga = 0; ga < P.qf; ++ga) {
            double xi[3];
            int span[3];
            int sa = Ba.span[ea], sb = Bb.span[eb];
            double la = Ba.t[sa], ha = Ba.t[sa + 1], lb = Bb.t[sb], hb = Bb.t[sb + 1];
            xi[a] = la + (ha - la) * 0.5 * (gx[ga] + 1.0);
            xi[b] = lb + (hb - lb) * 0.5 * (gx[gb] + 1.0);
            xi[d] = (double)side;
            span[a] = sa;
            span[b] = sb;
            span[d] = side ? P.b[d].n - 1 : P.b[d].p;
            double wpar = gw[ga] * 0.5 * (ha - la) * gw[gb] * 0.5 * (hb - lb);
            eval_point(P, xi, span, pe);
            double ta[3] = {pe.J[0][a], pe.J[1][a], pe.J[2][a]};
            double tb[3] = {pe.J[0][b], pe.J[1][b], pe.J[2][b]};
            double td[3] = {pe.J[0][d], pe.J[1][d], pe.J[2][d]};
            double c[3] = {ta[1] * tb[2] - ta[2] * tb[1], ta[2] * tb[0] - ta[0] * tb[2],
                           ta[0] * tb[1] - ta[1] * tb[0]};
            double dS = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            double dot = c[0] * td[0] + c[1] * td[1] + c[2] * td[2];
            double sgn = (dot >= 0 ? 1.0 : -1.0) * (side ? 1.0 : -1.0);
            for (int i = 0; i < 3; ++i) {
              bt.x.push_back(pe.x[i]);
              bt.nrm.push_back(sgn * c[i] / dS);
            }
            bt.wdS.push_back(wpar * dS);
            bt.role.push_back((int8_t)P.role[f]);
            const int keep_l = side ? P.b[d].p : 0;
            for (int l = 0; l < pe.L; ++l) {
              if (pe.loc[l][d] != keep_l) continue;
              bt.fidx.push_back(pe.idx[l]);
              bt.fval.push_back(pe.R[l]);
            }
            bt.fptr.push_back((int64_t)bt.fidx.size());
            ++q;
          }
  }
  bt.face_off[6] = q;
  bt.nq = q;

  // Dirichlet DOFs: the end layers of the DIRICHLET faces
  const int64_t nd = P.ndof;
  m.free_mask.assign(nd, 1);
  for (int f = 0; f < 6; ++f) {
    if (P.role[f] != SA_FACE_DIRICHLET) continue;
    const int d = f / 2, side = f % 2, layer = side ? P.n[d] - 1 : 0;
    for (int64_t A = 0; A < nd; ++A) {
      int a[3] = {(int)(A % P.n[0]), (int)((A / P.n[0]) % P.n[1]), (int)(A / ((int64_t)P.n[0] * P.n[1]))};
      if (a[d] == layer) m.free_mask[A] = 0;
    }
  }
  build_transfer(bt, nd, m.free_mask, m.load, m.dir_dofs, m.dproj, m.mass_dir);
  m.free_box_ok = 1;
}

// ---------------------------------------------------------------------------
// fast diagonalisation: generalized eigenpairs of 1-D parametric matrices
// ---------------------------------------------------------------------------
static void param_mats_1d(const Basis1D &B, int nq, std::vector<double> &M, std::vector<double> &K) {
  const int n = B.n, p = B.p;
  M.assign((size_t)n * n, 0.0);
  K.assign((size_t)n * n, 0.0);
  std::vector<double> gx, gw;
  gauss_legendre(nq, gx, gw);
  double N[kMaxDeg + 1], dN[kMaxDeg + 1];
  for (int e = 0; e < B.n_el(); ++e) {
    int s = B.span[e];
    double lo = B.t[s], hi = B.t[s + 1];
    for (int g = 0; g < nq; ++g) {
      double xi = lo + (hi - lo) * 0.5 * (gx[g] + 1.0);
      double w = gw[g] * 0.5 * (hi - lo);
      B.eval(s, xi, N, dN);
      for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p; ++b) {
          M[(size_t)(s - p + a) * n + (s - p + b)] += w * N[a] * N[b];
          K[(size_t)(s - p + a) * n + (s - p + b)] += w * dN[a] * dN[b];
        }
    }
  }
}

// symmetric eigen-decomposition by cyclic Jacobi rotations: A = V diag(ev) V^T
static void jacobi_eigen(int n, std::vector<double> A, std::vector<double> &V, std::vector<double> &ev) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        if (i != j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        else diag += A[(size_t)i * n + i] * A[(size_t)i * n + i];
      }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int pI = 0; pI < n - 1; ++pI)
      for (int qI = pI + 1; qI < n; ++qI) {
        double apq = A[(size_t)pI * n + qI];
        if (apq == 0.0) continue;
        double app = A[(size_t)pI * n + pI], aqq = A[(size_t)qI * n + qI];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[(size_t)k * n + pI], akq = A[(size_t)k * n + qI];
          A[(size_t)k * n + pI] = c * akp - s * akq;
          A[(size_t)k * n + qI] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[(size_t)pI * n + k], aqk = A[(size_t)qI * n + k];
          A[(size_t)pI * n + k] = c * apk - s * aqk;
          A[(size_t)qI * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + pI], vkq = V[(size_t)k * n + qI];
          V[(size_t)k * n + pI] = c * vkp - s * vkq;
          V[(size_t)k * n + qI] = s * vkp + c * vkq;
        }
      }
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = A[(size_t)i * n + i];
}

// Generalized eigenvectors of (K, M) on the index range [lo, lo+m):
// U^T M U = I, U^T K U = diag(lam).  U row-major [k][j].
static void gen_eigen(const std::vector<double> &Mf, const std::vector<double> &Kf, int n, int lo, int m,
                      std::vector<double> &U, std::vector<double> &lam) {
  std::vector<double> M((size_t)m * m), K((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      M[(size_t)i * m + j] = Mf[(size_t)(lo + i) * n + lo + j];
      K[(size_t)i * m + j] = Kf[(size_t)(lo + i) * n + lo + j];
    }
  // Cholesky M = L L^T
  std::vector<double> L((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    double s = M[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
    if (!(s > 0)) fail(SA_EINVAL, "parametric mass matrix is not positive definite");
    L[(size_t)j * m + j] = std::sqrt(s);
    for (int i = j + 1; i < m; ++i) {
      double t = M[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
      L[(size_t)i * m + j] = t / L[(size_t)j * m + j];
    }
  }
  // Linv
  std::vector<double> Li((size_t)m * m, 0.0);
  for (int c = 0; c < m; ++c) {
    for (int i = 0; i < m; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[(size_t)i * m + k] * Li[(size_t)k * m + c];
      Li[(size_t)i * m + c] = s / L[(size_t)i * m + i];
    }
  }
  // C = Linv K Linv^T
  std::vector<double> T((size_t)m * m, 0.0), C((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += Li[(size_t)i * m + k] * K[(size_t)k * m + j];
      T[(size_t)i * m + j] = s;
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += T[(size_t)i * m + k] * Li[(size_t)j * m + k];
      C[(size_t)i * m + j] = s;
    }
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) {
      double a = 0.5 * (C[(size_t)i * m + j] + C[(size_t)j * m + i]);
      C[(size_t)i * m + j] = C[(size_t)j * m + i] = a;
    }
  std::vector<double> Q;
  jacobi_eigen(m, C, Q, lam);
  // U = Linv^T Q
  U.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += Li[(size_t)k * m + i] * Q[(size_t)k * m + j];
      U[(size_t)i * m + j] = s;
    }
}

void build_fd(Model &m) {
  PatchData &P = m.P;
  // 1-D factors integrated with the rules the assembled matrices use, so that
  // on an affine patch the Kronecker operator equals them exactly
  std::vector<double> Mh[3], Kh[3], Mf[3], Kf[3];
  for (int d = 0; d < 3; ++d) {
    param_mats_1d(P.b[d], P.qv[d], Mh[d], Kh[d]);
    param_mats_1d(P.b[d], P.qf, Mf[d], Kf[d]);
    m.M1[d] = Mh[d];
    m.K1[d] = Kh[d];
  }
  // main operator A = M/dt + theta K on the box of free DOFs
  FdData &F = m.fd_main;
  std::vector<double> lam[3];
  for (int d = 0; d < 3; ++d) {
    F.n[d] = P.n[d];
    int lo = P.role[2 * d] == SA_FACE_DIRICHLET ? 1 : 0;
    int hi = P.role[2 * d + 1] == SA_FACE_DIRICHLET ? P.n[d] - 1 : P.n[d];
    F.lo[d] = lo;
    F.m[d] = hi - lo;
    if (F.m[d] < 1) fail(SA_EINVAL, "no free control variables along a direction");
    gen_eigen(Mh[d], Kh[d], P.n[d], lo, F.m[d], F.U[d], lam[d]);
  }
  const double cM = m.mat.rho * m.mat.cp * m.mean_detJ / m.dt;
  const double th = m.opt.theta;
  double cK[3];
  for (int d = 0; d < 3; ++d) cK[d] = th * m.mat.k * m.mean_metric[d];
  F.inv_diag.resize((size_t)F.m[0] * F.m[1] * F.m[2]);
  for (int j2 = 0; j2 < F.m[2]; ++j2)
    for (int j1 = 0; j1 < F.m[1]; ++j1)
      for (int j0 = 0; j0 < F.m[0]; ++j0)
        F.inv_diag[(size_t)j0 + F.m[0] * ((size_t)j1 + F.m[1] * j2)] =
            1.0 / (cM + cK[0] * lam[0][j0] + cK[1] * lam[1][j1] + cK[2] * lam[2][j2]);

  // Dirichlet projection: one DIRICHLET face -> Kronecker of the two in-face
  // parametric mass matrices scaled by the face area
  int nf = 0, face = -1;
  for (int f = 0; f < 6; ++f)
    if (P.role[f] == SA_FACE_DIRICHLET) { nf++; face = f; }
  m.fd_dir_ok = false;
  if (nf == 1) {
    const int d = face / 2;
    int a = (d == 0) ? 1 : 0, b = (d == 2) ? 1 : 2;
    double area = 0.0;
    for (int64_t i = m.bt.face_off[face]; i < m.bt.face_off[face + 1]; ++i) area += m.bt.wdS[i];
    FdData &G = m.fd_dir;
    const int dims[2] = {a, b};
    std::vector<double> lm[3];
    for (int k = 0; k < 2; ++k) {
      int dd = dims[k];
      G.n[k] = P.n[dd];
      G.lo[k] = 0;
      G.m[k] = P.n[dd];
      gen_eigen(Mf[dd], Kf[dd], P.n[dd], 0, P.n[dd], G.U[k], lm[k]);
    }
    G.n[2] = G.m[2] = 1;
    G.lo[2] = 0;
    G.U[2].assign(1, 1.0);
    G.inv_diag.assign((size_t)G.m[0] * G.m[1], 1.0 / area);
    m.fd_dir_ok = true;
  }
}

// z = P^{-1} r on the free box (host reference of the device FD solve);
// r and z are full vectors on the n-grid, z is zero outside the box
void fd_apply_host(const FdData &F, const double *r, double *z, int64_t n_full) {
  const int m0 = F.m[0], m1 = F.m[1], m2 = F.m[2];
  const int64_t nb = (int64_t)m0 * m1 * m2;
  std::vector<double> t(nb), u(nb);
  auto full = [&](int j0, int j1, int j2) {
    return (int64_t)(j0 + F.lo[0]) + (int64_t)F.n[0] * ((j1 + F.lo[1]) + (int64_t)F.n[1] * (j2 + F.lo[2]));
  };
  auto cidx = [&](int j0, int j1, int j2) { return (int64_t)j0 + (int64_t)m0 * (j1 + (int64_t)m1 * j2); };
  for (int j2 = 0; j2 < m2; ++j2)
    for (int j1 = 0; j1 < m1; ++j1)
      for (int j0 = 0; j0 < m0; ++j0) {
        double s = 0;
        for (int k = 0; k < m0; ++k) s += F.U[0][(size_t)k * m0 + j0] * r[full(k, j1, j2)];
        t[cidx(j0, j1, j2)] = s;
      }
  for (int j2 = 0; j2 < m2; ++j2)
    for (int j1 = 0; j1 < m1; ++j1)
      for (int j0 = 0; j0 < m0; ++j0) {
        double s = 0;
        for (int k = 0; k < m1; ++k) s += F.U[1][(size_t)k * m1 + j1] * t[cidx(j0, k, j2)];
        u[cidx(j0, j1, j2)] = s;
      }
  for (int j2 = 0; j2 < m2; ++j2)
    for (int j1 = 0; j1 < m1; ++j1)
      for (int j0 = 0; j0 < m0; ++j0) {
        double s = 0;
        for (int k = 0; k < m2; ++k) s += F.U[2][(size_t)k * m2 + j2] * u[cidx(j0, j1, k)];
        t[cidx(j0, j1, j2)] = s * F.inv_diag[cidx(j0, j1, j2)];
      }
  for (int k2 = 0; k2 < m2; ++k2)
    for (int j1 = 0; j1 < m1; ++j1)
      for (int j0 = 0; j0 < m0; ++j0) {
        double s = 0;
        for (int j = 0; j < m2; ++j) s += F.U[2][(size_t)k2 * m2 + j] * t[cidx(j0, j1, j)];
        u[cidx(j0, j1, k2)] = s;
      }
  for (int k2 = 0; k2 < m2; ++k2)
    for (int k1 = 0; k1 < m1; ++k1)
      for (int j0 = 0; j0 < m0; ++j0) {
        double s = 0;
        for (int j = 0; j < m1; ++j) s += F.U[1][(size_t)k1 * m1 + j] * u[cidx(j0, j, k2)];
        t[cidx(j0, k1, k2)] = s;
      }
  for (int64_t i = 0; i < n_full; ++i) z[i] = 0.0;
  for (int k2 = 0; k2 < m2; ++k2)
    for (int k1 = 0; k1 < m1; ++k1)
      for (int k0 = 0; k0 < m0; ++k0) {
        double s = 0;
        for (int j = 0; j < m0; ++j) s += F.U[0][(size_t)k0 * m0 + j] * t[cidx(j, k1, k2)];
        z[full(k0, k1, k2)] = s;
      }
}

// Is the FD solve an exact inverse of the operator S restricted to the free
// box (affine axis-aligned geometry)?  Checked on a fixed pseudo-random vector.
double fd_inverse_defect(const FdData &F, const Stencil &S, const std::vector<double> &Sval,
                         const std::vector<uint8_t> &free_mask) {
  const int64_t n = S.nrow;
  std::vector<double> y(n, 0.0), z(n), w(n);
  uint64_t st = 0x9e3779b97f4a7c15ull;
  for (int64_t i = 0; i < n; ++i) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    if (free_mask[i]) y[i] = (double)(st >> 11) / 9007199254740992.0 - 0.5;
  }
  fd_apply_host(F, y.data(), z.data(), n);
  Stencil T = S;
  T.val = Sval;
  T.apply(z.data(), w.data());
  double num = 0, den = 0;
  for (int64_t i = 0; i < n; ++i)
    if (free_mask[i]) {
      num = std::max(num, std::fabs(w[i] - y[i]));
      den = std::max(den, std::fabs(y[i]));
    }
  return den > 0 ? num / den : 0.0;
}


// ---------------------------------------------------------------------------
// chunking of the source history of the kernel sum: enough workgroups to fill
// the chip, the FP64 sources weighted by their cost.  The chunk lengths
// depend on the point count, the batch and the source counts only, never on
// the tile shape (points per lane, waves per group), so every tile shape
// gives bitwise the same sums.
// ---------------------------------------------------------------------------
SumPlan plan_sum(const sa_solver_options &o, int64_t nq, int count, int64_t max_far, int64_t max_near) {
  constexpr int64_t kRefBlockPoints = 512;
  constexpr int64_t kTargetGroups = 2048;
  SumPlan pl{};
  pl.points_per_lane = o.points_per_lane ? o.points_per_lane : 2;
  pl.waves = o.waves_per_group ? std::min(o.waves_per_group, 8) : 4;
  pl.nq = nq;
  pl.chunk_far = pl.chunk_near = 1;
  auto tile_up = [](int64_t n) { return (n + kFarChunkQuantum - 1) / kFarChunkQuantum * kFarChunkQuantum; };
  if (o.chunk_sources > 0) {
    pl.chunk_near = o.chunk_sources;
    pl.chunk_far = (int)tile_up(o.chunk_sources);   // far chunks start on FP32 record blocks
    pl.n_chunks_far = (int)((max_far + pl.chunk_far - 1) / pl.chunk_far);
    pl.n_chunks_near = (int)((max_near + pl.chunk_near - 1) / pl.chunk_near);
    return pl;
  }
  const int64_t n_ref = std::max<int64_t>(1, (nq + kRefBlockPoints - 1) / kRefBlockPoints);
  const int64_t C = std::max<int64_t>(1, (kTargetGroups + n_ref * count - 1) / (n_ref * count));
  const double wf = (double)max_far, wn = 3.0 * (double)max_near;
  int64_t cf = 0, cn = 0;
  if (max_far > 0 && max_near > 0) {
    cf = std::max<int64_t>(1, (int64_t)std::llround(C * wf / (wf + wn)));
    cn = std::max<int64_t>(1, C - cf);
  } else if (max_far > 0) {
    cf = C;
  } else if (max_near > 0) {
    cn = C;
  }
  const int64_t min_chunk = 32;
  if (cf) {
    const int64_t len = tile_up(std::max<int64_t>(min_chunk, (max_far + cf - 1) / cf));
    pl.chunk_far = (int)len;
    pl.n_chunks_far = (int)((max_far + len - 1) / len);
  }
  if (cn) {
    const int64_t len = std::max<int64_t>(min_chunk, (max_near + cn - 1) / cn);
    pl.chunk_near = (int)len;
    pl.n_chunks_near = (int)((max_near + len - 1) / len);
  }
  return pl;
}

// Parametric point of the physical point x (inverse of the geometry map):
// the element centre nearest to x, then Newton steps xi <- xi + J^{-1}
// (x - x(xi)) kept in [0,1]^3, until |x - x(xi)| <= tol.  false if x is
// not reached (it lies outside the patch).
bool locate_point(const PatchData &P, const std::vector<double> &centres, const std::vector<double> &cxi,
                  const double x[3], double tol, double xi[3]) {
  int64_t best = -1;
  double bd = INFINITY;
  for (int64_t e = 0; e < (int64_t)centres.size() / 3; ++e) {
    const double d0 = centres[3 * e] - x[0], d1 = centres[3 * e + 1] - x[1], d2 = centres[3 * e + 2] - x[2];
    const double d = d0 * d0 + d1 * d1 + d2 * d2;
    if (d < bd) {
      bd = d;
      best = e;
    }
  }
  if (best < 0) return false;
  for (int c = 0; c < 3; ++c) xi[c] = cxi[3 * best + c];
  PointEval pe;
  for (int it = 0; it < 60; ++it) {
    int span[3];
    for (int c = 0; c < 3; ++c) span[c] = P.b[c].find_span(xi[c]);
    eval_point(P, xi, span, pe);
    const double r[3] = {x[0] - pe.x[0], x[1] - pe.x[1], x[2] - pe.x[2]};
    const double res = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (res <= tol) return true;
    const double(&J)[3][3] = pe.J;
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(std::fabs(det) > 0.0)) return false;
    // J^{-1} r by Cramer's rule
    double d[3];
    for (int c = 0; c < 3; ++c) {
      double M[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = (j == c) ? r[i] : J[i][j];
      d[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
              M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) /
             det;
    }
    for (int c = 0; c < 3; ++c) xi[c] = std::min(1.0, std::max(0.0, xi[c] + d[c]));
  }
  return false;
}

// physical and parametric centres of the patch's elements ([n_el][3] each)
void element_centres(const PatchData &P, std::vector<double> &centres, std::vector<double> &cxi) {
  centres.clear();
  cxi.clear();
  PointEval pe;
  for (int e2 = 0; e2 < P.b[2].n_el(); ++e2)
    for (int e1 = 0; e1 < P.b[1].n_el(); ++e1)
      for (int e0 = 0; e0 < P.b[0].n_el(); ++e0) {
        const int es[3] = {e0, e1, e2};
        double c[3];
        int span[3];
        for (int d = 0; d < 3; ++d) {
          span[d] = P.b[d].span[es[d]];
          c[d] = 0.5 * (P.b[d].t[span[d]] + P.b[d].t[span[d] + 1]);
        }
        eval_point(P, c, span, pe);
        for (int d = 0; d < 3; ++d) {
          cxi.push_back(c[d]);
          centres.push_back(pe.x[d]);
        }
      }
}

// 1e-13 of the control net's extent about its centre
double locate_tolerance(const PatchData &P) {
  double ext = 0.0;
  for (int64_t A = 0; A < P.ndof; ++A)
    for (int c = 0; c < 3; ++c) ext = std::max(ext, std::fabs(P.ctrl[4 * A + c] - P.center[c]));
  return 1e-13 * std::max(ext, 1e-300);
}

// Gauss points (quad per element) of the edge where parametric face `face`
// meets face `edge_face` (faces of different directions), ordered by element:
// their parametric points xi [n][3], the outward unit normals of `face`
// [n][3] and the arc-length weights ds [n]; returns n
int64_t edge_points(const PatchData &P, int face, int edge_face, int quad, std::vector<double> &xi,
                    std::vector<double> &nrm, std::vector<double> &dsv) {
  const int d = face / 2, de = edge_face / 2, e = 3 - d - de;
  const int64_t n = (int64_t)P.b[e].n_el() * quad;
  // Gauss points of the elements along the edge, ordered by element
  std::vector<double> g, gw;
  gauss_legendre(quad, g, gw);
  std::vector<double> w((size_t)n);
  xi.assign((size_t)3 * n, 0.0);
  nrm.assign((size_t)3 * n, 0.0);
  dsv.assign((size_t)n, 0.0);
  const Basis1D &B = P.b[e];
  for (int el = 0; el < B.n_el(); ++el) {
    const double lo = B.t[B.span[el]], hi = B.t[B.span[el] + 1];
    for (int k = 0; k < quad; ++k) {
      const int64_t i = (int64_t)el * quad + k;
      xi[3 * i + d] = (double)(face % 2);
      xi[3 * i + de] = (double)(edge_face % 2);
      xi[3 * i + e] = lo + 0.5 * (hi - lo) * (g[k] + 1.0);
      w[i] = 0.5 * (hi - lo) * gw[k];
    }
  }
  // arc length along the edge and the face's outward normal: the gradient
  // of xi_d (row d of J^{-1}), signed by the side of the face
  PointEval pe;
  for (int64_t i = 0; i < n; ++i) {
    int span[3];
    for (int c = 0; c < 3; ++c) span[c] = P.b[c].find_span(xi[3 * i + c]);
    eval_point(P, &xi[3 * i], span, pe);
    const double(&J)[3][3] = pe.J;
    dsv[i] = std::sqrt(J[0][e] * J[0][e] + J[1][e] * J[1][e] + J[2][e] * J[2][e]) * w[i];
    // row d of J^{-1}: the cross product of the other two columns of J over det J
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    double gd[3] = {J[1][a] * J[2][b] - J[2][a] * J[1][b], J[2][a] * J[0][b] - J[0][a] * J[2][b],
                    J[0][a] * J[1][b] - J[1][a] * J[0][b]};
    const double det = gd[0] * J[0][d] + gd[1] * J[1][d] + gd[2] * J[2][d];
    const double len = std::sqrt(gd[0] * gd[0] + gd[1] * gd[1] + gd[2] * gd[2]);
    const double sg = ((face % 2) ? 1.0 : -1.0) * (det > 0 ? 1.0 : -1.0) / len;
    for (int c = 0; c < 3; ++c) nrm[3 * i + c] = sg * gd[c];
  }
  return n;
}

}  // namespace sa
