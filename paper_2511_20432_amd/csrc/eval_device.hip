// Correction field T^ = sum_A R_A u_A (Eq. 21) and its physical gradient at
// parametric points held on the device: one thread per point computes the
// knot spans, the B-spline values and first derivatives per direction
// (Cox-de Boor), the rational basis through the weighted sums, the geometry
// map and its Jacobian, and contracts with the control values.
#include "eval_device.h"

#include <cmath>

namespace sa {

namespace {

constexpr int kDeg = 6;
constexpr int kThreads = 128;

// last s with t_s <= xi < t_{s+1}; xi = t_n (the right end) goes to s = n - 1
__device__ int span_of(const double *t, int p, int n, double xi) {
  if (xi >= t[n]) return n - 1;
  int lo = p, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (xi < t[mid]) hi = mid;
    else lo = mid;
  }
  return lo;
}

// values N[0..p] and derivatives dN[0..p] of the functions s-p .. s at xi
__device__ void basis_at(const double *t, int p, int s, double xi, double *N, double *dN) {
  double left[kDeg + 2], right[kDeg + 2], low[kDeg + 1];
  N[0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    if (j == p)
      for (int r = 0; r < p; ++r) low[r] = N[r];
    left[j] = xi - t[s + 1 - j];
    right[j] = t[s + j] - xi;
    double carry = 0.0;
    for (int r = 0; r < j; ++r) {
      const double den = right[r + 1] + left[j - r];
      const double q = den != 0.0 ? N[r] / den : 0.0;
      N[r] = carry + right[r + 1] * q;
      carry = left[j - r] * q;
    }
    N[j] = carry;
  }
  if (p == 0) {
    dN[0] = 0.0;
    return;
  }
  // derivative of a degree-p function from the two degree-(p-1) ones it is made of
  for (int r = 0; r <= p; ++r) {
    const int i = s - p + r;
    double a = 0.0, b = 0.0;
    if (r >= 1) {
      const double den = t[i + p] - t[i];
      if (den != 0.0) a = low[r - 1] / den;
    }
    if (r <= p - 1) {
      const double den = t[i + p + 1] - t[i + 1];
      if (den != 0.0) b = low[r] / den;
    }
    dN[r] = p * (a - b);
  }
}

__global__ __launch_bounds__(kThreads) void k_eval_hat(int64_t n, const double *__restrict__ xi, GeoDev g,
                                                       const double *__restrict__ u, double *__restrict__ x,
                                                       double *__restrict__ Th, double *__restrict__ Gh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double N[3][kDeg + 1], dN[3][kDeg + 1];
  int s[3];
  bool inside = true;
  for (int d = 0; d < 3; ++d) {
    const double v = xi[3 * i + d];
    if (!(v >= 0.0 && v <= 1.0)) {
      inside = false;
      break;
    }
    s[d] = span_of(g.t[d], g.p[d], g.n[d], v);
    basis_at(g.t[d], g.p[d], s[d], v, N[d], dN[d]);
  }
  if (!inside) {
    const double nan = __builtin_nan("");
    for (int c = 0; c < 3; ++c) {
      x[3 * i + c] = nan;
      Gh[c * n + i] = nan;
    }
    Th[i] = nan;
    return;
  }
  // weighted sums: W = sum N w, P = sum N w X, U = sum N w u and their
  // parametric derivatives (D*[k] = d/dxi_k)
  double W = 0.0, DW[3] = {0.0, 0.0, 0.0}, P[3] = {0.0, 0.0, 0.0}, DP[3][3] = {}, U = 0.0, DU[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c <= g.p[2]; ++c) {
    const int i2 = s[2] - g.p[2] + c;
    for (int b = 0; b <= g.p[1]; ++b) {
      const int i1 = s[1] - g.p[1] + b;
      const double n12 = N[1][b] * N[2][c], d1 = dN[1][b] * N[2][c], d2 = N[1][b] * dN[2][c];
      for (int a = 0; a <= g.p[0]; ++a) {
        const int64_t A = ((int64_t)i2 * g.n[1] + i1) * g.n[0] + (s[0] - g.p[0] + a);
        const double *X = g.ctrl + 4 * A;
        const double w = X[3];
        const double v = N[0][a] * n12 * w;
        const double dv[3] = {dN[0][a] * n12 * w, N[0][a] * d1 * w, N[0][a] * d2 * w};
        const double uA = u[A];
        W += v;
        U += v * uA;
        for (int m = 0; m < 3; ++m) P[m] += v * X[m];
        for (int k = 0; k < 3; ++k) {
          DW[k] += dv[k];
          DU[k] += dv[k] * uA;
          for (int m = 0; m < 3; ++m) DP[m][k] += dv[k] * X[m];
        }
      }
    }
  }
  // quotient rule: x = P / W, dx/dxi = (DP - x DW) / W; the same for T^
  double xm[3], J[3][3], du[3];
  for (int m = 0; m < 3; ++m) xm[m] = P[m] / W;
  for (int m = 0; m < 3; ++m)
    for (int k = 0; k < 3; ++k) J[m][k] = (DP[m][k] - xm[m] * DW[k]) / W;
  const double th = U / W;
  for (int k = 0; k < 3; ++k) du[k] = (DU[k] - th * DW[k]) / W;
  // grad T^ = J^-T du: the inverse by cofactors
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  const double id = 1.0 / det;
  double Ji[3][3];
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  for (int c = 0; c < 3; ++c) {
    x[3 * i + c] = xm[c];
    Gh[c * n + i] = du[0] * Ji[0][c] + du[1] * Ji[1][c] + du[2] * Ji[2][c];
  }
  Th[i] = th;
}

__global__ void k_eval_combine(int64_t n, double T0, const double *__restrict__ Th, const double *__restrict__ Gh,
                               const double *__restrict__ Tt, const double *__restrict__ Gt, double *__restrict__ T,
                               double *__restrict__ gradT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T[i] = T0 + Th[i] + Tt[i];
  if (gradT)
    for (int c = 0; c < 3; ++c) gradT[3 * i + c] = Gh[c * n + i] + Gt[c * n + i];
}

unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

void launch_eval_hat(hipStream_t st, int64_t n, const double *xi, const GeoDev &g, const double *u, double *x,
                     double *Th, double *Gh) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_eval_hat, dim3(blocks(n)), dim3(kThreads), 0, st, n, xi, g, u, x, Th, Gh);
}

void launch_eval_combine(hipStream_t st, int64_t n, double T0, const double *Th, const double *Gh, const double *Tt,
                         const double *Gt, double *T, double *gradT) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_eval_combine, dim3(blocks(n)), dim3(kThreads), 0, st, n, T0, Th, Gh, Tt, Gt, T, gradT);
}

}  // namespace sa
