// Fused solver kernels for the theta-scheme (Eq. 20) and the Dirichlet
// projection (Eq. 11) on gfx950.
//
//  * k_gather_rows   load vector F (lane-parallel rows) + copy of v into x
//  * k_copy_free     first iterate: v on the free DOFs
//  * k_dirichlet     one workgroup: projection rhs gather, then the whole
//                    PCG for the trace mass matrix with the 2-D fast-
//                    diagonalisation preconditioner held in LDS; writes the
//                    Dirichlet values and scatters them into x
//  * k_stencil_sl    banded stencil product, 64 rows per block and one wave
//                    per z-offset slice (theta rhs/residual or A p with p.Ap)
//  * k_fd_xfwd       (optional PCG update) + mode 0 of the FD solve, one
//                    x-fiber of the free box per block
//  * k_fd_plane      modes 1 and 2 and the eigenvalue scaling, one (y, z)
//                    plane per block, in LDS
//  * k_fd_xbwd       mode 0 back to z (+ p = z on the first pass)
//  * k_pcg_dir       convergence test and p = z + beta p
// The scalar recurrences are recomputed in every block from fixed-order
// partial sums, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"
#include "solver.h"

namespace sa {

namespace {

constexpr int kB = 256;

// The theta-step kernels form a chain of short dependent launches that runs
// beside the long kernel sum; their waves take the SIMD's issue slots first
// (wave priority), so the chain is not stretched by the sum's instructions.
__device__ __forceinline__ void issue_first() { __builtin_amdgcn_s_setprio(3); }

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// block sum for any block size <= 1024; all threads get the result
__device__ __forceinline__ double bsum(double v, double *sh) {
  v = wsum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (int)(blockDim.x >> 6);
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

__device__ __forceinline__ double reduce_n(const double *part, int n, double *sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  return bsum(s, sh);
}

}  // namespace

// ---------------------------------------------------------------------------
// load vector: 16 lanes per non-empty row
// ---------------------------------------------------------------------------
__global__ void k_gather_rows(SlotMap sm, int64_t nrows, const int32_t *__restrict__ rows,
                              const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                              const double *__restrict__ val, const double *__restrict__ ldb, int64_t ls,
                              double *__restrict__ Fb, int64_t fs, int64_t ncopy, const double *__restrict__ vb,
                              double *__restrict__ xb) {
  const int64_t pth = sm.path[blockIdx.y];
  const double *ld = ldb + pth * ls;
  double *F = Fb + pth * fs;
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sub = threadIdx.x & 15;
  const int64_t r = gt >> 4;
  double s = 0.0;
  if (r < nrows) {
    for (int64_t e = rowptr[r] + sub; e < rowptr[r + 1]; e += 16) s = fma(val[e], ld[col[e]], s);
  }
  for (int off = 8; off > 0; off >>= 1) s += __shfl_down(s, off, 16);
  if (r < nrows && sub == 0) F[rows[r]] = s;
  if (ncopy > 0) {
    const double *v = vb + pth * fs;
    double *x = xb + pth * fs;
    for (int64_t i = gt; i < ncopy; i += (int64_t)gridDim.x * blockDim.x) x[i] = v[i];
  }
}

// two gathers of the same densities in one launch: the first blocks1 blocks
// take g1 -> F1, the rest g2 -> F2
__global__ void k_gather_rows2(SlotMap sm, int64_t blocks1, GatherRows g1, double *__restrict__ F1b, int64_t fs1,
                               GatherRows g2, double *__restrict__ F2b, int64_t fs2,
                               const double *__restrict__ ldb, int64_t ls) {
  const int64_t pth = sm.path[blockIdx.y];
  const double *ld = ldb + pth * ls;
  const bool second = (int64_t)blockIdx.x >= blocks1;
  const GatherRows &g = second ? g2 : g1;
  double *F = second ? F2b + pth * fs2 : F1b + pth * fs1;
  const int64_t gt = ((int64_t)blockIdx.x - (second ? blocks1 : 0)) * blockDim.x + threadIdx.x;
  const int sub = threadIdx.x & 15;
  const int64_t r = gt >> 4;
  double s = 0.0;
  if (r < g.nrows) {
    for (int64_t e = g.rowptr[r] + sub; e < g.rowptr[r + 1]; e += 16) s = fma(g.val[e], ld[g.col[e]], s);
  }
  for (int off = 8; off > 0; off >>= 1) s += __shfl_down(s, off, 16);
  if (r < g.nrows && sub == 0) F[g.rows[r]] = s;
}

void launch_gather_rows2(hipStream_t st, const SlotMap &sm, const GatherRows &g1, double *F1, int64_t fs1,
                         const GatherRows &g2, double *F2, int64_t fs2, const double *ld, int64_t ls) {
  if (sm.count <= 0) return;
  const int64_t b1 = std::max<int64_t>(1, (g1.nrows * 16 + kB - 1) / kB);
  const int64_t b2 = std::max<int64_t>(1, (g2.nrows * 16 + kB - 1) / kB);
  hipLaunchKernelGGL(k_gather_rows2, dim3((unsigned)(b1 + b2), (unsigned)sm.count), dim3(kB), 0, st, sm, b1, g1, F1,
                     fs1, g2, F2, fs2, ld, ls);
}

void launch_gather_rows(hipStream_t st, const SlotMap &sm, const GatherRows &g, const double *ld, int64_t ls,
                        double *F, int64_t fs, int64_t ncopy, const double *v, double *x) {
  if (sm.count <= 0) return;
  int64_t threads = g.nrows * 16;
  int64_t blocks = (threads + kB - 1) / kB;
  int64_t cb = (ncopy + kB - 1) / kB;
  if (cb > blocks) blocks = cb;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)blocks, (unsigned)sm.count), dim3(kB), 0, st, sm, g.nrows,
                     g.rows, g.rowptr, g.col, g.val, ld, ls, F, fs, ncopy, v, x);
}

// ---------------------------------------------------------------------------
// first iterate of the theta-step: u^n on the free DOFs, the new Dirichlet
// values (already in x) on the others
// ---------------------------------------------------------------------------
__global__ void k_copy_free(SlotMap sm, int64_t n, const uint8_t *__restrict__ mask, const double *__restrict__ vb,
                            double *__restrict__ xb) {
  const int64_t pth = sm.path[blockIdx.y];
  const double *v = vb + pth * n;
  double *x = xb + pth * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (mask[i]) x[i] = v[i];
}

void launch_copy_free(hipStream_t st, const SlotMap &sm, int64_t n, const uint8_t *mask, const double *v,
                      double *x) {
  if (sm.count <= 0 || n <= 0) return;
  const int64_t blocks = (n + kB - 1) / kB;
  hipLaunchKernelGGL(k_copy_free, dim3((unsigned)blocks, (unsigned)sm.count), dim3(kB), 0, st, sm, n, mask, v, x);
}

// ---------------------------------------------------------------------------
// Dirichlet projection in one workgroup
// ---------------------------------------------------------------------------
constexpr int kDirThreads = 1024;

// z = P^{-1} r for the 2-D Kronecker preconditioner (or Jacobi), in LDS
__device__ void dir_precond(const DirArgs &a, const double *Ua, const double *Ub, const double *r, double *z,
                            double *t1, double *t2) {
  const int n = a.nD;
  if (!a.fd) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) z[j] = a.jacobi[j] * r[j];
    __syncthreads();
    return;
  }
  const int na = a.na, nb = a.nb;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {       // t1 = Ua^T along a
    const int ja = t % na, kb = t / na;
    double s = 0.0;
    for (int k = 0; k < na; ++k) s = fma(Ua[k * na + ja], r[k + na * kb], s);
    t1[t] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += blockDim.x) {       // t2 = D^{-1} Ub^T along b
    const int ja = t % na, jb = t / na;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s = fma(Ub[k * nb + jb], t1[ja + na * k], s);
    t2[t] = s * a.inv[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += blockDim.x) {       // t1 = Ub along b
    const int ja = t % na, kb = t / na;
    double s = 0.0;
    for (int j = 0; j < nb; ++j) s = fma(Ub[kb * nb + j], t2[ja + na * j], s);
    t1[t] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += blockDim.x) {       // z = Ua along a
    const int ka = t % na, kb = t / na;
    double s = 0.0;
    for (int j = 0; j < na; ++j) s = fma(Ua[ka * na + j], t1[j + na * kb], s);
    z[t] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kDirThreads) void k_dirichlet(SlotMap sm, DirArgs a) {
  extern __shared__ double lds[];
  __shared__ double sh[16];
  const int n = a.nD;
  {
    const int64_t pth = sm.path[blockIdx.x];
    a.b += pth * n;
    a.vD += pth * n;
    a.xfull += pth * a.xs;
    if (a.status) a.status += blockIdx.x;
  }
  double *r = lds, *z = lds + n, *p = lds + 2 * n, *t1 = lds + 3 * n, *t2 = lds + 4 * n;
  // the preconditioner's eigenvector matrices live in LDS when they fit
  const double *Ua = a.Ua, *Ub = a.Ub;
  if (a.fd && a.u_in_lds) {
    double *ua = lds + 5 * n, *ub = ua + a.na * a.na;
    for (int i = threadIdx.x; i < a.na * a.na; i += blockDim.x) ua[i] = a.Ua[i];
    for (int i = threadIdx.x; i < a.nb * a.nb; i += blockDim.x) ub[i] = a.Ub[i];
    Ua = ua;
    Ub = ub;
  }
  double *x = a.vD;
  // r = b - M x (warm start from the previous values)
  double bb = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double b = a.b[j];
    double mx = 0.0;
#pragma unroll 4
    for (int64_t e = a.mrow[j]; e < a.mrow[j + 1]; ++e) mx = fma(a.mval[e], x[a.mcol[e]], mx);
    r[j] = b - mx;
    bb = fma(b, b, bb);
  }
  bb = bsum(bb, sh);
  dir_precond(a, Ua, Ub, r, z, t1, t2);
  double rz = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    p[j] = z[j];
    rz = fma(r[j], z[j], rz);
  }
  rz = bsum(rz, sh);
  int it = 0, done = (rz == 0.0) ? 1 : 0;
  double rr = 0.0;
  constexpr int kMaxPer = 4;  // rows per thread (n <= kDirThreads * kMaxPer)
  while (!done && it < a.max_iter) {
    double q[kMaxPer];
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
      const int j = threadIdx.x + k * blockDim.x;
      q[k] = 0.0;
      if (j < n) {
        double s = 0.0;
#pragma unroll 4
        for (int64_t e = a.mrow[j]; e < a.mrow[j + 1]; ++e) s = fma(a.mval[e], p[a.mcol[e]], s);
        q[k] = s;
        pq = fma(p[j], s, pq);
      }
    }
    pq = bsum(pq, sh);
    if (!(pq > 0.0)) { done = 2; break; }
    const double alpha = rz / pq;
    rr = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
      const int j = threadIdx.x + k * blockDim.x;
      if (j < n) {
        x[j] = fma(alpha, p[j], x[j]);
        const double rj = fma(-alpha, q[k], r[j]);
        r[j] = rj;
        rr = fma(rj, rj, rr);
      }
    }
    rr = bsum(rr, sh);
    ++it;
    if (rr <= a.rtol2 * bb) { done = 1; break; }
    dir_precond(a, Ua, Ub, r, z, t1, t2);
    double rzn = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) rzn = fma(r[j], z[j], rzn);
    rzn = bsum(rzn, sh);
    const double beta = rzn / rz;
    rz = rzn;
    for (int j = threadIdx.x; j < n; j += blockDim.x) p[j] = fma(beta, p[j], z[j]);
    __syncthreads();
  }
  // scatter the values into the theta-step iterate
  for (int j = threadIdx.x; j < n; j += blockDim.x) a.xfull[a.dofs[j]] = x[j];
  if (threadIdx.x == 0 && a.status) {
    a.status->iter = it;
    a.status->done = done;
    a.status->relres2 = bb > 0 ? rr / bb : 0.0;
  }
}

bool dirichlet_fits(int64_t nD) { return nD > 0 && nD <= 4 * kDirThreads; }

size_t dirichlet_lds(const DirArgs &a) {
  size_t n = (size_t)5 * a.nD;
  if (a.fd && a.u_in_lds) n += (size_t)a.na * a.na + (size_t)a.nb * a.nb;
  return n * sizeof(double);
}

void launch_dirichlet(hipStream_t st, const SlotMap &sm, const DirArgs &a) {
  if (sm.count <= 0) return;
  hipLaunchKernelGGL(k_dirichlet, dim3((unsigned)sm.count), dim3(kDirThreads), dirichlet_lds(a), st, sm, a);
}

// ---------------------------------------------------------------------------
// banded stencil products: 64 rows per block, one wave per z-offset
// ---------------------------------------------------------------------------
template <int HW0, bool THETA>
__global__ void k_stencil_sl(SlotMap sm, SlArgs a) {
  extern __shared__ double shr[];          // [waves][64]
  __shared__ double sh[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);
  {
    const int64_t pth = sm.path[blockIdx.y];
    const int64_t off = pth * a.vs;
    a.x += off;
    a.out += off;
    a.part += pth * a.np;
    if (THETA) {
      a.v += off;
      a.F1 += off;
      a.F0 += off;
      if (a.sc_w) a.sc_w += pth;
    } else if (a.sc) {
      a.sc += pth;
    }
  }
  if (!THETA && a.sc && a.sc->done) return;
  const int64_t row = (int64_t)blockIdx.x * 64 + lane;
  const int64_t nrow = a.nrow, nm1 = nrow - 1;
  const int n0 = a.n0;
  const int64_t n01 = (int64_t)a.n0 * a.n1;
  const int hw1 = a.hw1;
  const int d2 = w - a.hw2;
  double acc = 0.0, accb = 0.0;
  const bool active = row < nrow && (!a.mask || a.mask[row]);
  if (active) {
    const int span0 = 2 * HW0 + 1;
    int o = ((w) * (2 * hw1 + 1)) * span0;
    for (int d1 = -hw1; d1 <= hw1; ++d1) {
      const int64_t base = row + (int64_t)d1 * n0 + (int64_t)d2 * n01;
#pragma unroll
      for (int d0 = -HW0; d0 <= HW0; ++d0) {
        int64_t nb = base + d0;
        nb = nb < 0 ? 0 : (nb > nm1 ? nm1 : nb);
        const int64_t oi = (int64_t)(o + d0 + HW0) * nrow + row;
        acc = fma(a.A[oi], a.x[nb], acc);
        if (THETA) accb = fma(a.B[oi], a.v[nb], accb);
      }
      o += span0;
    }
  }
  shr[w * 64 + lane] = acc;
  if (THETA) shr[(nw + w) * 64 + lane] = accb;
  __syncthreads();
  double part = 0.0;
  if (w == 0) {
    double s = 0.0, sb = 0.0;
    for (int k = 0; k < nw; ++k) {
      s += shr[k * 64 + lane];
      if (THETA) sb += shr[(nw + k) * 64 + lane];
    }
    if (row < nrow) {
      if (THETA) {
        double rv = 0.0;
        if (active) {
          const double rhs = sb + a.theta * a.F1[row] + (1.0 - a.theta) * a.F0[row];
          part = rhs * rhs;
          rv = rhs - s;
        }
        a.out[row] = rv;
      } else {
        a.out[row] = active ? s : 0.0;
        part = active ? a.x[row] * s : 0.0;
      }
    }
  }
  part = bsum(part, sh);
  if (threadIdx.x == 0) a.part[blockIdx.x] = part;
  if (THETA && blockIdx.x == 0 && threadIdx.x == 0 && a.sc_w) a.sc_w->done = 0;
}

// ---------------------------------------------------------------------------
// matrix-free Kronecker operators: one banded product along one axis per pass,
// thread per row
// ---------------------------------------------------------------------------
// sum_j f[i][j] in[base + (j - i) stride] over the band j in [i - p, i + p] of 0..n-1
// the band of half-width P unrolled, so that its loads issue together; the
// same terms in the same order as the loop below
template <int P>
__device__ __forceinline__ double band_dot_p(const double *__restrict__ b, int i, int n,
                                             const double *__restrict__ in, int64_t base, int64_t stride) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k <= 2 * P; ++k) {
    const int j = i - P + k;
    if (j >= 0 && j < n) s = fma(b[k], in[base + (int64_t)(k - P) * stride], s);
  }
  return s;
}

__device__ __forceinline__ double band_dot(const double *__restrict__ band, int p, int i, int n,
                                           const double *__restrict__ in, int64_t base, int64_t stride) {
  const double *b = band + (int64_t)i * (2 * p + 1);
  switch (p) {
    case 1: return band_dot_p<1>(b, i, n, in, base, stride);
    case 2: return band_dot_p<2>(b, i, n, in, base, stride);
    case 3: return band_dot_p<3>(b, i, n, in, base, stride);
    case 4: return band_dot_p<4>(b, i, n, in, base, stride);
    default: break;
  }
  const int j0 = i - p < 0 ? 0 : i - p, j1 = i + p > n - 1 ? n - 1 : i + p;
  double s = 0.0;
  for (int j = j0; j <= j1; ++j) s = fma(b[j - i + p], in[base + (int64_t)(j - i) * stride], s);
  return s;
}

// band product of the first iterate: v on the free DOFs, x (the new Dirichlet
// values) on the others
__device__ __forceinline__ void band_dot_init(const double *__restrict__ Mb, const double *__restrict__ Kb, int p,
                                              int i, int n, const uint8_t *__restrict__ mask,
                                              const double *__restrict__ v, const double *x,
                                              const double *__restrict__ dv, const int32_t *__restrict__ didx,
                                              int64_t base, double &sm_, double &sk) {
  const double *bm = Mb + (int64_t)i * (2 * p + 1), *bk = Kb + (int64_t)i * (2 * p + 1);
  const int j0 = i - p < 0 ? 0 : i - p, j1 = i + p > n - 1 ? n - 1 : i + p;
  double s0 = 0.0, s1 = 0.0;
  for (int j = j0; j <= j1; ++j) {
    const int64_t q = base + (j - i);
    const double xv = mask[q] ? v[q] : (dv ? dv[didx[q]] : x[q]);
    s0 = fma(bm[j - i + p], xv, s0);
    s1 = fma(bk[j - i + p], xv, s1);
  }
  sm_ = s0;
  sk = s1;
}

template <bool THETA>
__global__ void k_kron_x(SlotMap sm, KronArgs a) {
  issue_first();
  const int64_t pth = sm.path[blockIdx.y];
  if (!THETA && a.sc && a.sc[pth].done) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = a.nrow;
  if (r >= N) return;
  const int n0 = a.op.n[0], p = a.op.p[0], i0 = (int)(r % n0);
  double *t = a.t + pth * a.ts;
  if (THETA && a.check_only) {
    // residual check alone: products of v only
  } else if (THETA && a.init_x) {
    // first iterate formed here: no thread reads x at a free DOF, where it is written
    double *x = a.x_init + pth * a.vs;
    const double *v = a.v + pth * a.vs;
    const double *dv = a.dv ? a.dv + (int64_t)blockIdx.y * a.dvs : nullptr;
    double s0, s1;
    band_dot_init(a.op.Mb[0], a.op.Kb[0], p, i0, n0, a.mask, v, x, dv, a.didx, r, s0, s1);
    t[r] = s0;
    t[N + r] = s1;
    if (a.mask[r]) x[r] = v[r];
    else if (dv) x[r] = dv[a.didx[r]];
  } else {
    const double *x = a.x + pth * a.vs;
    t[r] = band_dot(a.op.Mb[0], p, i0, n0, x, r, 1);
    t[N + r] = band_dot(a.op.Kb[0], p, i0, n0, x, r, 1);
  }
  if (THETA) {
    const double *v = a.v + pth * a.vs;
    t[2 * N + r] = band_dot(a.op.Mb[0], p, i0, n0, v, r, 1);
    t[3 * N + r] = band_dot(a.op.Kb[0], p, i0, n0, v, r, 1);
  }
}

template <bool THETA>
__global__ void k_kron_y(SlotMap sm, KronArgs a) {
  issue_first();
  const int64_t pth = sm.path[blockIdx.y];
  if (!THETA && a.sc && a.sc[pth].done) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = a.nrow;
  if (r >= N) return;
  const int n0 = a.op.n[0], n1 = a.op.n[1], p = a.op.p[1];
  const int i1 = (int)((r / n0) % n1);
  const double *Mb = a.op.Mb[1], *Kb = a.op.Kb[1];
  double *t = a.t + pth * a.ts;
  if (THETA && a.check_only) {
    const double bmm = band_dot(Mb, p, i1, n1, t + 2 * N, r, n0);
    const double bmk = band_dot(Mb, p, i1, n1, t + 3 * N, r, n0);
    const double bkm = band_dot(Kb, p, i1, n1, t + 2 * N, r, n0);
    t[8 * N + r] = a.op.cM * bmm + a.op.cA[0] * bmk + a.op.cA[1] * bkm;
    t[9 * N + r] = a.op.cA[2] * bmm;
    return;
  }
  // A: (M y M x) x, (M y K x) x, (K y M x) x  ->  the parts taken by M z and K z
  const double mm = band_dot(Mb, p, i1, n1, t, r, n0);
  const double mk = band_dot(Mb, p, i1, n1, t + N, r, n0);
  const double km = band_dot(Kb, p, i1, n1, t, r, n0);
  t[4 * N + r] = a.op.cM * mm + a.op.cA[0] * mk + a.op.cA[1] * km;
  t[5 * N + r] = a.op.cA[2] * mm;
  if (THETA) {
    const double bmm = band_dot(Mb, p, i1, n1, t + 2 * N, r, n0);
    const double bmk = band_dot(Mb, p, i1, n1, t + 3 * N, r, n0);
    const double bkm = band_dot(Kb, p, i1, n1, t + 2 * N, r, n0);
    t[6 * N + r] = a.op.cM * bmm + a.op.cB[0] * bmk + a.op.cB[1] * bkm;
    t[7 * N + r] = a.op.cB[2] * bmm;
    if (a.check) {   // the same products of v, combined as A
      t[8 * N + r] = a.op.cM * bmm + a.op.cA[0] * bmk + a.op.cA[1] * bkm;
      t[9 * N + r] = a.op.cA[2] * bmm;
    }
  }
}

template <bool THETA>
__global__ __launch_bounds__(kB) void k_kron_z(SlotMap sm, KronArgs a) {
  issue_first();
  const int64_t pth = sm.path[blockIdx.y];
  if (!THETA && a.sc && a.sc[pth].done) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = a.nrow;
  const int n0 = a.op.n[0], n1 = a.op.n[1], n2 = a.op.n[2], p = a.op.p[2];
  const int64_t n01 = (int64_t)n0 * n1;
  const double *t = a.t + pth * a.ts;
  const bool chk = THETA && a.check;
  double part = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0;
  if (r < N) {
    const int i2 = (int)(r / n01);
    const bool active = !a.mask || a.mask[r];
    const int64_t g = pth * a.vs + r;
    if (THETA) {
      double rhs = 0.0, rv = 0.0;
      if (active && !a.check_only) {
        const double ax = band_dot(a.op.Mb[2], p, i2, n2, t + 4 * N, r, n01) +
                          band_dot(a.op.Kb[2], p, i2, n2, t + 5 * N, r, n01);
        const double bv = band_dot(a.op.Mb[2], p, i2, n2, t + 6 * N, r, n01) +
                          band_dot(a.op.Kb[2], p, i2, n2, t + 7 * N, r, n01);
        const double f1 = a.F1[a.f1_slot ? (int64_t)blockIdx.y * a.f1s + r : g];
        const double f0 = a.F0[a.f0_slot ? (int64_t)blockIdx.y * a.f0s + r : g];
        rhs = bv + a.theta * f1 + (1.0 - a.theta) * f0;
        part = rhs * rhs;
        rv = rhs - ax;
      }
      if (chk && active) {
        // residual of the step that produced v, against its right-hand side
        const double av = band_dot(a.op.Mb[2], p, i2, n2, t + 8 * N, r, n01) +
                          band_dot(a.op.Kb[2], p, i2, n2, t + 9 * N, r, n01);
        const double bp = a.bprev[g], vv = a.v[g], d = bp - av;
        c0 = d * d;
        c1 = bp * bp;
        c2 = vv * vv;
        if (!a.check_only) a.bprev[g] = rhs;
      }
      if (!a.check_only) a.out[g] = rv;
    } else {
      const double ax = band_dot(a.op.Mb[2], p, i2, n2, t + 4 * N, r, n01) +
                        band_dot(a.op.Kb[2], p, i2, n2, t + 5 * N, r, n01);
      a.out[g] = active ? ax : 0.0;
      part = active ? a.x[g] * ax : 0.0;
    }
  }
  const int64_t wi = r >> 6;
  const bool lead = (threadIdx.x & 63) == 0 && wi < a.np;
  if (!(THETA && a.check_only)) {
    part = wsum(part);                     // lane 0: the sum over these 64 rows
    if (lead) a.part[pth * a.np + wi] = part;
  }
  if (chk) {
    c0 = wsum(c0);
    c1 = wsum(c1);
    c2 = wsum(c2);
    if (lead) {
      double *pc = a.part_chk + pth * 3 * a.np + wi;
      pc[0] = c0;
      pc[a.np] = c1;
      pc[2 * a.np] = c2;
    }
  }
  if (THETA && blockIdx.x == 0 && threadIdx.x == 0 && a.sc_w) a.sc_w[pth].done = 0;
}

void launch_kron(hipStream_t st, const SlotMap &sm, const KronArgs &a, bool theta) {
  if (sm.count <= 0 || a.nrow <= 0) return;
  dim3 g((unsigned)((a.nrow + kB - 1) / kB), (unsigned)sm.count), b(kB);
  if (theta) {
    hipLaunchKernelGGL(k_kron_x<true>, g, b, 0, st, sm, a);
    hipLaunchKernelGGL(k_kron_y<true>, g, b, 0, st, sm, a);
    hipLaunchKernelGGL(k_kron_z<true>, g, b, 0, st, sm, a);
  } else {
    hipLaunchKernelGGL(k_kron_x<false>, g, b, 0, st, sm, a);
    hipLaunchKernelGGL(k_kron_y<false>, g, b, 0, st, sm, a);
    hipLaunchKernelGGL(k_kron_z<false>, g, b, 0, st, sm, a);
  }
}

int stencil_blocks(int64_t nrow) { return (int)((nrow + 63) / 64); }

void launch_stencil_sl(hipStream_t st, const SlotMap &sm, const SlArgs &a, int hw0, bool theta) {
  if (sm.count <= 0) return;
  const int waves = 2 * a.hw2 + 1;
  dim3 g((unsigned)stencil_blocks(a.nrow), (unsigned)sm.count), b(64 * waves);
  const size_t lds = (size_t)(theta ? 2 : 1) * waves * 64 * sizeof(double);
#define SA_SL_CASE(H)                                                                             \
  case H:                                                                                         \
    if (theta) hipLaunchKernelGGL((k_stencil_sl<H, true>), g, b, lds, st, sm, a);                 \
    else hipLaunchKernelGGL((k_stencil_sl<H, false>), g, b, lds, st, sm, a);                      \
    break;
  switch (hw0) {
    SA_SL_CASE(1)
    SA_SL_CASE(2)
    SA_SL_CASE(3)
    SA_SL_CASE(4)
    SA_SL_CASE(5)
    default: SA_SL_CASE(6)
  }
#undef SA_SL_CASE
}

// ---------------------------------------------------------------------------
// fast-diagonalisation solve on the box of free DOFs, fused with the PCG update
// ---------------------------------------------------------------------------
// the data of the path handled by launch slot `slot`
__device__ __forceinline__ FusedPcg at_path(const FusedPcg &f, const SlotMap &sm, int slot) {
  FusedPcg g = f;
  const int64_t p = sm.path[slot];
  if (g.x) g.x += p * f.vs;
  if (g.r) g.r += p * f.vs;
  if (g.z) g.z += p * f.vs;
  if (g.p) g.p += p * f.vs;
  if (g.q) g.q += p * f.vs;
  if (g.t) g.t += p * f.ts;
  if (g.part_rz) g.part_rz += p * 2 * f.np_rz;
  if (g.part_rr) g.part_rr += p * f.np_rz;
  if (g.part_xx) g.part_xx += p * f.np_rz;
  if (g.part_pq) g.part_pq += p * f.np_pq;
  if (g.part_b) g.part_b += p * f.np_b;
  if (g.part_chk) g.part_chk += p * 3 * f.np_chk;
  g.sc += p;
  if (g.status) g.status += slot;
  if (g.scatter_out) g.scatter_out += p * f.sos;
  return g;
}

// status record of a theta-step whose residual was formed afterwards (by the
// next right-hand side pass or a check pass): pc holds the partials of
// |b - A u|^2, |b|^2 and |u|^2 over the free rows, np of each; the test is
// that of k_pcg_dir
__device__ void check_record(const double *pc, int np, double rtol2, double bw2, SolveStatus *st, double *sh) {
  const double rr = reduce_n(pc, np, sh);
  const double bb = reduce_n(pc + np, np, sh);
  const double xx = reduce_n(pc + 2 * np, np, sh);
  if (threadIdx.x == 0) {
    const bool conv = rr <= rtol2 * bb || rr <= bw2 * xx || bb <= 1e-280;
    st->iter = 1;
    st->done = conv ? 1 : 0;
    st->relres2 = bb > 0 ? rr / bb : 0.0;
  }
}

__device__ __forceinline__ int64_t full_index(const FusedPcg &f, int j0, int j1, int j2) {
  return (int64_t)(j0 + f.lo[0]) + (int64_t)f.n[0] * ((j1 + f.lo[1]) + (int64_t)f.n[1] * (j2 + f.lo[2]));
}

// The FD solve on the box of free DOFs, in three launches:
//   k_fd_xfwd   block = x-fiber (k1, k2): optional PCG update of its rows,
//               t[:, k1, k2] = U0^T r[:, k1, k2]
//   k_fd_plane  block = plane j0: modes 1 and 2, eigenvalue scaling, back
//   k_fd_xbwd   block = x-fiber: z = U0 t, partial r.z, p = z on the first pass
//               (checked update: x += z)
// t is stored plane-major: t[j0 * (m1 m2) + k2 * m1 + k1].  The checked
// update uses k_kron_zx in place of k_fd_xfwd and, inside a block of steps,
// k_xbwd_x in place of k_fd_xbwd (both further below).
constexpr int kFib = 64;

__global__ __launch_bounds__(kFib) void k_fd_xfwd(SlotMap sm, FusedPcg f0, int k, int first) {
  issue_first();
  __shared__ double fib[256];
  __shared__ double sh[16];
  const FusedPcg f = at_path(f0, sm, blockIdx.y);
  if (f.sc->done) return;
  const int m0 = f.m[0], m1 = f.m[1];
  const int64_t P = (int64_t)m1 * f.m[2];
  const int b = blockIdx.x;
  const int k1 = b % m1, k2 = b / m1;
  const int64_t base = full_index(f, 0, k1, k2);
  // first: 1 = transform r only; 0 = PCG update, then transform; 2 = update only
  if (first != 1) {
    const double rz = reduce_n(f.part_rz + (k & 1) * f.np_rz, f.np_rz, sh);
    const double pq = reduce_n(f.part_pq, f.np_pq, sh);
    if (rz == 0.0 || !(pq > 0.0)) {
      // zero residual (nothing to solve) or breakdown: record the exit here
      if (b == 0 && threadIdx.x == 0) {   // first fiber block of this path
        const int d = (rz == 0.0) ? 1 : 2;
        f.sc->done = d;
        if (f.status) {
          f.status->iter = k;
          f.status->done = d;
          f.status->relres2 = 0.0;
        }
      }
      return;
    }
    const double alpha = rz / pq;
    double rr = 0.0, xx = 0.0;
    for (int i = threadIdx.x; i < m0; i += blockDim.x) {
      const int64_t g = base + i;
      const double xi = fma(alpha, f.p[g], f.x[g]);
      f.x[g] = xi;
      xx = fma(xi, xi, xx);
      const double ri = fma(-alpha, f.q[g], f.r[g]);
      f.r[g] = ri;
      fib[i] = ri;
      rr = fma(ri, ri, rr);
    }
    rr = bsum(rr, sh);
    xx = bsum(xx, sh);
    if (threadIdx.x == 0) {
      f.part_rr[b] = rr;
      if (f.part_xx) f.part_xx[b] = xx;
    }
    if (first == 2) return;                 // last iteration: no preconditioned residual needed
  } else {
    for (int i = threadIdx.x; i < m0; i += blockDim.x) fib[i] = f.r[base + i];
    __syncthreads();
  }
  for (int j0 = threadIdx.x; j0 < m0; j0 += blockDim.x) {
    double s = 0.0;
    #pragma unroll 8
    for (int kk = 0; kk < m0; ++kk) s = fma(f.U0[kk * m0 + j0], fib[kk], s);
    f.t[(int64_t)j0 * P + (int64_t)k2 * m1 + k1] = s;
  }
}

__global__ void k_fd_plane(SlotMap sm, FusedPcg f0) {
  issue_first();
  extern __shared__ double lds[];
  __shared__ double sh[16];
  const FusedPcg f = at_path(f0, sm, blockIdx.y);
  if (f.sc->done) return;
  if (f.update_x && blockIdx.x == 0 && f.status) {
    // checked update: the record of this path's previous theta-step
    if ((f.check_mask >> blockIdx.y) & 1) {
      check_record(f.part_chk, f.np_chk, f.chk_rtol2, f.chk_bw2, f.status, sh);
    } else if (threadIdx.x == 0) {
      f.status->iter = -1;                 // nothing to check
      f.status->done = 1;
      f.status->relres2 = 0.0;
    }
  }
  const int m0 = f.m[0], m1 = f.m[1], m2 = f.m[2];
  const int P = m1 * m2;
  const int j0 = blockIdx.x;
  // the plane twice and the y and z eigenvector matrices, all in LDS
  double *A = lds, *Bv = lds + P, *U1 = lds + 2 * P, *U2 = U1 + m1 * m1;
  double *t = f.t + (int64_t)j0 * P;
  for (int i = threadIdx.x; i < P; i += blockDim.x) A[i] = t[i];
  for (int i = threadIdx.x; i < m1 * m1; i += blockDim.x) U1[i] = f.U1[i];
  for (int i = threadIdx.x; i < m2 * m2; i += blockDim.x) U2[i] = f.U2[i];
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += blockDim.x) {       // mode 1: U1^T along y
    const int j1 = i % m1, k2 = i / m1;
    double s = 0.0;
    #pragma unroll 8
    for (int kk = 0; kk < m1; ++kk) s = fma(U1[kk * m1 + j1], A[k2 * m1 + kk], s);
    Bv[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += blockDim.x) {       // mode 2: U2^T along z, scale
    const int j1 = i % m1, j2 = i / m1;
    double s = 0.0;
    #pragma unroll 8
    for (int kk = 0; kk < m2; ++kk) s = fma(U2[kk * m2 + j2], Bv[kk * m1 + j1], s);
    A[i] = s * f.inv[j0 + (int64_t)m0 * (j1 + (int64_t)m1 * j2)];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += blockDim.x) {       // mode 2 back
    const int j1 = i % m1, k2 = i / m1;
    double s = 0.0;
    #pragma unroll 8
    for (int j = 0; j < m2; ++j) s = fma(U2[k2 * m2 + j], A[j * m1 + j1], s);
    Bv[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += blockDim.x) {       // mode 1 back
    const int k1 = i % m1, k2 = i / m1;
    double s = 0.0;
    #pragma unroll 8
    for (int j = 0; j < m1; ++j) s = fma(U1[k1 * m1 + j], Bv[k2 * m1 + j], s);
    t[i] = s;
  }
}

__global__ __launch_bounds__(kFib) void k_fd_xbwd(SlotMap sm, FusedPcg f0, int slot, int first) {
  issue_first();
  __shared__ double fib[256];
  __shared__ double sh[16];
  const FusedPcg f = at_path(f0, sm, blockIdx.y);
  if (f.sc->done) return;
  const int m0 = f.m[0], m1 = f.m[1];
  const int64_t P = (int64_t)m1 * f.m[2];
  const int b = blockIdx.x;
  const int k1 = b % m1, k2 = b / m1;
  const int64_t base = full_index(f, 0, k1, k2);
  for (int j = threadIdx.x; j < m0; j += blockDim.x) fib[j] = f.t[(int64_t)j * P + (int64_t)k2 * m1 + k1];
  __syncthreads();
  if (f.update_x) {   // x += P r: one application of the exact inverse
    for (int k0 = threadIdx.x; k0 < m0; k0 += blockDim.x) {
      double s = 0.0;
      if (f.U0T)
        #pragma unroll 8
        for (int j = 0; j < m0; ++j) s = fma(f.U0T[j * m0 + k0], fib[j], s);
      else
        #pragma unroll 8
        for (int j = 0; j < m0; ++j) s = fma(f.U0[k0 * m0 + j], fib[j], s);
      f.x[base + k0] += s;
    }
    return;
  }
  double rz = 0.0;
  for (int k0 = threadIdx.x; k0 < m0; k0 += blockDim.x) {
    double s = 0.0;
    #pragma unroll 8
    for (int j = 0; j < m0; ++j) s = fma(f.U0[k0 * m0 + j], fib[j], s);
    const int64_t g = base + k0;
    f.z[g] = s;
    if (first) f.p[g] = s;
    if (f.scatter_out) f.scatter_out[f.scatter_idx[g]] = s;
    rz = fma(f.r[g], s, rz);
  }
  if (!f.part_rz) return;
  rz = bsum(rz, sh);
  if (threadIdx.x == 0) f.part_rz[slot * f.np_rz + b] = rz;
}

// convergence test on r.r; p = z + beta p on the box
__global__ void k_pcg_dir(SlotMap sm, FusedPcg f0, int k, int last) {
  __shared__ double sh[16];
  const FusedPcg f = at_path(f0, sm, blockIdx.y);
  if (f.sc->done) return;
  const double rr = reduce_n(f.part_rr, f.np_rz, sh);
  const double bb = reduce_n(f.part_b, f.np_b, sh);
  const double xx = f.part_xx ? reduce_n(f.part_xx, f.np_rz, sh) : 0.0;
  // converged: relative residual at the tolerance; or the residual at the
  // FP64 rounding floor of the system (normwise backward error 64 eps), below
  // which no iteration can go; or |b| at the FP64 underflow edge, where the
  // solution is zero to that precision
  const bool conv = rr <= f.rtol2 * bb || rr <= f.bw2 * xx || bb <= 1e-280;
  if (!conv && !last) {
    const double rz_old = reduce_n(f.part_rz + (k & 1) * f.np_rz, f.np_rz, sh);
    const double rz_new = reduce_n(f.part_rz + ((k + 1) & 1) * f.np_rz, f.np_rz, sh);
    const double beta = rz_new / rz_old;
    const int m0 = f.m[0], m1 = f.m[1];
    const int64_t nbox = (int64_t)m0 * m1 * f.m[2];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nbox; t += (int64_t)gridDim.x * blockDim.x) {
      const int64_t i = full_index(f, (int)(t % m0), (int)((t / m0) % m1), (int)(t / ((int64_t)m0 * m1)));
      f.p[i] = fma(beta, f.p[i], f.z[i]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    f.sc->iter = k + 1;
    f.sc->rr = rr;
    f.sc->bnorm2 = bb;
    if (conv) f.sc->done = 1;
    if (f.status) {
      f.status->iter = k + 1;
      f.status->done = conv ? 1 : 0;
      f.status->relres2 = bb > 0 ? rr / bb : 0.0;
    }
  }
}

// one thread per plane entry (up to 1024): each transform is one dot product per thread
unsigned plane_threads(const int m[3]) {
  const int64_t P = (int64_t)m[1] * m[2];
  const int64_t t = (P + 63) / 64 * 64;
  return (unsigned)(t > 1024 ? 1024 : (t < 64 ? 64 : t));
}

bool fused_fits(const int m[3]) { return m[0] <= 256 && (int64_t)m[1] * m[2] <= 4096; }

size_t fd_plane_lds(const int m[3]) {
  return ((size_t)2 * m[1] * m[2] + (size_t)m[1] * m[1] + (size_t)m[2] * m[2]) * sizeof(double);
}

// Checked update, first part: the z pass of the theta right-hand side and
// residual r (as k_kron_z<true> with check) for whole x-rows, R rows per
// block (zx_rows), then the first FD transform t = U0^T r of the rows in the
// free box (as k_fd_xfwd); r stays in LDS.  The residual-check partials are
// summed per block (part_chk: gridDim.x of each kind per path).
//
// The x transforms of these kernels (here and in k_xbwd_x, k_fd_xbwd_rows)
// form, in launches of four paths or more, one transform output for four
// rows per thread (one U0 value, four row values per term), otherwise one
// output per thread; U0 (or U0^T) is read through the caches (staged in LDS,
// its 36 KB per block kept these blocks off the compute units shared with
// the kernel sum, for no gain).  Each sum over kk in ascending order, as in
// the fiber kernels.  Rows of
// a block are consecutive, so each transform output's four rows are four
// consecutive entries of t's plane (plane-major t: t[j0 P + k2 m1 + k1]).
constexpr int kZxThreads = 320;
constexpr int kZxMaxRow = 640;
constexpr int kZxRowsMax = 16;
constexpr int kZxFib = 1280;     // LDS row buffer (doubles): R n0 <= kZxFib

__host__ __device__ inline int zx_rows(int n0) {
  const int r = n0 > 0 ? kZxFib / n0 : 1;
  return r < 1 ? 1 : (r > kZxRowsMax ? kZxRowsMax : r);
}

// rows per block: up to 16 for launches of four paths or more; four for fewer
// paths (more blocks for the latency-bound small grids)
static int rows_for(int n0, int count) {
  const int r = zx_rows(n0);
  return count >= 4 ? r : (r < 4 ? r : 4);
}

// s[q] = sum_kk U(kk, j) v[q][kk] for the four rows q of group rg (rows past
// nr contribute nothing), U(kk, j) = U[kk * m + j]
__device__ __forceinline__ void xform4(const double *U, int m, int j, const double *v, int ldv, int q0, int nq,
                                       double s[4]) {
  s[0] = s[1] = s[2] = s[3] = 0.0;
  const double *v0 = v + (int64_t)q0 * ldv;
  if (nq == 1) {
#pragma unroll 8
    for (int kk = 0; kk < m; ++kk) s[0] = fma(U[kk * m + j], v0[kk], s[0]);
  } else if (nq == 4) {
#pragma unroll 4
    for (int kk = 0; kk < m; ++kk) {
      const double u = U[kk * m + j];
      s[0] = fma(u, v0[kk], s[0]);
      s[1] = fma(u, v0[ldv + kk], s[1]);
      s[2] = fma(u, v0[2 * ldv + kk], s[2]);
      s[3] = fma(u, v0[3 * ldv + kk], s[3]);
    }
  } else {
    for (int kk = 0; kk < m; ++kk) {
      const double u = U[kk * m + j];
      for (int q = 0; q < nq; ++q) s[q] = fma(u, v0[q * ldv + kk], s[q]);
    }
  }
}

__global__ __launch_bounds__(kZxThreads) void k_kron_zx(SlotMap sm, KronArgs a, FusedPcg f0, int R, int G) {
  issue_first();
  __shared__ double fib[kZxFib];
  __shared__ double sh[16];
  const int64_t pth = sm.path[blockIdx.y];
  const FusedPcg f = at_path(f0, sm, blockIdx.y);
  const int n0 = a.op.n[0], n1 = a.op.n[1], n2 = a.op.n[2], p = a.op.p[2];
  const int64_t n01 = (int64_t)n0 * n1, nrows = (int64_t)n1 * n2;
  const int64_t row0 = (int64_t)blockIdx.x * R;
  const int ne = R * n0;
  const int m0 = f.m[0], m1 = f.m[1];
  const double *U0 = f.U0;
  const double *t = a.t + pth * a.ts;
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int64_t row = row0 + e / n0;
    double rv = 0.0;
    if (row < nrows) {
      const int64_t r = row * n0 + e % n0;
      const int i2 = (int)(r / n01);
      const int64_t g = pth * a.vs + r;
      if (a.mask[r]) {
        const double ax = band_dot(a.op.Mb[2], p, i2, n2, t + 4 * a.nrow, r, n01) +
                          band_dot(a.op.Kb[2], p, i2, n2, t + 5 * a.nrow, r, n01);
        const double bv = band_dot(a.op.Mb[2], p, i2, n2, t + 6 * a.nrow, r, n01) +
                          band_dot(a.op.Kb[2], p, i2, n2, t + 7 * a.nrow, r, n01);
        const double f1 = a.F1[a.f1_slot ? (int64_t)blockIdx.y * a.f1s + r : g];
        const double f0 = a.F0[a.f0_slot ? (int64_t)blockIdx.y * a.f0s + r : g];
        const double rhs = bv + a.theta * f1 + (1.0 - a.theta) * f0;
        rv = rhs - ax;
        const double av = band_dot(a.op.Mb[2], p, i2, n2, t + 8 * a.nrow, r, n01) +
                          band_dot(a.op.Kb[2], p, i2, n2, t + 9 * a.nrow, r, n01);
        const double bp = a.bprev[g], vv = a.v[g], d = bp - av;
        c0 = fma(d, d, c0);
        c1 = fma(bp, bp, c1);
        c2 = fma(vv, vv, c2);
        a.bprev[g] = rhs;
      }
    }
    fib[e] = rv;
  }
  c0 = bsum(c0, sh);
  c1 = bsum(c1, sh);
  c2 = bsum(c2, sh);
  if (threadIdx.x == 0) {
    // a.np partials per kind whatever the grid (blocks past it: zeros), so
    // that a later launch of another size reads this step's check
    double *pc = a.part_chk + pth * 3 * a.np;
    pc[blockIdx.x] = c0;
    pc[a.np + blockIdx.x] = c1;
    pc[2 * a.np + blockIdx.x] = c2;
    for (int j = blockIdx.x + gridDim.x; j < a.np; j += gridDim.x) pc[j] = pc[a.np + j] = pc[2 * a.np + j] = 0.0;
    if (blockIdx.x == 0 && a.sc_w) a.sc_w[pth].done = 0;
  }
  // (bsum ends with a barrier: fib is complete)
  const int64_t P = (int64_t)m1 * f.m[2];
  const int ng = (R + G - 1) / G;
  for (int o = threadIdx.x; o < ng * m0; o += blockDim.x) {
    const int j0 = o % m0, q0 = G * (o / m0);
    const int nq = R - q0 < G ? R - q0 : G;
    double sv[4];
    xform4(U0, m0, j0, fib + f.lo[0], n0, q0, nq, sv);
    for (int q = 0; q < nq; ++q) {
      const int64_t row = row0 + q0 + q;
      if (row >= nrows) break;
      const int k1 = (int)(row % n1) - f.lo[1], k2 = (int)(row / n1) - f.lo[2];
      if (k1 < 0 || k1 >= m1 || k2 < 0 || k2 >= f.m[2]) continue;
      f.t[(int64_t)j0 * P + (int64_t)k2 * m1 + k1] = sv[q];
    }
  }
}

bool zx_fits(int n0) { return n0 <= kZxMaxRow; }

// partials per kind of the residual check: the blocks of the smallest rows
// per block
int zx_blocks(const KronOp &op) {
  const int R = rows_for(op.n[0], 1);
  return (int)(((int64_t)op.n[1] * op.n[2] + R - 1) / R);
}

// outputs per thread: four rows with the larger blocks, one otherwise
static int rows_per_output(int R) { return R >= 8 ? 4 : 1; }

void launch_theta_checked_rhs(hipStream_t st, const SlotMap &sm, const KronArgs &a0, const FusedPcg &f,
                              bool with_x) {
  if (sm.count <= 0 || a0.nrow <= 0) return;
  KronArgs a = a0;
  a.np = zx_blocks(a.op);
  dim3 g((unsigned)((a.nrow + kB - 1) / kB), (unsigned)sm.count), b(kB);
  if (with_x) hipLaunchKernelGGL(k_kron_x<true>, g, b, 0, st, sm, a);
  hipLaunchKernelGGL(k_kron_y<true>, g, b, 0, st, sm, a);
  const int R = rows_for(a.op.n[0], sm.count);
  const unsigned nb = (unsigned)(((int64_t)a.op.n[1] * a.op.n[2] + R - 1) / R);
  hipLaunchKernelGGL(k_kron_zx, dim3(nb, (unsigned)sm.count), dim3(kZxThreads), 0, st, sm, a, f, R,
                     rows_per_output(R));
}

// Checked update, last transform: x += U0 t' on R consecutive rows of the
// free box per block (t' read as R consecutive entries of each plane)
__global__ __launch_bounds__(kZxThreads) void k_fd_xbwd_rows(SlotMap sm, FusedPcg f0, int R, int G) {
  issue_first();
  __shared__ double tf[kZxFib];
  const FusedPcg f = at_path(f0, sm, blockIdx.y);
  if (f.sc->done) return;
  const int m0 = f.m[0], m1 = f.m[1];
  const int64_t P = (int64_t)m1 * f.m[2];
  const int64_t row0 = (int64_t)blockIdx.x * R;
  const int nr = P - row0 < R ? (int)(P - row0) : R;
  const double *U0T = f.U0T;
  // tf[q * m0 + j] = t[j P + row0 + q]
  for (int e = threadIdx.x; e < m0 * R; e += blockDim.x) {
    const int j = e / R, q = e % R;
    tf[q * m0 + j] = q < nr ? f.t[(int64_t)j * P + row0 + q] : 0.0;
  }
  __syncthreads();
  const int ng = (nr + G - 1) / G;
  for (int o = threadIdx.x; o < ng * m0; o += blockDim.x) {
    const int k0 = o % m0, q0 = G * (o / m0);
    const int nq = nr - q0 < G ? nr - q0 : G;
    double sv[4];
    xform4(U0T, m0, k0, tf, m0, q0, nq, sv);
    for (int q = 0; q < nq; ++q) {
      const int64_t row = row0 + q0 + q;
      const int k1 = (int)(row % m1), k2 = (int)(row / m1);
      f.x[full_index(f, k0, k1, k2)] += sv[q];
    }
  }
}

void launch_theta_checked_solve(hipStream_t st, const SlotMap &sm, const FusedPcg &f, bool with_xbwd) {
  if (sm.count <= 0) return;
  hipLaunchKernelGGL(k_fd_plane, dim3((unsigned)f.m[0], (unsigned)sm.count), dim3(plane_threads(f.m)),
                     fd_plane_lds(f.m), st, sm, f);
  if (!with_xbwd) return;
  if (!f.U0T) {
    const unsigned nfib = (unsigned)(f.m[1] * f.m[2]);
    hipLaunchKernelGGL(k_fd_xbwd, dim3(nfib, (unsigned)sm.count), dim3(kFib), 0, st, sm, f, 0, 1);
    return;
  }
  const int64_t P = (int64_t)f.m[1] * f.m[2];
  const int R = rows_for(f.m[0], sm.count);
  hipLaunchKernelGGL(k_fd_xbwd_rows, dim3((unsigned)((P + R - 1) / R), (unsigned)sm.count), dim3(kZxThreads), 0,
                     st, sm, f, R, rows_per_output(R));
}

// band products along x of one row (u: the row's values of u^{n+1}) for the
// first iterate (u on the free DOFs, Dirichlet values dv or xi elsewhere)
// and for u; each sum over the band in ascending order.  P < 0: half-width p
// at run time.
template <int P>
__device__ __forceinline__ void xrow_products(const double *__restrict__ bm, const double *__restrict__ bk, int i0,
                                              int n0, const double *u, const uint8_t *__restrict__ mask,
                                              int64_t r, const double *__restrict__ dv,
                                              const int32_t *__restrict__ didx, const double *xi, double &s0,
                                              double &s1, double &s2, double &s3, int p = P) {
  s0 = s1 = s2 = s3 = 0.0;
  if (P >= 0) {
#pragma unroll
    for (int k = 0; k <= 2 * (P < 0 ? 0 : P); ++k) {
      const int jj = i0 - P + k;
      if (jj < 0 || jj >= n0) continue;
      const int64_t q = r + (k - P);
      const double uq = u[jj];
      const double x0 = mask[q] ? uq : (dv ? dv[didx[q]] : xi[q]);
      s0 = fma(bm[k], x0, s0);
      s1 = fma(bk[k], x0, s1);
      s2 = fma(bm[k], uq, s2);
      s3 = fma(bk[k], uq, s3);
    }
  } else {
    const int j0 = i0 - p < 0 ? 0 : i0 - p, j1 = i0 + p > n0 - 1 ? n0 - 1 : i0 + p;
    for (int jj = j0; jj <= j1; ++jj) {
      const int64_t q = r + (jj - i0);
      const double uq = u[jj];
      const double x0 = mask[q] ? uq : (dv ? dv[didx[q]] : xi[q]);
      s0 = fma(bm[jj - i0 + p], x0, s0);
      s1 = fma(bk[jj - i0 + p], x0, s1);
      s2 = fma(bm[jj - i0 + p], uq, s2);
      s3 = fma(bk[jj - i0 + p], uq, s3);
    }
  }
}

// x-rows as in k_kron_zx: the box part of each row's t fiber into LDS, then
// u^{n+1} = x0 + U0 t on the box (stored, and kept in LDS for the row), then
// the band products along x of step n+1's first iterate (u^{n+1} on the free
// DOFs, its Dirichlet values elsewhere) and of u^{n+1}
__global__ __launch_bounds__(kZxThreads) void k_xbwd_x(SlotMap sm, FusedPcg f0, KronArgs a, int R, int G) {
  issue_first();
  __shared__ double tf[kZxFib];
  __shared__ double u[kZxFib];
  const int64_t pth = sm.path[blockIdx.y];
  const FusedPcg f = at_path(f0, sm, blockIdx.y);
  const int n0 = a.op.n[0], n1 = a.op.n[1], p = a.op.p[0];
  const int64_t nrows = (int64_t)n1 * a.op.n[2], N = a.nrow;
  const int64_t row0 = (int64_t)blockIdx.x * R;
  const int ne = R * n0;
  const int m0 = f.m[0], m1 = f.m[1];
  const int64_t P = (int64_t)m1 * f.m[2];
  const double *U0T = f.U0T;
  auto in_box = [&](int64_t row, int &k1, int &k2) {
    k1 = (int)(row % n1) - f.lo[1];
    k2 = (int)(row / n1) - f.lo[2];
    return row < nrows && k1 >= 0 && k1 < m1 && k2 >= 0 && k2 < f.m[2];
  };
  // tf[j m0 + j0] = t[j0 P + (k1, k2 of row j)]: consecutive threads, consecutive rows
  for (int o = threadIdx.x; o < R * m0; o += blockDim.x) {
    const int j0 = o / R, j = o % R;
    int k1, k2;
    tf[j * m0 + j0] = in_box(row0 + j, k1, k2) ? f.t[(int64_t)j0 * P + (int64_t)k2 * m1 + k1] : 0.0;
  }
  // the entries outside the box keep x
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int j = e / n0, k0 = e % n0 - f.lo[0];
    int k1, k2;
    const int64_t row = row0 + j;
    if (row < nrows && !(in_box(row, k1, k2) && k0 >= 0 && k0 < m0)) u[e] = f.x[row * n0 + e % n0];
  }
  __syncthreads();
  const int ng = (R + G - 1) / G;
  for (int o = threadIdx.x; o < ng * m0; o += blockDim.x) {
    const int k0 = o % m0, q0 = G * (o / m0);
    const int nq = R - q0 < G ? R - q0 : G;
    double sv[4];
    xform4(U0T, m0, k0, tf, m0, q0, nq, sv);
    for (int q = 0; q < nq; ++q) {
      int k1, k2;
      const int64_t row = row0 + q0 + q;
      if (!in_box(row, k1, k2)) continue;
      const int64_t r = row * n0 + f.lo[0] + k0;
      const double xv = f.x[r] + sv[q];
      f.x[r] = xv;
      u[(q0 + q) * n0 + f.lo[0] + k0] = xv;
    }
  }
  __syncthreads();
  double *t = a.t + pth * a.ts;
  double *xi = a.x_init + pth * a.vs;
  const double *dv = a.dv ? a.dv + (int64_t)blockIdx.y * a.dvs : nullptr;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int j = e / n0, i0 = e % n0;
    const int64_t row = row0 + j;
    if (row >= nrows) continue;
    const int64_t r = row * n0 + i0;
    const double *bm = a.op.Mb[0] + (int64_t)i0 * (2 * p + 1), *bk = a.op.Kb[0] + (int64_t)i0 * (2 * p + 1);
    double s0, s1, s2, s3;
    switch (p) {
      case 1: xrow_products<1>(bm, bk, i0, n0, u + j * n0, a.mask, r, dv, a.didx, xi, s0, s1, s2, s3); break;
      case 2: xrow_products<2>(bm, bk, i0, n0, u + j * n0, a.mask, r, dv, a.didx, xi, s0, s1, s2, s3); break;
      case 3: xrow_products<3>(bm, bk, i0, n0, u + j * n0, a.mask, r, dv, a.didx, xi, s0, s1, s2, s3); break;
      case 4: xrow_products<4>(bm, bk, i0, n0, u + j * n0, a.mask, r, dv, a.didx, xi, s0, s1, s2, s3); break;
      default: xrow_products<-1>(bm, bk, i0, n0, u + j * n0, a.mask, r, dv, a.didx, xi, s0, s1, s2, s3, p);
    }
    t[r] = s0;
    t[N + r] = s1;
    t[2 * N + r] = s2;
    t[3 * N + r] = s3;
    if (a.mask[r]) xi[r] = u[e];
    else if (dv) xi[r] = dv[a.didx[r]];
  }
}

void launch_xbwd_x(hipStream_t st, const SlotMap &sm, const FusedPcg &f, const KronArgs &a) {
  if (sm.count <= 0) return;
  const int R = rows_for(a.op.n[0], sm.count);
  const unsigned nb = (unsigned)(((int64_t)a.op.n[1] * a.op.n[2] + R - 1) / R);
  hipLaunchKernelGGL(k_xbwd_x, dim3(nb, (unsigned)sm.count), dim3(kZxThreads), 0, st, sm, f, a, R,
                     rows_per_output(R));
}

void launch_fd_pass(hipStream_t st, const SlotMap &sm, const FusedPcg &f, int k, bool first, bool update) {
  if (sm.count <= 0) return;
  const unsigned nfib = (unsigned)(f.m[1] * f.m[2]);
  hipLaunchKernelGGL(k_fd_xfwd, dim3(nfib, (unsigned)sm.count), dim3(kFib), 0, st, sm, f, k, update ? 0 : 1);
  hipLaunchKernelGGL(k_fd_plane, dim3((unsigned)f.m[0], (unsigned)sm.count), dim3(plane_threads(f.m)),
                     fd_plane_lds(f.m), st, sm, f);
  const int slot = first ? 0 : ((k + 1) & 1);
  hipLaunchKernelGGL(k_fd_xbwd, dim3(nfib, (unsigned)sm.count), dim3(kFib), 0, st, sm, f, slot, first ? 1 : 0);
}

void launch_pcg_dir(hipStream_t st, const SlotMap &sm, const FusedPcg &f, int k, bool last) {
  if (sm.count <= 0) return;
  const int64_t nbox = (int64_t)f.m[0] * f.m[1] * f.m[2];
  int64_t blocks = last ? 1 : (nbox + kB - 1) / kB;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_pcg_dir, dim3((unsigned)blocks, (unsigned)sm.count), dim3(kB), 0, st, sm, f, k,
                     last ? 1 : 0);
}

__global__ __launch_bounds__(256) void k_check_status(SlotMap sm, const double *part_chk, int np, double rtol2,
                                                      double bw2, SolveStatus *status) {
  __shared__ double sh[16];
  const int64_t p = sm.path[blockIdx.y];
  check_record(part_chk + p * 3 * np, np, rtol2, bw2, status + blockIdx.y, sh);
}

void launch_check_status(hipStream_t st, const SlotMap &sm, const double *part_chk, int np, double rtol2,
                         double bw2, SolveStatus *status) {
  if (sm.count <= 0) return;
  hipLaunchKernelGGL(k_check_status, dim3(1, (unsigned)sm.count), dim3(256), 0, st, sm, part_chk, np, rtol2, bw2,
                     status);
}

__global__ void k_copy_jobs(SlotMap sm, CopyJob j0, CopyJob j1, CopyJob j2, CopyJob j3) {
  const CopyJob j = blockIdx.z == 0 ? j0 : (blockIdx.z == 1 ? j1 : (blockIdx.z == 2 ? j2 : j3));
  const int64_t s = blockIdx.y, p = sm.path[s];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < j.n; i += (int64_t)gridDim.x * blockDim.x)
    j.dst[p * j.ds + i] = j.src[s * j.ss + i];
}

void launch_copy_jobs(hipStream_t st, const SlotMap &sm, const CopyJob *jobs, int njobs) {
  if (sm.count <= 0 || njobs <= 0 || njobs > 4) return;
  CopyJob j[4] = {};
  int64_t n = 0;
  for (int k = 0; k < njobs; ++k) {
    j[k] = jobs[k];
    n = std::max(n, jobs[k].n);
  }
  int64_t blocks = (n + kB - 1) / kB;
  if (blocks > 256) blocks = 256;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy_jobs, dim3((unsigned)blocks, (unsigned)sm.count, (unsigned)njobs), dim3(kB), 0, st, sm,
                     j[0], j[1], j[2], j[3]);
}

void launch_pcg_last_update(hipStream_t st, const SlotMap &sm, const FusedPcg &f, int k) {
  if (sm.count <= 0) return;
  const unsigned nfib = (unsigned)(f.m[1] * f.m[2]);
  hipLaunchKernelGGL(k_fd_xfwd, dim3(nfib, (unsigned)sm.count), dim3(kFib), 0, st, sm, f, k, 2);
}

// ---------------------------------------------------------------------------
// Dirichlet projection by the exact inverse of a Kronecker trace mass matrix,
// one workgroup per path, everything in LDS
// ---------------------------------------------------------------------------
constexpr int kDD = 1024;

__global__ __launch_bounds__(kDD) void k_dir_direct(SlotMap sm, DirDirect a) {
  extern __shared__ double lds[];
  const int64_t pth = sm.path[blockIdx.x];
  const int na = a.na, nb = a.nb, n = na * nb;
  double *B = lds, *T = lds + n, *Ia = lds + 2 * n, *Ib = Ia + na * na;
  const double *b = a.b + pth * a.vs;
  for (int i = threadIdx.x; i < n; i += kDD) B[i] = b[i];
  for (int i = threadIdx.x; i < na * na; i += kDD) Ia[i] = a.Ia[i];
  for (int i = threadIdx.x; i < nb * nb; i += kDD) Ib[i] = a.Ib[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kDD) {          // along the first in-face direction
    const int j0 = i % na, k1 = i / na;
    double s = 0.0;
    for (int k0 = 0; k0 < na; ++k0) s = fma(Ia[j0 * na + k0], B[k0 + na * k1], s);
    T[i] = s;
  }
  __syncthreads();
  double *vD = a.vD + pth * a.vs, *x = a.xfull ? a.xfull + pth * a.xs : nullptr;
  for (int i = threadIdx.x; i < n; i += kDD) {          // along the second, scaled
    const int j0 = i % na, j1 = i / na;
    double s = 0.0;
    for (int k1 = 0; k1 < nb; ++k1) s = fma(Ib[j1 * nb + k1], T[j0 + na * k1], s);
    s *= a.inv_area;
    vD[i] = s;
    if (a.xfull) x[a.dofs[i]] = s;
  }
}

// the same two passes spread over the chip: one workgroup per column of the
// first in-face direction, then one per row of the second
__global__ __launch_bounds__(64) void k_dir_cols(SlotMap sm, DirDirect a) {
  __shared__ double col[256];
  const int64_t pth = sm.path[blockIdx.y];
  const int na = a.na, k1 = blockIdx.x;
  const double *b = a.b + pth * a.vs + (int64_t)na * k1;
  for (int i = threadIdx.x; i < na; i += 64) col[i] = b[i];
  __syncthreads();
  double *T = a.tmp + pth * (int64_t)na * a.nb + (int64_t)na * k1;
  for (int j0 = threadIdx.x; j0 < na; j0 += 64) {
    double s = 0.0;
    for (int k0 = 0; k0 < na; ++k0) s = fma(a.Ia[j0 * na + k0], col[k0], s);
    T[j0] = s;
  }
}

__global__ __launch_bounds__(64) void k_dir_rows(SlotMap sm, DirDirect a) {
  __shared__ double row[256];
  const int64_t pth = sm.path[blockIdx.y];
  const int na = a.na, nb = a.nb, j0 = blockIdx.x;
  const double *T = a.tmp + pth * (int64_t)na * nb;
  for (int k = threadIdx.x; k < nb; k += 64) row[k] = T[j0 + (int64_t)na * k];
  __syncthreads();
  double *vD = a.vD + pth * a.vs, *x = a.xfull ? a.xfull + pth * a.xs : nullptr;
  for (int j1 = threadIdx.x; j1 < nb; j1 += 64) {
    double s = 0.0;
    for (int k1 = 0; k1 < nb; ++k1) s = fma(a.Ib[j1 * nb + k1], row[k1], s);
    s *= a.inv_area;
    const int64_t i = j0 + (int64_t)na * j1;
    vD[i] = s;
    if (a.xfull) x[a.dofs[i]] = s;
  }
}

size_t dir_direct_lds(int na, int nb) {
  return (size_t)(2 * na * nb + na * na + nb * nb) * sizeof(double);
}

bool dir_direct_prepare(size_t lds) {
  return hipFuncSetAttribute((const void *)k_dir_direct, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
         hipSuccess;
}

void launch_dir_direct(hipStream_t st, const SlotMap &sm, const DirDirect &a) {
  if (sm.count <= 0) return;
  if (a.tmp && a.na <= 256 && a.nb <= 256) {
    hipLaunchKernelGGL(k_dir_cols, dim3((unsigned)a.nb, (unsigned)sm.count), dim3(64), 0, st, sm, a);
    hipLaunchKernelGGL(k_dir_rows, dim3((unsigned)a.na, (unsigned)sm.count), dim3(64), 0, st, sm, a);
    return;
  }
  hipLaunchKernelGGL(k_dir_direct, dim3((unsigned)sm.count), dim3(kDD), dir_direct_lds(a.na, a.nb), st, sm, a);
}

}  // namespace sa
