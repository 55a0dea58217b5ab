// Multi-patch models (C ABI sa_mp_*): NURBS patches glued conformingly by a
// global numbering of their control points (shared control points on the
// interfaces, C0 across them), the parts of Sec. 3.3 built from several
// patches.  Set-up on the host: each patch's matrices (Eqs. 16-17) and
// boundary tables (Eq. 18) as for one patch, scattered to the global
// numbering; the load gather and the Dirichlet projection data (Eqs. 10-11)
// from the joined tables.  A step on the device, one scan path:
//   coefficients of the switched-on sources (Eq. 8), the kernel sum pair by
//   pair at every boundary point (Eqs. 7-8), the reduction to T~, grad T~
//   and the load densities, the load vector and the projection right-hand
//   side as CSR gathers, the projection M_D u_D = b_D and the theta-step
//   (Eq. 20) on the free unknowns with the Dirichlet columns moved to the
//   right-hand side, both by Jacobi-preconditioned conjugate gradients.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "multipatch.h"
#include "sa_internal.h"

namespace {

struct MpHipFail {
  hipError_t e;
  const char *what;
};

inline void mp_check(hipError_t e, const char *what) {
  if (e != hipSuccess) throw MpHipFail{e, what};
}

template <class T>
T *mp_alloc(std::vector<void *> &owned, size_t n) {
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw sa::SaError{SA_ENOMEM, "hipMalloc failed"};
  owned.push_back(p);
  return (T *)p;
}

template <class T>
T *mp_upload(std::vector<void *> &owned, const std::vector<T> &h, hipStream_t st) {
  T *p = mp_alloc<T>(owned, h.size());
  if (!h.empty()) mp_check(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st), "upload");
  return p;
}

// Additive Schwarz preconditioner z = sum_p S_p^T A_p^-1 S_p r over the
// patches, A_p^-1 the fast-diagonalisation solve of patch p's own operator
// (its 1-D factors; exact on an affine patch), S_p the restriction of the
// system's unknowns to the patch's grid (zero where the patch's grid holds no
// unknown of the system).
struct Schwarz {
  bool on = false;
  std::vector<sa::FdOp> fd;        // per patch, device tables
  std::vector<int64_t> off, len;   // per patch: its slice of the concatenated vectors
  int64_t total = 0;
  int64_t *gidx = nullptr;         // [total]: unknown of the system or -1
  int64_t *rowptr = nullptr, *pos = nullptr;   // per unknown: its entries in the concatenated vectors
  double *rp = nullptr, *zp = nullptr;         // [total]
  sa::FdBatch batch{};             // all patches' solves in one launch per mode product (up to kFdBatchMax)
  bool batched = false;
};

struct MpCsr {
  int64_t nrow = 0;
  int64_t *rowptr = nullptr;
  int32_t *col = nullptr;
  double *val = nullptr;
  sa::CsrOp op() const { return sa::CsrOp{nrow, rowptr, col, val}; }
};

MpCsr upload_csr(std::vector<void *> &owned, const sa::Csr &c, hipStream_t st) {
  MpCsr d;
  d.nrow = c.nrow;
  d.rowptr = mp_upload(owned, c.rowptr, st);
  d.col = mp_upload(owned, c.col, st);
  d.val = mp_upload(owned, c.val, st);
  return d;
}

// global CSR from (row, col, value) triples, duplicates summed in input order
sa::Csr csr_from_triples(int64_t nrow, std::vector<int64_t> &r, std::vector<int64_t> &c, std::vector<double> &v) {
  std::vector<size_t> ord(r.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return r[a] != r[b] ? r[a] < r[b] : c[a] < c[b]; });
  sa::Csr m;
  m.nrow = nrow;
  m.rowptr.assign(nrow + 1, 0);
  int64_t pr = -1, pc = -1;
  for (size_t k : ord) {
    if (r[k] == pr && c[k] == pc) {
      m.val.back() += v[k];
      continue;
    }
    pr = r[k];
    pc = c[k];
    m.col.push_back((int32_t)c[k]);
    m.val.push_back(v[k]);
    m.rowptr[r[k] + 1]++;
  }
  for (int64_t i = 0; i < nrow; ++i) m.rowptr[i + 1] += m.rowptr[i];
  return m;
}

}  // namespace

// one scan path: its sources (rows src0 .. src0 + n_src - 1 of the source
// arrays, ticks non-decreasing), its step, its state and its statistics
struct MpPath {
  int64_t src0 = 0, n_src = 0, n_steps = 0, step = 0;
  double *T = nullptr, *G = nullptr;   // boundary fields of the last completed step
  double *w = nullptr, *F = nullptr, *F1 = nullptr, *vD = nullptr, *vDn = nullptr;
  int64_t pcg_its = 0, dir_its = 0;
  double last_relres = 0.0;
};

struct sa_multipatch {
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<void *> owned;
  std::vector<sa::PatchData> P;
  std::vector<std::vector<double>> el_centre, el_xi;   // per patch, for the inverse map (built on first use)
  std::vector<std::vector<int64_t>> gmap;
  sa_material mat{};
  sa_solver_options opt{};
  double center[3] = {0, 0, 0};
  int64_t nd = 0, nq = 0, stride = 0, nD = 0, nI = 0, nnz = 0;
  sa::BoundaryTables bt;
  // scan
  std::vector<int64_t> tick;
  int64_t tau_ticks = 0;
  std::vector<MpPath> paths;
  int ns = 1;
  sa::CoeffParams cp{};
  // device: points and sources
  double *px = nullptr, *py = nullptr, *pz = nullptr, *pq2 = nullptr, *nx = nullptr, *ny = nullptr, *nz = nullptr,
         *wdS = nullptr;
  float *fx = nullptr, *fy = nullptr, *fz = nullptr, *fq2 = nullptr;
  int8_t *role = nullptr;
  double *sx = nullptr, *sy = nullptr, *sz = nullptr, *sE = nullptr, *c64 = nullptr;
  int64_t *stick = nullptr;
  float *c32 = nullptr;
  double *part = nullptr;
  int64_t part_cap = 0;
  // device: work shared by the paths (the state is per path); the step's
  // boundary fields go to Tw, Gw and become the path's when the step completes
  double *Tw = nullptr, *Gw = nullptr, *LD = nullptr, *bD = nullptr;
  double *Bw = nullptr, *AIDvD = nullptr, *bI = nullptr, *xI = nullptr;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double *part_b = nullptr, *part_rz = nullptr, *part_pq = nullptr, *part_rr = nullptr;
  sa::PcgScalars *sc = nullptr, *h_sc = nullptr;
  MpCsr load, dproj, mdir, Bop, AII, AID;
  int64_t *I_idx = nullptr, *D_idx = nullptr;
  double *aii_inv = nullptr, *mdir_inv = nullptr;
  // additive Schwarz over the patches (SA_PRECOND_FD): one per system
  Schwarz as_main, as_dir;
  ~sa_multipatch() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void *x : owned) (void)hipFree(x);
    if (h_sc) (void)hipHostFree(h_sc);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

template <class F>
int mp_guarded(F &&f) {
  try {
    return f();
  } catch (const sa::SaError &e) {
    sa::set_last_error(e.msg);
    return e.code;
  } catch (const MpHipFail &e) {
    sa::set_last_error(std::string(e.what) + ": " + hipGetErrorString(e.e));
    return SA_EDEVICE;
  } catch (const std::bad_alloc &) {
    sa::set_last_error("host allocation failed");
    return SA_ENOMEM;
  } catch (...) {
    sa::set_last_error("unexpected failure");
    return SA_EINVAL;
  }
}

// z = M^-1 r and the partials of r . z (parts_for(n) of them): the additive
// Schwarz solve when it is set up, else Jacobi
void precondition(sa_multipatch *h, const Schwarz &as, const double *inv_diag, int64_t n, const double *r,
                  double *z, double *part, const sa::PcgScalars *sc) {
  const hipStream_t st = h->stream;
  if (!as.on) {
    sa::launch_jacobi(st, n, inv_diag, r, z, part, const_cast<sa::PcgScalars *>(sc));
    return;
  }
  if (as.batched && as.batch.gidx) {
    // the batched solves gather their inputs from r themselves
    sa::launch_fd_batch(st, as.batch, r, as.zp, sc);
  } else if (as.batched) {
    sa::launch_mp_as_gather(st, as.total, as.gidx, r, as.rp, sc);
    sa::launch_fd_batch(st, as.batch, as.rp, as.zp, sc);
  } else {
    sa::launch_mp_as_gather(st, as.total, as.gidx, r, as.rp, sc);
    for (size_t p = 0; p < as.fd.size(); ++p)
      sa::launch_fd(st, as.fd[p], as.len[p], as.rp + as.off[p], as.zp + as.off[p], nullptr,
                    const_cast<sa::PcgScalars *>(sc));
  }
  sa::launch_mp_as_combine(st, n, as.rowptr, as.pos, as.zp, r, z, part, sc);
}

// preconditioned conjugate gradients on A x = b (device arrays of n values;
// x holds the first iterate), to |r| <= rtol |b|
int cg_solve(sa_multipatch *h, const sa::CsrOp &A, const Schwarz &as, const double *inv_diag, const double *b,
             double *x, double *relres) {
  const hipStream_t st = h->stream;
  const int64_t n = A.nrow;
  if (n <= 0) {
    *relres = 0.0;
    return 0;
  }
  const int np = sa::parts_for(n);
  sa::launch_csr_init(st, A, b, x, h->r, h->part_b);
  precondition(h, as, inv_diag, n, h->r, h->z, h->part_rz, nullptr);
  sa::launch_pcg_start(st, n, np, h->part_b, np, h->part_rz, h->z, h->p, h->sc, h->opt.pcg_rtol);
  int chunk = as.on ? 4 : 8;
  for (;;) {
    for (int k = 0; k < chunk; ++k) {
      sa::launch_csr_apply_dot(st, A, h->p, h->q, h->part_pq, h->sc);
      sa::launch_pcg_update(st, n, np, h->part_pq, np, h->part_rz, h->p, h->q, x, h->r, h->part_rr, h->sc);
      precondition(h, as, inv_diag, n, h->r, h->z, h->part_rz, h->sc);
      sa::launch_pcg_direction(st, n, np, np, h->part_rr, h->part_rz, h->z, h->p, h->sc);
    }
    mp_check(hipMemcpyAsync(h->h_sc, h->sc, sizeof(sa::PcgScalars), hipMemcpyDeviceToHost, st), "status copy");
    mp_check(hipStreamSynchronize(st), "sync");
    const sa::PcgScalars s = *h->h_sc;
    // converged; or |b| at the FP64 underflow edge, where no relative test
    // can pass and the solution is zero to that precision
    if (s.done == 1 || s.bnorm2 <= 1e-280) {
      *relres = s.bnorm2 > 0 ? std::sqrt(std::max(s.rr, 0.0) / s.bnorm2) : 0.0;
      return s.iter;
    }
    if (s.done == 2) throw sa::SaError{SA_ENOCONV, "CG breakdown (operator not positive definite)"};
    if (!std::isfinite(s.rz) || !std::isfinite(s.rr)) throw sa::SaError{SA_ENOCONV, "CG produced NaN/Inf"};
    if (s.iter >= h->opt.pcg_max_iter) throw sa::SaError{SA_ENOCONV, "CG did not converge within pcg_max_iter"};
    chunk = std::min({chunk * 2, 64, std::max(1, h->opt.pcg_max_iter - s.iter)});
  }
}

// the device side of a Schwarz preconditioner: per patch its FD tables and
// the map from its grid (`len` entries, entry k of patch p -> unknown
// unk[p][k] of the system, or -1 outside the system or the patch's FD box)
// to the n unknowns.  Left off (Jacobi) if an unknown lies in no patch's box.
void setup_schwarz(sa_multipatch *h, Schwarz &as, const std::vector<const sa::FdData *> &fds,
                   const std::vector<std::vector<int64_t>> &unk, int64_t n) {
  as.on = false;
  if (n <= 0 || fds.empty()) return;
  const hipStream_t st = h->stream;
  const size_t np = fds.size();
  as.fd.resize(np);
  as.off.resize(np);
  as.len.resize(np);
  as.total = 0;
  for (size_t p = 0; p < np; ++p) {
    as.off[p] = as.total;
    as.len[p] = (int64_t)unk[p].size();
    as.total += as.len[p];
  }
  std::vector<int64_t> gidx((size_t)as.total), count((size_t)n + 1, 0);
  for (size_t p = 0; p < np; ++p)
    for (int64_t k = 0; k < as.len[p]; ++k) {
      const int64_t u = unk[p][k];
      gidx[as.off[p] + k] = u;
      if (u >= 0) count[u + 1]++;
    }
  std::vector<int64_t> rowptr((size_t)n + 1, 0), fill((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] = rowptr[i] + count[i + 1];
  std::vector<int64_t> pos((size_t)std::max<int64_t>(rowptr[n], 1));
  for (size_t p = 0; p < np; ++p)   // patch order within each unknown's entries
    for (int64_t k = 0; k < as.len[p]; ++k) {
      const int64_t u = unk[p][k];
      if (u >= 0) pos[rowptr[u] + fill[u]++] = as.off[p] + k;
    }
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] == rowptr[i]) return;
  as.gidx = mp_upload(h->owned, gidx, st);
  as.rowptr = mp_upload(h->owned, rowptr, st);
  as.pos = mp_upload(h->owned, pos, st);
  as.rp = mp_alloc<double>(h->owned, (size_t)as.total);
  as.zp = mp_alloc<double>(h->owned, (size_t)as.total);
  // the entries outside the patches' boxes: zero for good (the batched
  // solves write only their boxes; the one-patch solves zero them again)
  mp_check(hipMemsetAsync(as.zp, 0, (size_t)std::max<int64_t>(as.total, 1) * sizeof(double), st), "memset");
  for (size_t p = 0; p < np; ++p) {
    const sa::FdData &D = *fds[p];
    sa::FdOp &F = as.fd[p];
    const int64_t nbox = (int64_t)D.m[0] * D.m[1] * D.m[2];
    for (int d = 0; d < 3; ++d) {
      F.n[d] = D.n[d];
      F.lo[d] = D.lo[d];
      F.m[d] = D.m[d];
      F.U[d] = mp_upload(h->owned, D.U[d], st);
    }
    F.inv_diag = mp_upload(h->owned, D.inv_diag, st);
    F.t1 = mp_alloc<double>(h->owned, (size_t)nbox);
    F.t2 = mp_alloc<double>(h->owned, (size_t)nbox);
  }
  as.batched = np <= (size_t)sa::kFdBatchMax;
  if (as.batched) {
    as.batch.count = (int)np;
    for (size_t p = 0; p < np; ++p) {
      as.batch.f[p] = as.fd[p];
      as.batch.off[p] = as.off[p];
    }
    as.batch.gidx = sa::fd_batch_in_lds(as.batch) ? as.gidx : nullptr;
  }
  as.on = true;
}

void ensure_part(sa_multipatch *h, int64_t doubles) {
  if (doubles <= h->part_cap) return;
  mp_check(hipStreamSynchronize(h->stream), "sync");
  if (h->part) {
    mp_check(hipFree(h->part), "free");
    h->owned.erase(std::find(h->owned.begin(), h->owned.end(), (void *)h->part));
  }
  h->part_cap = std::max<int64_t>(doubles, 2 * h->part_cap);
  h->part = mp_alloc<double>(h->owned, (size_t)h->part_cap);
}

// sources of path P switched on at tick `now`
int64_t active_sources(const sa_multipatch *h, const MpPath &P, int64_t now) {
  const auto t0 = h->tick.begin() + P.src0;
  return (int64_t)(std::upper_bound(t0, t0 + P.n_src, now) - t0);
}

// one theta-step n -> n+1 of path P
void mp_step_one(sa_multipatch *h, MpPath &P) {
  const hipStream_t st = h->stream;
  const int64_t s1 = P.step + 1, now = s1 * h->ns;
  sa::PathTab tab{};
  tab.count = 1;
  tab.path[0] = 0;
  tab.src0[0] = P.src0;
  tab.now[0] = now;
  const int64_t a = active_sources(h, P, now);
  int64_t f = 0;
  if (h->opt.precision == SA_PREC_FP32_FAR && a > 0) {
    const auto t0 = h->tick.begin() + P.src0;
    f = std::min<int64_t>(a, (int64_t)(std::lower_bound(t0, t0 + a, now - h->tau_ticks) - t0));
  }
  tab.n_act[0] = (int32_t)a;
  tab.n_far[0] = (int32_t)f;
  tab.mode[0] = 0;
  // Eqs. 7-8 at the boundary points, their reduction and the load densities
  if (a > 0) sa::launch_coeff(st, tab, a, h->stick, h->sx, h->sy, h->sz, h->sE, h->cp, h->c64, h->c32);
  sa::SumPlan pl = sa::plan_sum(h->opt, h->nq, 1, f, a - f);
  pl.part_stride = h->stride;
  const int nch = pl.n_chunks_far + pl.n_chunks_near;
  ensure_part(h, (int64_t)std::max(nch, 1) * 5 * h->stride);
  if (nch > 0)
    sa::launch_sum(st, pl, tab, h->px, h->py, h->pz, h->pq2, h->fx, h->fy, h->fz, h->fq2, h->c64, h->c32, h->part);
  sa::launch_finalize(st, tab, true, h->nq, nch, h->stride, h->part, h->px, h->py, h->pz, h->nx, h->ny, h->nz, h->wdS,
                      h->role, h->mat.k, h->stride, h->Tw, h->Gw, h->LD, nullptr, 0);
  // load vector (Eq. 18) and the Dirichlet projection (Eq. 11)
  sa::launch_gather(st, h->load.nrow, h->load.rowptr, h->load.col, h->load.val, h->LD, P.F1);
  double rel = 0.0;
  if (h->nD > 0) {
    sa::launch_gather(st, h->dproj.nrow, h->dproj.rowptr, h->dproj.col, h->dproj.val, h->LD, h->bD);
    mp_check(hipMemcpyAsync(P.vDn, P.vD, h->nD * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
    P.dir_its += cg_solve(h, h->mdir.op(), h->as_dir, h->mdir_inv, h->bD, P.vDn, &rel);
  }
  // theta-scheme (Eq. 20) on the free unknowns
  sa::launch_csr_eval(st, h->nd, h->Bop.rowptr, h->Bop.col, h->Bop.val, P.w, h->Bw);
  if (h->nD > 0) sa::launch_csr_eval(st, h->nI, h->AID.rowptr, h->AID.col, h->AID.val, P.vDn, h->AIDvD);
  sa::launch_mp_rhs(st, h->nI, h->I_idx, h->Bw, P.F1, P.F, h->opt.theta, h->nD > 0 ? h->AIDvD : nullptr, P.w, h->bI,
                    h->xI);
  P.pcg_its += cg_solve(h, h->AII.op(), h->as_main, h->aii_inv, h->bI, h->xI, &rel);
  P.last_relres = rel;
  // commit: u^{n+1}, F^{n+1}, the Dirichlet values
  sa::launch_mp_commit(st, h->nI, h->I_idx, h->xI, h->nD, h->D_idx, P.vDn, P.w);
  std::swap(P.F, P.F1);
  std::swap(P.vD, P.vDn);
  std::swap(P.T, h->Tw);
  std::swap(P.G, h->Gw);
  mp_check(hipGetLastError(), "kernel launch");
  P.step = s1;
}

void setup(sa_multipatch *h, const sa_patch *patches, int32_t n_patches, const int64_t *index_map,
           const sa_material *mat, const sa_scan_path *scan, const sa_solver_options &opt) {
  if (n_patches < 1 || !patches || !index_map) throw sa::SaError{SA_EINVAL, "need at least one patch and the index map"};
  for (int32_t p = 0; p < n_patches; ++p) sa::validate_inputs(&patches[p], mat, scan, opt, true);
  if (opt.precision != SA_PREC_FP64 && opt.precision != SA_PREC_FP32_FAR)
    throw sa::SaError{SA_EINVAL, "multi-patch models take SA_PREC_FP64 or SA_PREC_FP32_FAR"};
  h->mat = *mat;
  h->opt = opt;
  const double dt = scan->dt;
  // per patch: matrices and boundary tables in its own numbering
  std::vector<sa::Model> pm(n_patches);
  int64_t off = 0, nd = 0;
  h->P.resize(n_patches);
  h->gmap.resize(n_patches);
  for (int32_t p = 0; p < n_patches; ++p) {
    sa::Model &m = pm[p];
    m.mat = *mat;
    m.opt = opt;
    m.dt = dt;
    sa::load_patch(&patches[p], m.P);
    h->gmap[p].assign(index_map + off, index_map + off + m.P.ndof);
    off += m.P.ndof;
    for (int64_t g : h->gmap[p]) {
      if (g < 0) throw sa::SaError{SA_EINVAL, "negative global index"};
      nd = std::max(nd, g + 1);
    }
  }
  // the index map: every global index used, joined control points coincide
  {
    std::vector<int64_t> first(nd, -1);
    std::vector<double> ref(4 * nd, 0.0);
    double ext = 0.0;
    for (int32_t p = 0; p < n_patches; ++p)
      for (int64_t A = 0; A < pm[p].P.ndof; ++A)
        for (int c = 0; c < 3; ++c) ext = std::max(ext, std::fabs(pm[p].P.ctrl[4 * A + c]));
    for (int32_t p = 0; p < n_patches; ++p)
      for (int64_t A = 0; A < pm[p].P.ndof; ++A) {
        const int64_t g = h->gmap[p][A];
        const double *c = &pm[p].P.ctrl[4 * A];
        if (first[g] < 0) {
          first[g] = 1;
          std::copy(c, c + 4, &ref[4 * g]);
          continue;
        }
        for (int k = 0; k < 3; ++k)
          if (std::fabs(c[k] - ref[4 * g + k]) > 1e-12 * ext)
            throw sa::SaError{SA_EINVAL, "the index map joins control points at different positions"};
        if (std::fabs(c[3] - ref[4 * g + 3]) > 1e-12 * std::fabs(ref[4 * g + 3]))
          throw sa::SaError{SA_EINVAL, "the index map joins control points of different weights"};
      }
    for (int64_t g = 0; g < nd; ++g)
      if (first[g] < 0) throw sa::SaError{SA_EINVAL, "the index map leaves a global index unused"};
  }
  h->nd = nd;
  // the inputs are valid: from here on the device
  mp_check(hipGetDevice(&h->device), "device");
  mp_check(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking), "stream");
  const hipStream_t st = h->stream;
  for (int c = 0; c < 3; ++c) {
    double lo = 1e300, hi = -1e300;
    for (auto &m : pm)
      for (int64_t A = 0; A < m.P.ndof; ++A) {
        lo = std::min(lo, m.P.ctrl[4 * A + c]);
        hi = std::max(hi, m.P.ctrl[4 * A + c]);
      }
    h->center[c] = 0.5 * (lo + hi);
  }
  // Eqs. 16-17 patch by patch, scattered to the global numbering
  std::vector<int64_t> rM, cM;
  std::vector<double> vM, vK;
  std::vector<uint8_t> free_mask(nd, 1);
  sa::BoundaryTables &bt = h->bt;
  bt.nq = 0;
  bt.fptr.assign(1, 0);
  for (int32_t p = 0; p < n_patches; ++p) {
    sa::Model &m = pm[p];
    sa::assemble_volume(m);
    sa::build_boundary(m);
    const auto &g = h->gmap[p];
    const sa::Stencil &S = m.M;
    for (int o = 0; o < S.n_off; ++o) {
      const int d0 = o % (2 * S.hw[0] + 1) - S.hw[0];
      const int d1 = (o / (2 * S.hw[0] + 1)) % (2 * S.hw[1] + 1) - S.hw[1];
      const int d2 = o / ((2 * S.hw[0] + 1) * (2 * S.hw[1] + 1)) - S.hw[2];
      for (int64_t A = 0; A < S.nrow; ++A) {
        const double mv = S.val[(size_t)o * S.nrow + A], kv = m.K.val[(size_t)o * S.nrow + A];
        if (mv == 0.0 && kv == 0.0) continue;
        const int a0 = (int)(A % S.n[0]) + d0, a1 = (int)((A / S.n[0]) % S.n[1]) + d1,
                  a2 = (int)(A / ((int64_t)S.n[0] * S.n[1])) + d2;
        if (a0 < 0 || a0 >= S.n[0] || a1 < 0 || a1 >= S.n[1] || a2 < 0 || a2 >= S.n[2]) continue;
        const int64_t B = a0 + (int64_t)S.n[0] * (a1 + (int64_t)S.n[1] * a2);
        rM.push_back(g[A]);
        cM.push_back(g[B]);
        vM.push_back(mv);
        vK.push_back(kv);
      }
    }
    // boundary points of the patch's non-interface faces, basis indices global
    const sa::BoundaryTables &b = m.bt;
    const int64_t base = bt.nq;
    bt.x.insert(bt.x.end(), b.x.begin(), b.x.end());
    bt.nrm.insert(bt.nrm.end(), b.nrm.begin(), b.nrm.end());
    bt.wdS.insert(bt.wdS.end(), b.wdS.begin(), b.wdS.end());
    bt.role.insert(bt.role.end(), b.role.begin(), b.role.end());
    for (int64_t i = 0; i < b.nq; ++i) {
      for (int64_t e = b.fptr[i]; e < b.fptr[i + 1]; ++e) {
        bt.fidx.push_back(g[b.fidx[e]]);
        bt.fval.push_back(b.fval[e]);
      }
      bt.fptr.push_back((int64_t)bt.fidx.size());
    }
    bt.nq = base + b.nq;
    for (int64_t A = 0; A < m.P.ndof; ++A)
      if (!m.free_mask[A]) free_mask[g[A]] = 0;
    h->P[p] = m.P;
  }
  for (int f = 0; f <= 6; ++f) bt.face_off[f] = 0;
  std::vector<int64_t> cK = cM, rK = rM;
  sa::Csr Mg = csr_from_triples(nd, rM, cM, vM);
  sa::Csr Kg = csr_from_triples(nd, rK, cK, vK);
  h->nnz = (int64_t)Mg.col.size();
  // A = M/dt + theta K, B = M/dt - (1 - theta) K (same sparsity)
  const double th = opt.theta;
  sa::Csr Bc = Mg, Ac = Mg;
  for (size_t e = 0; e < Mg.val.size(); ++e) {
    Ac.val[e] = Mg.val[e] / dt + th * Kg.val[e];
    Bc.val[e] = Mg.val[e] / dt - (1.0 - th) * Kg.val[e];
  }
  // load gather, Dirichlet unknowns, projection data from the joined tables
  sa::Csr L, Dp, Md;
  std::vector<int64_t> dir_dofs;
  sa::build_transfer(bt, nd, free_mask, L, dir_dofs, Dp, Md);
  h->nD = (int64_t)dir_dofs.size();
  std::vector<int64_t> I, pos(nd, -1), dpos(nd, -1);
  for (int64_t A = 0; A < nd; ++A)
    if (free_mask[A]) {
      pos[A] = (int64_t)I.size();
      I.push_back(A);
    }
  for (int64_t j = 0; j < h->nD; ++j) dpos[dir_dofs[j]] = j;
  h->nI = (int64_t)I.size();
  sa::Csr AII, AID;
  AII.nrow = AID.nrow = h->nI;
  AII.rowptr.assign(1, 0);
  AID.rowptr.assign(1, 0);
  std::vector<double> aii_inv(std::max<int64_t>(h->nI, 1), 1.0);
  for (int64_t i = 0; i < h->nI; ++i) {
    const int64_t A = I[i];
    for (int64_t e = Ac.rowptr[A]; e < Ac.rowptr[A + 1]; ++e) {
      const int64_t B = Ac.col[e];
      if (pos[B] >= 0) {
        AII.col.push_back((int32_t)pos[B]);
        AII.val.push_back(Ac.val[e]);
        if (B == A) aii_inv[i] = 1.0 / Ac.val[e];
      } else {
        AID.col.push_back((int32_t)dpos[B]);
        AID.val.push_back(Ac.val[e]);
      }
    }
    AII.rowptr.push_back((int64_t)AII.col.size());
    AID.rowptr.push_back((int64_t)AID.col.size());
  }
  std::vector<double> md_inv(std::max<int64_t>(h->nD, 1), 1.0);
  for (int64_t j = 0; j < h->nD; ++j)
    for (int64_t e = Md.rowptr[j]; e < Md.rowptr[j + 1]; ++e)
      if (Md.col[e] == j) md_inv[j] = 1.0 / Md.val[e];
  // additive Schwarz: each patch's FD solve of its own operator (A = M/dt +
  // theta K on its box of free control points; the trace mass matrix on its
  // Dirichlet face)
  if (opt.preconditioner == SA_PRECOND_FD) {
    bool fd_ok = true;
    for (auto &m : pm) {
      try {
        sa::build_fd(m);
      } catch (const sa::SaError &) {
        fd_ok = false;
      }
    }
    if (fd_ok) {
      std::vector<const sa::FdData *> fds;
      std::vector<std::vector<int64_t>> unk;
      for (int32_t p = 0; p < n_patches; ++p) {
        const sa::FdData &D = pm[p].fd_main;
        const int *n3 = pm[p].P.n;
        std::vector<int64_t> u((size_t)pm[p].P.ndof, -1);
        for (int64_t A = 0; A < pm[p].P.ndof; ++A) {
          const int i[3] = {(int)(A % n3[0]), (int)((A / n3[0]) % n3[1]), (int)(A / ((int64_t)n3[0] * n3[1]))};
          bool inside = true;
          for (int d = 0; d < 3; ++d) inside = inside && i[d] >= D.lo[d] && i[d] < D.lo[d] + D.m[d];
          if (inside) u[A] = pos[h->gmap[p][A]];
        }
        fds.push_back(&D);
        unk.push_back(std::move(u));
      }
      setup_schwarz(h, h->as_main, fds, unk, h->nI);
      // the Dirichlet projection: patches with one Dirichlet face
      fds.clear();
      unk.clear();
      bool dir_ok = h->nD > 0;
      for (int32_t p = 0; p < n_patches && dir_ok; ++p) {
        const sa::PatchData &P = pm[p].P;
        int nf = 0, face = -1;
        for (int f = 0; f < 6; ++f)
          if (P.role[f] == SA_FACE_DIRICHLET) {
            nf++;
            face = f;
          }
        if (nf == 0) continue;
        if (!pm[p].fd_dir_ok) {
          dir_ok = false;
          break;
        }
        const int d = face / 2, a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
        const int layer = face % 2 == 0 ? 0 : P.n[d] - 1;
        std::vector<int64_t> u((size_t)P.n[a] * P.n[b], -1);
        for (int ib = 0; ib < P.n[b]; ++ib)
          for (int ia = 0; ia < P.n[a]; ++ia) {
            int i[3];
            i[d] = layer;
            i[a] = ia;
            i[b] = ib;
            const int64_t A = i[0] + (int64_t)P.n[0] * (i[1] + (int64_t)P.n[1] * i[2]);
            u[ia + (size_t)P.n[a] * ib] = dpos[h->gmap[p][A]];
          }
        fds.push_back(&pm[p].fd_dir);
        unk.push_back(std::move(u));
      }
      if (dir_ok) setup_schwarz(h, h->as_dir, fds, unk, h->nD);
    }
  }
  // device: operators and index lists
  h->Bop = upload_csr(h->owned, Bc, st);
  h->AII = upload_csr(h->owned, AII, st);
  h->AID = upload_csr(h->owned, AID, st);
  h->load = upload_csr(h->owned, L, st);
  h->dproj = upload_csr(h->owned, Dp, st);
  h->mdir = upload_csr(h->owned, Md, st);
  h->I_idx = mp_upload(h->owned, I, st);
  h->D_idx = mp_upload(h->owned, dir_dofs, st);
  h->aii_inv = mp_upload(h->owned, aii_inv, st);
  h->mdir_inv = mp_upload(h->owned, md_inv, st);
  // boundary points (centred coordinates)
  h->nq = bt.nq;
  h->stride = (bt.nq + 63) / 64 * 64;
  {
    const int64_t n = bt.nq;
    std::vector<double> x(n), y(n), zz(n), q2(n), nx(n), ny(n), nz(n);
    std::vector<float> fx(n), fy(n), fz(n), fq(n);
    for (int64_t i = 0; i < n; ++i) {
      x[i] = bt.x[3 * i] - h->center[0];
      y[i] = bt.x[3 * i + 1] - h->center[1];
      zz[i] = bt.x[3 * i + 2] - h->center[2];
      q2[i] = x[i] * x[i] + y[i] * y[i] + zz[i] * zz[i];
      nx[i] = bt.nrm[3 * i];
      ny[i] = bt.nrm[3 * i + 1];
      nz[i] = bt.nrm[3 * i + 2];
      fx[i] = (float)x[i];
      fy[i] = (float)y[i];
      fz[i] = (float)zz[i];
      fq[i] = (float)q2[i];
    }
    h->px = mp_upload(h->owned, x, st);
    h->py = mp_upload(h->owned, y, st);
    h->pz = mp_upload(h->owned, zz, st);
    h->pq2 = mp_upload(h->owned, q2, st);
    h->fx = mp_upload(h->owned, fx, st);
    h->fy = mp_upload(h->owned, fy, st);
    h->fz = mp_upload(h->owned, fz, st);
    h->fq2 = mp_upload(h->owned, fq, st);
    h->nx = mp_upload(h->owned, nx, st);
    h->ny = mp_upload(h->owned, ny, st);
    h->nz = mp_upload(h->owned, nz, st);
    h->wdS = mp_upload(h->owned, bt.wdS, st);
    h->role = mp_upload(h->owned, bt.role, st);
    mp_check(hipStreamSynchronize(st), "sync");
  }
  // sources (centred), the paths' one after another
  const int64_t N = scan->src_offset[scan->n_paths];
  h->paths.resize(scan->n_paths);
  for (int k = 0; k < scan->n_paths; ++k) {
    MpPath &P = h->paths[k];
    P.src0 = scan->src_offset[k];
    P.n_src = scan->src_offset[k + 1] - P.src0;
    P.n_steps = scan->n_steps[k];
    if (P.n_src > 2000000000) throw sa::SaError{SA_EINVAL, "a path holds more than 2e9 sources"};
  }
  h->tick.assign(scan->tick, scan->tick + N);
  {
    std::vector<double> x(N), y(N), zz(N), E(N);
    for (int64_t i = 0; i < N; ++i) {
      x[i] = scan->xyz[3 * i] - h->center[0];
      y[i] = scan->xyz[3 * i + 1] - h->center[1];
      zz[i] = scan->xyz[3 * i + 2] - h->center[2];
      E[i] = scan->energy[i];
    }
    h->sx = mp_upload(h->owned, x, st);
    h->sy = mp_upload(h->owned, y, st);
    h->sz = mp_upload(h->owned, zz, st);
    h->sE = mp_upload(h->owned, E, st);
    h->stick = mp_upload(h->owned, h->tick, st);
  }
  h->ns = scan->sources_per_step;
  const double rc = mat->rho * mat->cp, alpha = mat->k / rc;
  h->cp = sa::CoeffParams{dt / scan->sources_per_step, scan->spot_radius * scan->spot_radius / (8.0 * alpha), alpha, rc,
                          opt.kernel_scale};
  h->tau_ticks = (int64_t)std::floor(opt.tau_near / h->cp.delta + 1e-9);
  h->c64 = mp_alloc<double>(h->owned, (size_t)std::max<int64_t>(N, 1) * sa::kCoefStride);
  h->c32 = mp_alloc<float>(h->owned, (size_t)std::max<int64_t>(N, 1) * sa::kCoefStride);
  // fields, state (u = T_c: w = 0, F = 0, Dirichlet deviations 0) and work
  auto zeros = [&](int64_t n) {
    double *d = mp_alloc<double>(h->owned, (size_t)std::max<int64_t>(n, 1));
    mp_check(hipMemsetAsync(d, 0, std::max<int64_t>(n, 1) * sizeof(double), st), "memset");
    return d;
  };
  for (MpPath &P : h->paths) {
    P.T = zeros(h->stride);
    P.G = zeros(3 * h->stride);
    P.w = zeros(nd);
    P.F = zeros(nd);
    P.F1 = zeros(nd);
    P.vD = zeros(h->nD);
    P.vDn = zeros(h->nD);
  }
  h->Tw = zeros(h->stride);
  h->Gw = zeros(3 * h->stride);
  h->LD = zeros(h->stride);
  h->Bw = zeros(nd);
  h->bD = zeros(h->nD);
  h->AIDvD = zeros(h->nI);
  h->bI = zeros(h->nI);
  h->xI = zeros(h->nI);
  const int64_t nmax = std::max(h->nI, h->nD);
  h->r = zeros(nmax);
  h->z = zeros(nmax);
  h->p = zeros(nmax);
  h->q = zeros(nmax);
  const int npart = sa::parts_for(nmax);
  h->part_b = zeros(npart);
  h->part_rz = zeros(npart);
  h->part_pq = zeros(npart);
  h->part_rr = zeros(npart);
  h->sc = mp_alloc<sa::PcgScalars>(h->owned, 1);
  mp_check(hipHostMalloc((void **)&h->h_sc, sizeof(sa::PcgScalars), hipHostMallocDefault), "pinned allocation");
  mp_check(hipStreamSynchronize(st), "sync");
}

// At n parametric points xi [n][3] of patch `patch` (SA_ERANGE outside
// [0,1]^3): the physical points x [n][3], and on the device (buffers in
// tmp, work on the object's stream) the basis rows with global columns
// (R and the physical gradients) and the source field T~, grad T~ [3][stride]
// of path `path` at its current step
struct MpPoints {
  int64_t stride = 0;
  std::vector<double> x;
  int64_t *rp = nullptr;
  int32_t *cl = nullptr;
  double *vals[4] = {nullptr, nullptr, nullptr, nullptr};
  double *dT = nullptr, *dG = nullptr;
};

MpPoints mp_points(sa_multipatch *h, const MpPath &path, int32_t patch, int64_t n, const double *xi,
                   std::vector<void *> &tmp) {
  MpPoints out;
  const sa::PatchData &P = h->P[patch];
  const auto &g = h->gmap[patch];
  // host basis tables of the points (global column indices), physical points
  std::vector<int64_t> rowptr(1, 0);
  std::vector<int32_t> col;
  std::vector<double> R, gx, gy, gz, xp(3 * n);
  sa::PointEval pe;
  for (int64_t i = 0; i < n; ++i) {
    double u[3];
    int span[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = xi[3 * i + d];
      if (!(u[d] >= 0.0 && u[d] <= 1.0)) throw sa::SaError{SA_ERANGE, "query point outside [0,1]^3"};
      span[d] = P.b[d].find_span(u[d]);
    }
    sa::eval_point(P, u, span, pe);
    const double(&J)[3][3] = pe.J;
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
    for (int l = 0; l < pe.L; ++l) {
      col.push_back((int32_t)g[pe.idx[l]]);
      R.push_back(pe.R[l]);
      double gg[3];
      for (int c = 0; c < 3; ++c) gg[c] = pe.dR[l][0] * Ji[0][c] + pe.dR[l][1] * Ji[1][c] + pe.dR[l][2] * Ji[2][c];
      gx.push_back(gg[0]);
      gy.push_back(gg[1]);
      gz.push_back(gg[2]);
    }
    rowptr.push_back((int64_t)col.size());
    for (int c = 0; c < 3; ++c) xp[3 * i + c] = pe.x[c] - h->center[c];
  }
  const hipStream_t st = h->stream;
  // the basis rows on the device
  out.rp = mp_upload(tmp, rowptr, st);
  out.cl = mp_upload(tmp, col, st);
  out.vals[0] = mp_upload(tmp, R, st);
  out.vals[1] = mp_upload(tmp, gx, st);
  out.vals[2] = mp_upload(tmp, gy, st);
  out.vals[3] = mp_upload(tmp, gz, st);
  // T~ and its gradient at the mapped points (the sources of the current step)
  const int64_t stride = (n + 63) / 64 * 64;
  std::vector<double> qx(n), qy(n), qz(n), q2(n);
  std::vector<float> fx(n), fy(n), fz(n), fq(n);
  for (int64_t i = 0; i < n; ++i) {
    qx[i] = xp[3 * i];
    qy[i] = xp[3 * i + 1];
    qz[i] = xp[3 * i + 2];
    q2[i] = qx[i] * qx[i] + qy[i] * qy[i] + qz[i] * qz[i];
    fx[i] = (float)qx[i];
    fy[i] = (float)qy[i];
    fz[i] = (float)qz[i];
    fq[i] = (float)q2[i];
  }
  double *dx = mp_upload(tmp, qx, st), *dy = mp_upload(tmp, qy, st), *dz = mp_upload(tmp, qz, st),
         *dq = mp_upload(tmp, q2, st);
  float *ex = mp_upload(tmp, fx, st), *ey = mp_upload(tmp, fy, st), *ez = mp_upload(tmp, fz, st),
        *eq = mp_upload(tmp, fq, st);
  std::vector<int8_t> rl(n, (int8_t)SA_FACE_SOURCE_PLANE);   // no load density at query points
  int8_t *drl = mp_upload(tmp, rl, st);
  double *dT = mp_alloc<double>(tmp, stride), *dG = mp_alloc<double>(tmp, 3 * stride),
         *dLD = mp_alloc<double>(tmp, stride);
  out.dT = dT;
  out.dG = dG;
  out.stride = stride;
  sa::PathTab tab{};
  tab.count = 1;
  tab.src0[0] = path.src0;
  tab.now[0] = path.step * h->ns;
  tab.n_act[0] = (int32_t)active_sources(h, path, tab.now[0]);
  tab.n_far[0] = 0;
  const int64_t a = tab.n_act[0];
  if (a > 0) sa::launch_coeff(st, tab, a, h->stick, h->sx, h->sy, h->sz, h->sE, h->cp, h->c64, h->c32);
  sa::SumPlan pl = sa::plan_sum(h->opt, n, 1, 0, a);
  pl.part_stride = stride;
  const int nch = pl.n_chunks_far + pl.n_chunks_near;
  double *part = mp_alloc<double>(tmp, (size_t)std::max(nch, 1) * 5 * stride);
  if (nch > 0) sa::launch_sum(st, pl, tab, dx, dy, dz, dq, ex, ey, ez, eq, h->c64, h->c32, part);
  sa::launch_finalize(st, tab, true, n, nch, stride, part, dx, dy, dz, dx, dy, dz, dq, drl, h->mat.k, stride, dT, dG,
                      dLD, nullptr, 0);  out.x.resize((size_t)3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) out.x[3 * i + c] = xp[3 * i + c] + h->center[c];
  return out;
}

const MpPath &path_at(const sa_multipatch *h, int32_t path) {
  if (path < 0 || path >= (int32_t)h->paths.size()) throw sa::SaError{SA_ERANGE, "path index out of range"};
  return h->paths[path];
}

struct TmpFree {
  std::vector<void *> v;
  ~TmpFree() {
    for (void *p : v) (void)hipFree(p);
  }
};

}  // namespace

extern "C" {

int sa_mp_setup(const sa_patch *patches, int32_t n_patches, const int64_t *index_map, const sa_material *mat,
                const sa_scan_path *scan, sa_multipatch **out) {
  return mp_guarded([&]() -> int {
    if (!out) throw sa::SaError{SA_EINVAL, "NULL out"};
    *out = nullptr;
    if (!scan || !mat) throw sa::SaError{SA_EINVAL, "NULL material or scan path"};
    sa_solver_options o{};
    if (scan->opt) {
      o = *scan->opt;
    } else {
      sa_iga_default_options(&o);
    }
    auto *h = new sa_multipatch();
    try {
      setup(h, patches, n_patches, index_map, mat, scan, o);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return SA_OK;
  });
}

int sa_mp_step(sa_multipatch *h, int32_t n_steps) {
  return mp_guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    if (n_steps < 0) throw sa::SaError{SA_EINVAL, "negative step count"};
    for (MpPath &P : h->paths)
      for (int32_t k = 0; k < n_steps && P.step < P.n_steps; ++k) {
        // the state of the last completed step survives a failing solve
        try {
          mp_step_one(h, P);
        } catch (const sa::SaError &) {
          (void)hipStreamSynchronize(h->stream);
          throw;
        }
      }
    mp_check(hipStreamSynchronize(h->stream), "sync");
    return SA_OK;
  });
}

int sa_mp_get_info(const sa_multipatch *h, int32_t path, sa_mp_info *info) {
  return mp_guarded([&]() -> int {
    if (!h || !info) throw sa::SaError{SA_EINVAL, "NULL argument"};
    const MpPath &P = path_at(h, path);
    *info = sa_mp_info{};
    info->n_paths = (int32_t)h->paths.size();
    info->n_patches = (int32_t)h->P.size();
    info->n_dof = h->nd;
    info->n_bpts = h->nq;
    info->n_dirichlet = h->nD;
    info->n_free = h->nI;
    info->nnz = h->nnz;
    info->step = P.step;
    info->n_steps = P.n_steps;
    info->pcg_iterations = P.pcg_its;
    info->dirichlet_iterations = P.dir_its;
    info->pcg_last_relres = P.last_relres;
    return SA_OK;
  });
}

int sa_mp_get_boundary_fields(sa_multipatch *h, int32_t path, double *T_gp, double *grad_gp, double *F,
                              double *du) {
  return mp_guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    const MpPath &P = path_at(h, path);
    const hipStream_t st = h->stream;
    if (T_gp) mp_check(hipMemcpyAsync(T_gp, P.T, h->nq * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    if (grad_gp)
      for (int c = 0; c < 3; ++c)
        mp_check(hipMemcpyAsync(grad_gp + c * h->nq, P.G + c * h->stride, h->nq * sizeof(double),
                                hipMemcpyDeviceToHost, st),
                 "download");
    if (F) mp_check(hipMemcpyAsync(F, P.F, h->nd * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    if (du) mp_check(hipMemcpyAsync(du, P.w, h->nd * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    mp_check(hipStreamSynchronize(st), "sync");
    return SA_OK;
  });
}

int sa_mp_eval_temperature_at(sa_multipatch *h, int32_t path, int64_t n, const double *x, double *T, double *grad,
                              int32_t *patch, double *xi_out) {
  return mp_guarded([&]() -> int {
    if (!h || (n > 0 && (!x || !T))) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (n < 0) throw sa::SaError{SA_EINVAL, "negative size"};
    (void)path_at(h, path);
    if (n == 0) return SA_OK;
    const int np = (int)h->P.size();
    if (h->el_centre.empty()) {
      h->el_centre.resize(np);
      h->el_xi.resize(np);
      for (int p = 0; p < np; ++p) sa::element_centres(h->P[p], h->el_centre[p], h->el_xi[p]);
    }
    // the first patch (in order) whose inverse map reaches the point
    std::vector<int32_t> owner((size_t)n, -1);
    std::vector<double> xi((size_t)3 * n, NAN);
    for (int p = 0; p < np; ++p) {
      const double tol = sa::locate_tolerance(h->P[p]);
      for (int64_t i = 0; i < n; ++i) {
        if (owner[i] >= 0) continue;
        double q[3];
        if (sa::locate_point(h->P[p], h->el_centre[p], h->el_xi[p], x + 3 * i, tol, q)) {
          owner[i] = p;
          for (int c = 0; c < 3; ++c) xi[3 * i + c] = q[c];
        }
      }
    }
    for (int64_t i = 0; i < n; ++i) {
      T[i] = NAN;
      if (grad)
        for (int c = 0; c < 3; ++c) grad[3 * i + c] = NAN;
    }
    for (int p = 0; p < np; ++p) {
      std::vector<int64_t> idx;
      std::vector<double> q;
      for (int64_t i = 0; i < n; ++i)
        if (owner[i] == p) {
          idx.push_back(i);
          for (int c = 0; c < 3; ++c) q.push_back(xi[3 * i + c]);
        }
      if (idx.empty()) continue;
      const int64_t m = (int64_t)idx.size();
      std::vector<double> Tp((size_t)m), Gp((size_t)3 * m);
      const int rc = sa_mp_eval_temperature(h, path, p, m, q.data(), Tp.data(), Gp.data());
      if (rc != SA_OK) throw sa::SaError{rc, sa_iga_last_error()};
      for (int64_t k = 0; k < m; ++k) {
        T[idx[k]] = Tp[k];
        if (grad)
          for (int c = 0; c < 3; ++c) grad[3 * idx[k] + c] = Gp[3 * k + c];
      }
    }
    if (patch) std::copy(owner.begin(), owner.end(), patch);
    if (xi_out) std::copy(xi.begin(), xi.end(), xi_out);
    return SA_OK;
  });
}

int sa_mp_get_boundary_points(sa_multipatch *h, double *x, double *normal, double *wdS) {
  return mp_guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    if (x) std::memcpy(x, h->bt.x.data(), h->bt.x.size() * sizeof(double));
    if (normal) std::memcpy(normal, h->bt.nrm.data(), h->bt.nrm.size() * sizeof(double));
    if (wdS) std::memcpy(wdS, h->bt.wdS.data(), h->bt.wdS.size() * sizeof(double));
    return SA_OK;
  });
}

int sa_mp_eval_temperature(sa_multipatch *h, int32_t path, int32_t patch, int64_t n, const double *xi, double *T,
                           double *grad) {
  return mp_guarded([&]() -> int {
    if (!h || (n > 0 && (!xi || !T))) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (n < 0) throw sa::SaError{SA_EINVAL, "negative size"};
    const MpPath &pth = path_at(h, path);
    if (patch < 0 || patch >= (int32_t)h->P.size()) throw sa::SaError{SA_ERANGE, "patch index out of range"};
    if (n == 0) return SA_OK;
    const hipStream_t st = h->stream;
    TmpFree tf;
    const MpPoints pts = mp_points(h, pth, patch, n, xi, tf.v);
    // T^ and its gradient: the contractions with the control values
    double *hat = mp_alloc<double>(tf.v, 4 * n);
    for (int k = 0; k < 4; ++k) sa::launch_csr_eval(st, n, pts.rp, pts.cl, pts.vals[k], pth.w, hat + k * n);
    const double *dT = pts.dT, *dG = pts.dG;
    const int64_t stride = pts.stride;
    std::vector<double> hv(4 * n), tt(n), tg(3 * n);
    mp_check(hipMemcpyAsync(hv.data(), hat, 4 * n * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    mp_check(hipMemcpyAsync(tt.data(), dT, n * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    for (int c = 0; c < 3; ++c)
      mp_check(hipMemcpyAsync(tg.data() + c * n, dG + c * stride, n * sizeof(double), hipMemcpyDeviceToHost, st),
               "download");
    mp_check(hipStreamSynchronize(st), "sync");
    mp_check(hipGetLastError(), "kernel launch");
    for (int64_t i = 0; i < n; ++i) {
      T[i] = h->mat.T0 + hv[i] + tt[i];
      if (grad)
        for (int c = 0; c < 3; ++c) grad[3 * i + c] = hv[(c + 1) * n + i] + tg[c * n + i];
    }
    return SA_OK;
  });
}

int sa_mp_heat_loss(sa_multipatch *h, int32_t path, int32_t patch, int32_t face, int32_t edge_face, int32_t quad,
                    int64_t *n_pts, double *x, double *normal, double *ds, double *q_tilde, double *q_hat,
                    double *integrals) {
  return mp_guarded([&]() -> int {
    if (!h || !n_pts) throw sa::SaError{SA_EINVAL, "NULL argument"};
    const MpPath &pth = path_at(h, path);
    if (patch < 0 || patch >= (int32_t)h->P.size()) throw sa::SaError{SA_ERANGE, "patch index out of range"};
    if (face < 0 || face > 5 || edge_face < 0 || edge_face > 5 || face / 2 == edge_face / 2)
      throw sa::SaError{SA_EINVAL, "face and edge_face must be parametric faces 0..5 that meet along an edge"};
    if (quad < 1 || quad > 16) throw sa::SaError{SA_EINVAL, "quad must be 1..16"};
    const sa::PatchData &P = h->P[patch];
    const int e = 3 - face / 2 - edge_face / 2;
    const int64_t n = (int64_t)P.b[e].n_el() * quad;
    const bool per_point = x || normal || ds || q_tilde || q_hat;
    if (!per_point && !integrals) {
      *n_pts = n;
      return SA_OK;
    }
    if (per_point && *n_pts < n) {
      *n_pts = n;
      throw sa::SaError{SA_EINVAL, "point arrays shorter than the number of edge points (returned in *n_pts)"};
    }
    std::vector<double> xi, nrm, dsv;
    sa::edge_points(P, face, edge_face, quad, xi, nrm, dsv);
    const hipStream_t st = h->stream;
    TmpFree tf;
    const MpPoints pts = mp_points(h, pth, patch, n, xi.data(), tf.v);
    double *dn = mp_upload(tf.v, nrm, st), *dds = mp_upload(tf.v, dsv, st);
    double *out = mp_alloc<double>(tf.v, (size_t)4 * n + 2);
    sa::launch_heat_loss(st, n, pts.rp, pts.cl, pts.vals[1], pts.vals[2], pts.vals[3], pth.w, pts.dG, pts.stride, dn,
                         dds, h->mat.k, out, out + n, out + 2 * n, out + 3 * n, out + 4 * n);
    mp_check(hipGetLastError(), "kernel launch");
    std::vector<double> hv((size_t)4 * n + 2);
    mp_check(hipMemcpyAsync(hv.data(), out, hv.size() * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    mp_check(hipStreamSynchronize(st), "sync");
    if (x) std::copy(pts.x.begin(), pts.x.end(), x);
    if (normal) std::copy(nrm.begin(), nrm.end(), normal);
    if (ds) std::copy(dsv.begin(), dsv.end(), ds);
    if (q_tilde) std::copy(hv.begin(), hv.begin() + n, q_tilde);
    if (q_hat) std::copy(hv.begin() + n, hv.begin() + 2 * n, q_hat);
    if (integrals) {
      integrals[0] = hv[(size_t)4 * n];
      integrals[1] = hv[(size_t)4 * n + 1];
    }
    *n_pts = n;
    return SA_OK;
  });
}

void sa_mp_destroy(sa_multipatch *h) { delete h; }

}  // extern "C"
