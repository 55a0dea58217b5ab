// C ABI of the semi-analytical IGA thermal model on gfx950: object set-up,
// the per-step device pipeline (all live scan paths advance together), PCG
// drivers, evaluation, checkpoints and statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "eval_device.h"
#include "kernels.h"
#include "mlp.h"
#include "noalloc.h"
#include "sa_internal.h"
#include "solver.h"

namespace {

thread_local std::string g_last_error;

struct HipFail {
  hipError_t e;
  const char *what;
};

inline void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) throw HipFail{e, what};
}

template <class T>
T *dev_alloc(std::vector<void *> &owned, size_t n) {
  void *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw sa::SaError{SA_ENOMEM, "hipMalloc failed"};
  owned.push_back(p);
  return (T *)p;
}

template <class T>
T *dev_upload(std::vector<void *> &owned, const std::vector<T> &h, hipStream_t st) {
  T *p = dev_alloc<T>(owned, h.size());
  if (!h.empty()) hip_check(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st), "upload");
  return p;
}

struct DevCsr {
  int64_t nrow = 0;
  int64_t *rowptr = nullptr;
  int32_t *col = nullptr;
  double *val = nullptr;
  sa::CsrOp op() const { return sa::CsrOp{nrow, rowptr, col, val}; }
};

struct DevFd {
  sa::FdOp op{};
};

struct PathState {
  int64_t src0 = 0, src1 = 0;
  int32_t n_steps = 0;
  int64_t step = 0;
};

struct StageEvents {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending, pool;
};

// slots (steps x paths) of one block of the blocked source side
constexpr int kBlockSlots = 8;

}  // namespace

struct sa_iga {
  sa::Model m;
  int device = 0;
  void *scratch = nullptr;       // this device's fixed scratch area (allocation-free evaluation)
  std::vector<double> el_centre, el_xi;   // element centres (physical, parametric) for the inverse map
  hipStream_t own_stream = nullptr, stream = nullptr;   // own_stream: the device's shared solve stream
  // The source side of a step (coefficients, kernel sum, load vector,
  // Dirichlet data) runs on its own stream `ss`, one step ahead of the
  // theta-step solves on `stream`: the sum of step n+2 overlaps the solve of
  // step n+1, which it does not depend on.
  // With the exact sum (no network) the reduction of the chunk partials,
  // the load vector and the Dirichlet data of step n+1 run on a third
  // stream `ps`, beside the sum of step n+2 (two partial buffers).
  hipStream_t ss = nullptr, ps = nullptr;   // sum; reduction, loads and Dirichlet data
  bool verbose = false;                    // SA_IGA_VERBOSE: set-up and host enqueue times on stderr
  double host_us[5] = {0, 0, 0, 0, 0};     // verbose: host time of the enqueue sections of the steps
  bool overlap = false, in_step = false;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  std::vector<hipEvent_t> ev_src, ev_rhs;   // rings: one event per batch
  int64_t ev_next = 0;
  std::vector<int> path_rhs;               // per path: ev_rhs slot of its last theta right-hand side, -1 none
  std::vector<void *> owned;
  int64_t nq = 0, stride = 0, nd = 0, nDa = 1, nbox = 1;
  int S = 0;                              // number of paths
  // boundary points (centred), normals, weights, roles
  double *px = nullptr, *py = nullptr, *pz = nullptr, *pq2 = nullptr;
  float *fx = nullptr, *fy = nullptr, *fz = nullptr, *fq2 = nullptr;
  double *nx = nullptr, *ny = nullptr, *nz = nullptr, *wdS = nullptr;
  int8_t *role = nullptr;
  DevCsr load, dproj, mdir;
  int64_t *dir_dofs = nullptr;
  int64_t nD = 0;
  double *mdir_invdiag = nullptr;
  // theta-scheme operators
  sa::StencilOp Aop{};
  double *Bval = nullptr;
  uint8_t *free_mask = nullptr;
  double *A_invdiag = nullptr;
  DevFd fd_main, fd_dir;
  // sources (all paths), centred
  double *sx = nullptr, *sy = nullptr, *sz = nullptr, *sE = nullptr;
  int64_t *stick = nullptr;
  std::vector<int64_t> h_tick;
  double *c64 = nullptr;
  float *c32 = nullptr;
  // per-path state: v = u - T0 and F in double buffers selected by step parity
  double *V[2] = {nullptr, nullptr}, *Fb[2] = {nullptr, nullptr};
  double *vD = nullptr, *bD = nullptr;   // [S][nDa]
  double *Tb = nullptr, *Gb = nullptr, *LD = nullptr;  // [S][stride], [S][3 stride], [S][stride]
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;  // [S][nd]
  double *t_box = nullptr;               // [S][nbox]
  double *pD = nullptr;                  // [S][nDa]
  double *part_b2 = nullptr, *part_pq2 = nullptr, *part_rz2 = nullptr, *part_rrs = nullptr;
  int np_st = 0, np_fd = 0;
  sa::PcgScalars *sc = nullptr;          // [S]
  sa::PcgScalars *h_sc = nullptr;        // pinned [S]
  // generic (unfused) solver work vectors
  double *gr = nullptr, *gz = nullptr, *gp = nullptr, *gq = nullptr;
  double *rD = nullptr, *zD = nullptr, *pDg = nullptr, *qD = nullptr;
  double *part_b = nullptr, *part_rz = nullptr, *part_pq = nullptr, *part_rr = nullptr;
  sa::PcgScalars *sc_gen = nullptr;
  // boundary points on tensor faces: their kernel sums run as matrix
  // products; the points of the other faces go through the generic kernel
  bool use_tensor = false;
  int n_tfaces = 0;
  sa::TensorArgs tens{};
  int32_t *gen_idx = nullptr;
  int64_t n_gen = 0;
  // kernel-sum partials: two buffers used in turn, so that the sum of the
  // next batch can run while the last one is reduced
  double *partb[2] = {nullptr, nullptr};
  int64_t part_cap = 0;
  int part_next = 0;
  hipEvent_t ev_sum[2] = {nullptr, nullptr};   // the sum into partb[b] is done
  hipEvent_t ev_part[2] = {nullptr, nullptr};  // the reduction of partb[b] is done
  bool part_live[2] = {false, false};
  std::vector<PathState> paths;
  double delta = 0, shift = 0, alpha = 0, rc = 0;
  int64_t tau_ticks = 0;
  int64_t age_max = -1;                    // the tensor sum's age tables cover ages 0..age_max
  int64_t ns = 1;                        // sources per theta-step
  sa_stats stats{};
  int sticky = 0;
  StageEvents ev[SA_N_STAGES];
  // fused solver path
  sa::GatherRows grows{}, drows{};
  bool dir_fused = false, dir_exact = false;
  sa::DirArgs dargs{};
  sa::FusedPcg fd_dirp{};                // direct Kronecker solve of the projection
  bool dir_direct = false;               // ... by one workgroup per path (dense 1-D inverses in LDS)
  sa::DirDirect ddir{};
  sa::PcgScalars *sc_dir = nullptr;      // [S], never set: the direct solve always runs
  bool pcg_fused = false, fd_exact = false;
  // PCG iterations launched per theta-step when the FD solve is exact.  One
  // nearly always reaches the tolerance; the steps of a call run with one,
  // and if any step needed more, the call is run again from its start with
  // two (a device checkpoint of the state is kept for that).
  int pcg_budget = 1;
  bool force_rollback = false;           // SA_IGA_FORCE_ROLLBACK: fail the one-iteration pass (tests)
  std::vector<double *> ckpt;            // V[0], V[1], Fb[0], Fb[1], vD
  sa::FusedPcg fp{};
  double bw2 = 0.0;                      // (64 eps |A|_inf)^2, attainable-accuracy test
  bool kron = false;                     // matrix-free Kronecker A and B (affine patch)
  bool zx_ok = false;                    // x-rows short enough for the fused z pass of the checked update
  sa::KronArgs kargs{};
  // Checked update (exact FD solve on a Kronecker operator, one iteration):
  // the theta-step is u^{n+1} = x0 + P r0, and its residual b - A u^{n+1} is
  // formed by the next step's right-hand side passes (which read u^{n+1}
  // anyway), or by a check pass at the end of the call.  bprev holds each
  // path's last right-hand side, chk_pending marks the paths whose last step
  // is still to be checked (never set between calls).
  double *bprev = nullptr, *part_chk = nullptr;
  std::vector<uint8_t> chk_pending;
  // Blocked source side (one path, or a few at one step parity): the sums,
  // reductions, load vectors and Dirichlet data of K steps go through one
  // launch each, as K x paths slots, into staging buffers (two sets, one per
  // block in flight); the theta-steps of the block then read them by slot.
  // At the block's end the last step's F, Dirichlet values, T~ and grad T~
  // are copied into the paths' state.
  bool blk_ok = false;
  int blk_steps = kBlockSlots;             // steps x paths per block (<= kBlockSlots)
  int blk_groups = 0, blk_pad = 0;         // sum grid cap (0: one group per item) and LDS padding
  int n_cu = 0;                            // compute units of the device
  int sum_groups_per_cu_batch = 8;         // matrix-core sum workgroups per compute unit, launches of >= 4 paths
  double *bF[2] = {nullptr, nullptr}, *bT[2] = {nullptr, nullptr}, *bG[2] = {nullptr, nullptr};
  double *bvD[2] = {nullptr, nullptr};
  double *bLD = nullptr, *bbD = nullptr, *btmp = nullptr;
  int32_t *didx = nullptr;                 // DOF -> index of its Dirichlet value (-1: free)
  hipEvent_t ev_blk_src = nullptr, ev_blk_done[2] = {nullptr, nullptr};
  // the sum of a block starts once the theta-steps of the previous block are
  // done but blk_overlap (its last blk_overlap steps run beside the sum)
  hipEvent_t ev_blk_mid = nullptr;
  bool blk_mid_live = false;
  int blk_overlap = kBlockSlots;
  bool blk_live[2] = {false, false};
  int blk_next = 0;
  int hw0 = 1;
  sa::SolveStatus *d_status = nullptr;   // ring of per-solve records
  std::vector<int8_t> status_kind;       // 0 projection, 1 theta-step
  int64_t status_cap = 0;
  size_t lds_per_block = 65536;
  // far-history network inputs (every precision: also used for training data)
  double box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};   // control-net bounding box
  float *pf = nullptr;                  // [nq][6] normalised position, normal
  int8_t *sbin = nullptr;               // [N] 4 x 4 x 4 bin of each source
  float *bins = nullptr;                // [kMaxBatch][64]
  // surrogate form
  bool net = false;
  double net_T = 1, net_G = 1, net_E = 1;   // output and input scales
  float *nw = nullptr;                  // FP32 parameters
  sa::bf16_t *nWb[3] = {};              // layers 2..4 in bfloat16
  sa::bf16_t *nW3p = nullptr, *nW4p = nullptr;   // W3, W4 with columns permuted for the fused kernel
  bool net_fused = false;
  float *cvec = nullptr;                // [kMaxBatch][256] first-layer constants
  double *netf = nullptr;               // [kMaxBatch][4][stride] network far field
  sa::bf16_t *hA = nullptr, *hB = nullptr;  // [net_rows][256] activations
  int64_t net_rows = 0;
  // per path: 1 while its far part comes from the exact sum (no audit yet,
  // or the last audit failed), 0 while it comes from the network
  std::vector<uint8_t> use_exact;
  std::vector<int64_t> next_audit;      // per path: step of its next audit; -1 = the first step with far sources
  // audit points: a fixed seeded subset of the boundary points
  int64_t na = 0, stride_a = 0;
  double *ax = nullptr, *ay = nullptr, *az = nullptr, *aq2 = nullptr;
  float *afx = nullptr, *afy = nullptr, *afz = nullptr, *afq2 = nullptr;
  int8_t *arole = nullptr;
  float *apf = nullptr;
  double *aT = nullptr, *aG = nullptr, *aLD = nullptr, *anet = nullptr;
  // device-pointer queries: the patch geometry on the device (uploaded on
  // first use) and a workspace that grows to the largest query
  sa::GeoDev geo{};
  bool geo_ready = false;
  void *evw = nullptr;
  size_t evw_bytes = 0;
  ~sa_iga();
};

sa_iga::~sa_iga() {
  if (ss) (void)hipStreamSynchronize(ss);
  if (ps) (void)hipStreamSynchronize(ps);
  if (stream) (void)hipStreamSynchronize(stream);
  for (hipEvent_t e : ev_src) (void)hipEventDestroy(e);
  for (hipEvent_t e : ev_rhs) (void)hipEventDestroy(e);
  if (ev_start) (void)hipEventDestroy(ev_start);
  for (hipEvent_t e : ev_sum) if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : ev_part) if (e) (void)hipEventDestroy(e);
  if (ev_end) (void)hipEventDestroy(ev_end);
  if (ev_blk_src) (void)hipEventDestroy(ev_blk_src);
  if (ev_blk_mid) (void)hipEventDestroy(ev_blk_mid);
  for (hipEvent_t e : ev_blk_done) if (e) (void)hipEventDestroy(e);
  for (auto &s : ev) {
    for (auto &pr : s.pending) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto &pr : s.pool) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
  }
  for (void *p : owned) (void)hipFree(p);
  if (h_sc) (void)hipHostFree(h_sc);
  // the streams belong to the per-device set shared by all objects
}

namespace {

int set_error(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

void sa::set_last_error(const std::string &msg) { g_last_error = msg; }

namespace {

template <class F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const sa::SaError &e) {
    return set_error(e.code, e.msg);
  } catch (const HipFail &e) {
    return set_error(SA_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc &) {
    return set_error(SA_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(SA_EINVAL, "unexpected failure");
  }
}

// ---- path state accessors -------------------------------------------------------
inline double *path_v(sa_iga *h, int p) { return h->V[h->paths[p].step & 1] + (int64_t)p * h->nd; }
inline double *path_F(sa_iga *h, int p) { return h->Fb[h->paths[p].step & 1] + (int64_t)p * h->nd; }
inline double *path_vD(sa_iga *h, int p) { return h->vD + (int64_t)p * h->nDa; }
inline double *path_T(sa_iga *h, int p) { return h->Tb + (int64_t)p * h->stride; }
inline double *path_G(sa_iga *h, int p) { return h->Gb + (int64_t)p * 3 * h->stride; }

// stream of the source-side work: its own while steps run overlapped
inline hipStream_t src_stream(const sa_iga *h) { return h->in_step && h->overlap ? h->ss : h->stream; }
// stream of the theta-step solves: the object's stream, which holds the
// state u^n at the end of every call
inline hipStream_t solve_stream(const sa_iga *h) { return h->stream; }
// stream of the reduction, load vector and Dirichlet data of a step
inline hipStream_t post_stream(const sa_iga *h) {
  return h->in_step && h->overlap && !h->net ? h->ps : src_stream(h);
}

void sync_all(sa_iga *h) {
  if (h->ss) hip_check(hipStreamSynchronize(h->ss), "sync");
  if (h->ps) hip_check(hipStreamSynchronize(h->ps), "sync");
  hip_check(hipStreamSynchronize(h->stream), "sync");
}

// ---- stage timing -----------------------------------------------------------
struct StageScope {
  sa_iga *h;
  int stage;
  hipStream_t st;
  hipEvent_t stop = nullptr;
  StageScope(sa_iga *h_, int s, hipStream_t st_) : h(h_), stage(s), st(st_) {
    if (!h->m.opt.timing) return;
    auto &E = h->ev[s];
    std::pair<hipEvent_t, hipEvent_t> pr;
    if (!E.pool.empty()) {
      pr = E.pool.back();
      E.pool.pop_back();
    } else {
      hip_check(hipEventCreate(&pr.first), "event");
      hip_check(hipEventCreate(&pr.second), "event");
    }
    hip_check(hipEventRecord(pr.first, st), "event record");
    E.pending.push_back(pr);
    stop = pr.second;
  }
  ~StageScope() {
    if (stop) {
      (void)hipEventRecord(stop, st);
      h->stats.stage_launches[stage]++;
    }
  }
};

void collect_timing(sa_iga *h) {
  if (!h->m.opt.timing) return;
  for (int s = 0; s < SA_N_STAGES; ++s) {
    auto &E = h->ev[s];
    for (auto &pr : E.pending) {
      float ms = 0.f;
      hip_check(hipEventSynchronize(pr.second), "event sync");
      hip_check(hipEventElapsedTime(&ms, pr.first, pr.second), "elapsed");
      h->stats.stage_ms[s] += ms;
      E.pool.push_back(pr);
    }
    E.pending.clear();
  }
}

// ---- kernel sum --------------------------------------------------------------
// chunking of the source history (sa::plan_sum)
sa::SumPlan make_plan(const sa_iga *h, int64_t nq, int count, int64_t max_far, int64_t max_near) {
  return sa::plan_sum(h->m.opt, nq, count, max_far, max_near);
}

void ensure_part(sa_iga *h, int64_t doubles) {
  if (doubles <= h->part_cap) return;
  const int64_t cap = std::max<int64_t>(doubles, 2 * h->part_cap);
  sync_all(h);
  for (double *&b : h->partb) {
    if (!b) continue;
    hip_check(hipFree(b), "free");
    h->owned.erase(std::find(h->owned.begin(), h->owned.end(), (void *)b));
    b = nullptr;
  }
  for (double *&b : h->partb) b = dev_alloc<double>(h->owned, (size_t)cap);
  h->part_cap = cap;
  h->part_live[0] = h->part_live[1] = false;
}

// slot s of `tab` <- path p at the end of step `step`: its switched-on and
// far-field source counts
void fill_slot(const sa_iga *h, sa::PathTab &tab, int s, int p, int64_t step) {
  const PathState &P = h->paths[p];
  const int64_t now = step * h->ns;
  auto b = h->h_tick.begin() + P.src0, e = h->h_tick.begin() + P.src1;
  const int64_t a = (int64_t)(std::upper_bound(b, e, now) - b);
  int64_t f = 0;
  if (h->m.opt.precision != SA_PREC_FP64 && a > 0) {
    const int64_t thr = now - h->tau_ticks;  // far iff tick < thr
    f = std::min<int64_t>(a, (int64_t)(std::lower_bound(b, b + a, thr) - b));
  }
  tab.path[s] = p;
  tab.src0[s] = P.src0;
  tab.now[s] = now;
  tab.n_act[s] = (int32_t)a;
  tab.n_far[s] = (int32_t)f;
  tab.mode[s] = 0;
}

// T~ and grad T~ of the slots of `tab` (each at its own time) at nq points
// (centred arrays); outputs indexed by path (boundary tables) or by slot
// (query points)
// slots of `tab` ordered by decreasing far (then switched-on) history: the
// sum's work items go slot by slot to the workgroups in launch order, so the
// longest run first and the short ones fill the end of the launch
sa::PathTab longest_first(const sa::PathTab &tab) {
  int ord[sa::kMaxBatch];
  for (int s = 0; s < tab.count; ++s) ord[s] = s;
  std::stable_sort(ord, ord + tab.count, [&](int a, int b) {
    return tab.n_far[a] != tab.n_far[b] ? tab.n_far[a] > tab.n_far[b] : tab.n_act[a] > tab.n_act[b];
  });
  sa::PathTab t = tab;
  for (int s = 0; s < tab.count; ++s) {
    const int o = ord[s];
    t.path[s] = tab.path[o];
    t.src0[s] = tab.src0[o];
    t.n_act[s] = tab.n_act[o];
    t.n_far[s] = tab.n_far[o];
    t.now[s] = tab.now[o];
    t.mode[s] = tab.mode[o];
  }
  return t;
}

void sum_points(sa_iga *h, const sa::PathTab &tab_in, int64_t nq, int64_t stride, const double *px,
                const double *py, const double *pz, const double *pq2, const float *fx, const float *fy,
                const float *fz, const float *fq2, const int8_t *role, const double *nx, const double *ny,
                const double *nz, const double *wdS, bool by_slot, int64_t ostride, double *T, double *G,
                double *ld, const double *net = nullptr, int64_t net_stride = 0, hipStream_t post = nullptr,
                bool boundary = false, int plan_count = 0) {
  // outputs indexed by path (not slot) and no network output indexed by
  // slot: the slots may be taken in any order, with the same results
  const bool reorder = !by_slot && !net && tab_in.count > 1 && !std::getenv("SA_IGA_SLOT_ORDER_AS_GIVEN");
  const sa::PathTab tab = reorder ? longest_first(tab_in) : tab_in;
  int64_t max_act = 0, max_far = 0, max_near = 0;
  for (int s = 0; s < tab.count; ++s) {
    const int64_t nf = tab.mode[s] ? 0 : tab.n_far[s];      // far sources summed here
    max_act = std::max<int64_t>(max_act, tab.n_act[s]);
    max_far = std::max<int64_t>(max_far, nf);
    max_near = std::max<int64_t>(max_near, tab.n_act[s] - tab.n_far[s]);
    h->stats.pairs += (int64_t)(tab.n_act[s] - tab.n_far[s] + nf) * nq;
    h->stats.pairs_near += (int64_t)(tab.n_act[s] - tab.n_far[s]) * nq;
    if (tab.mode[s]) h->stats.pairs_net += (int64_t)tab.n_far[s] * nq;
  }
  const hipStream_t st = src_stream(h);
  // the tensor sum takes its coefficients from the age tables when it is the
  // only sum of this call and they cover every slot's time
  bool tables = boundary && h->use_tensor && h->n_gen == 0;
  for (int s = 0; s < tab.count && tables; ++s) tables = tab.now[s] <= h->age_max;
  if (max_act > 0 && !tables) {
    StageScope s(h, SA_STAGE_COEFF, st);
    sa::CoeffParams cp{h->delta, h->shift, h->alpha, h->rc, h->m.opt.kernel_scale};
    sa::launch_coeff(st, tab, max_act, h->stick, h->sx, h->sy, h->sz, h->sE, cp, h->c64, h->c32);
  }
  // the chunking follows plan_count paths (the slots of a blocked call cut
  // their histories as one-step calls do)
  sa::SumPlan pl = make_plan(h, nq, plan_count > 0 ? plan_count : tab.count, max_far, max_near);
  pl.part_stride = stride;
  const int nch = pl.n_chunks_far + pl.n_chunks_near;
  ensure_part(h, (int64_t)tab.count * std::max(nch, 1) * 5 * stride);
  // the partials go to the buffer whose last reduction is longest done
  const int b = h->part_next;
  h->part_next ^= 1;
  double *part = h->partb[b];
  const hipStream_t fs = post ? post : st;
  if (h->part_live[b]) hip_check(hipStreamWaitEvent(st, h->ev_part[b], 0), "stream wait");
  if (nch > 0) {
    StageScope s(h, SA_STAGE_SUM, st);
    if (boundary && h->use_tensor) {
      sa::TensorArgs ta = h->tens;
      ta.c64 = h->c64;
      if (!tables) ta.age_c = nullptr;
      if (plan_count > 0 && plan_count < 4) {   // a blocked call of one to three paths
        ta.max_groups = ta.max_groups_batch = h->blk_groups;
        ta.lds_pad = h->blk_pad;
      }
      ta.part = part;
      ta.stride = stride;
      sa::launch_sum_tensor(st, pl, tab, ta);
      if (h->n_gen > 0) {
        sa::SumPlan pg = pl;
        pg.nq = h->n_gen;
        sa::launch_sum(st, pg, tab, px, py, pz, pq2, fx, fy, fz, fq2, h->c64, h->c32, part, h->gen_idx);
      }
    } else {
      sa::launch_sum(st, pl, tab, px, py, pz, pq2, fx, fy, fz, fq2, h->c64, h->c32, part);
    }
  }
  if (fs != st) {
    hip_check(hipEventRecord(h->ev_sum[b], st), "event record");
    hip_check(hipStreamWaitEvent(fs, h->ev_sum[b], 0), "stream wait");
  }
  {
    StageScope s(h, SA_STAGE_REDUCE, fs);
    sa::launch_finalize(fs, tab, by_slot, nq, nch, stride, part, px, py, pz, nx, ny, nz, wdS, role,
                        h->m.mat.k, ostride, T, G, ld, net, net_stride);
  }
  hip_check(hipEventRecord(h->ev_part[b], fs), "event record");
  h->part_live[b] = true;
}

// ---- generic PCG driver (single path; Jacobi or oversize problems) ---------------
struct PcgSpec {
  int64_t n = 0;
  bool stencil = true;
  sa::StencilOp st{};
  sa::CsrOp csr{};
  bool fd = false;
  sa::FdOp fdop{};
  const double *invdiag = nullptr;
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  int n_part_b = 0;
};

int apply_precond(sa_iga *h, PcgSpec &s, const double *r, double *z, sa::PcgScalars *sc) {
  if (s.fd) {
    sa::launch_fd(h->stream, s.fdop, s.n, r, z, h->part_rz, sc);
    return sa::parts_for((int64_t)s.fdop.m[0] * s.fdop.m[1] * s.fdop.m[2]);
  }
  sa::launch_jacobi(h->stream, s.n, s.invdiag, r, z, h->part_rz, sc);
  return sa::parts_for(s.n);
}

// Solve on the prepared residual r = b - A x (partials of |b|^2 in part_b).
int pcg_run(sa_iga *h, PcgSpec &s, double *relres) {
  const int64_t n = s.n;
  const int np = sa::parts_for(n);
  int np_rz = apply_precond(h, s, s.r, s.z, nullptr);
  sa::launch_pcg_start(h->stream, n, s.n_part_b, h->part_b, np_rz, h->part_rz, s.z, s.p, h->sc_gen,
                       h->m.opt.pcg_rtol);
  int chunk = s.fd ? 2 : 8;
  for (;;) {
    for (int k = 0; k < chunk; ++k) {
      if (s.stencil) sa::launch_stencil_apply_dot(h->stream, s.st, s.p, s.q, h->part_pq, h->sc_gen);
      else sa::launch_csr_apply_dot(h->stream, s.csr, s.p, s.q, h->part_pq, h->sc_gen);
      sa::launch_pcg_update(h->stream, n, np, h->part_pq, np_rz, h->part_rz, s.p, s.q, s.x, s.r, h->part_rr,
                            h->sc_gen);
      np_rz = apply_precond(h, s, s.r, s.z, h->sc_gen);
      sa::launch_pcg_direction(h->stream, n, np, np_rz, h->part_rr, h->part_rz, s.z, s.p, h->sc_gen);
    }
    hip_check(hipMemcpyAsync(h->h_sc, h->sc_gen, sizeof(sa::PcgScalars), hipMemcpyDeviceToHost, h->stream),
              "status copy");
    hip_check(hipStreamSynchronize(h->stream), "sync");
    const sa::PcgScalars st = *h->h_sc;
    if (st.done == 1) {
      *relres = st.bnorm2 > 0 ? std::sqrt(std::max(st.rr, 0.0) / st.bnorm2) : 0.0;
      return st.iter;
    }
    if (st.done == 2) throw sa::SaError{SA_ENOCONV, "PCG breakdown (operator not positive definite)"};
    if (!std::isfinite(st.rz) || !std::isfinite(st.rr)) throw sa::SaError{SA_ENOCONV, "PCG produced NaN/Inf"};
    if (st.iter >= h->m.opt.pcg_max_iter)
      throw sa::SaError{SA_ENOCONV, "PCG did not converge within pcg_max_iter"};
    chunk = std::min(chunk * 2, 64);
    chunk = std::min(chunk, std::max(1, h->m.opt.pcg_max_iter - st.iter));
  }
}

// ---- device solve records ----------------------------------------------------
// a theta-step that one PCG iteration did not bring to the tolerance (the
// call is then run again with two)
struct BudgetExceeded {};

void check_statuses(sa_iga *h) {
  const size_t used = h->status_kind.size();
  if (used == 0) return;
  if (h->ps) hip_check(hipStreamSynchronize(h->ps), "sync");   // records of the projection solves
  std::vector<sa::SolveStatus> st(used);
  hip_check(hipMemcpyAsync(st.data(), h->d_status, used * sizeof(sa::SolveStatus), hipMemcpyDeviceToHost,
                           h->stream),
            "status copy");
  hip_check(hipStreamSynchronize(h->stream), "sync");
  std::vector<int8_t> kind;
  kind.swap(h->status_kind);
  int bad = -1;
  for (size_t i = 0; i < used; ++i) {
    if (st[i].done != 1 && bad < 0) bad = (int)i;
    if (st[i].iter < 0) continue;          // a checked update with no previous step to check
    if (kind[i] == 0) {
      h->stats.dirichlet_iterations += st[i].iter;
    } else {
      h->stats.pcg_iterations += st[i].iter;
      h->stats.pcg_last_iterations = st[i].iter;
      h->stats.pcg_last_relres = std::sqrt(std::max(st[i].relres2, 0.0));
    }
  }
  if (bad >= 0 && kind[bad] == 1 && st[bad].done == 0 && h->fd_exact && h->pcg_budget == 1)
    throw BudgetExceeded{};
  if (bad >= 0) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "a solve did not converge within its iteration budget (record %d, %s, done %d, |r|/|b| = %.3e)",
                  bad, kind[bad] ? "theta-step" : "projection", st[bad].done,
                  std::sqrt(std::max(st[bad].relres2, 0.0)));
    throw sa::SaError{SA_ENOCONV, msg};
  }
}

// reserve n consecutive records of the given kind
sa::SolveStatus *next_status(sa_iga *h, int n, int8_t kind) {
  if ((int64_t)h->status_kind.size() + n > h->status_cap) check_statuses(h);
  sa::SolveStatus *s = h->d_status + h->status_kind.size();
  for (int i = 0; i < n; ++i) h->status_kind.push_back(kind);
  return s;
}

// ---- far-history network ------------------------------------------------------------
// network far field of the first `tab.count` slots at nq points (point inputs
// pf [nq][6]) into out[(s*4 + c) * ostride + q]; rows go through the layers
// in chunks of net_rows so the activations stay cache-sized
void run_network(sa_iga *h, const sa::PathTab &tab, int64_t nq, const float *pf, int64_t ostride, double *out) {
  if (tab.count <= 0 || nq <= 0) return;
  const hipStream_t st = src_stream(h);
  StageScope sc(h, SA_STAGE_NET, st);
  const float *W1 = h->nw + sa::MlpLayout::W1, *b1 = h->nw + sa::MlpLayout::b1;
  sa::launch_far_bins(st, tab, h->sbin, h->sE, h->net_E, h->bins);
  sa::launch_layer1_const(st, tab.count, h->bins, W1, b1, h->cvec);
  const int64_t total = (int64_t)tab.count * nq, H = sa::kMlpHid;
  if (h->net_fused) {
    sa::NetArgs na{};
    na.r0 = 0;
    na.rows = total;
    na.nq = nq;
    na.pf = pf;
    na.c = h->cvec;
    na.W1 = W1;
    na.W2 = h->nWb[0];
    na.W3p = h->nW3p;
    na.W4p = h->nW4p;
    na.b2 = h->nw + sa::MlpLayout::b2;
    na.b3 = h->nw + sa::MlpLayout::b3;
    na.b4 = h->nw + sa::MlpLayout::b4;
    na.W5 = h->nw + sa::MlpLayout::W5;
    na.b5 = h->nw + sa::MlpLayout::b5;
    na.ts = h->net_T;
    na.gs = h->net_G;
    na.ostride = ostride;
    na.net = out;
    sa::launch_net_fused(st, na);
    return;
  }
  const int64_t bias[3] = {sa::MlpLayout::b2, sa::MlpLayout::b3, sa::MlpLayout::b4};
  for (int64_t r0 = 0; r0 < total; r0 += h->net_rows) {
    const int64_t rows = std::min(h->net_rows, total - r0);
    sa::launch_layer1_points(st, r0, rows, nq, pf, h->cvec, W1, h->hA);
    sa::bf16_t *in = h->hA, *outb = h->hB;
    for (int l = 0; l < 3; ++l) {
      sa::GemmArgs g{};
      g.M = rows;
      g.N = H;
      g.K = H;
      g.A = in;
      g.a_sm = H;
      g.a_sk = 1;
      g.B = h->nWb[l];
      g.b_sk = 1;
      g.b_sn = H;
      g.bias = h->nw + bias[l];
      g.act = 1;
      g.out = outb;
      g.ldo = H;
      sa::launch_gemm_bf16(st, g);
      std::swap(in, outb);
    }
    sa::launch_layer_out_field(st, r0, rows, nq, in, h->nw + sa::MlpLayout::W5, h->nw + sa::MlpLayout::b5,
                               h->net_T, h->net_G, ostride, out);
  }
}

// Audit of the slots `aud` of `tab` (their steps' far parts): the exact FP64
// far sum and the network at the audit points; a path whose largest error of
// the far temperature exceeds audit_tol uses the exact far sum until an audit
// passes again.
void audit_slots(sa_iga *h, const sa::PathTab &tab, const std::vector<int> &aud) {
  if (aud.empty()) return;
  sa::PathTab ex{}, nt{};
  ex.count = nt.count = (int)aud.size();
  for (int i = 0; i < ex.count; ++i) {
    const int s = aud[i];
    ex.path[i] = nt.path[i] = tab.path[s];
    ex.src0[i] = nt.src0[i] = tab.src0[s];
    ex.now[i] = nt.now[i] = tab.now[s];
    ex.n_act[i] = tab.n_far[s];       // the far sources only, all in FP64
    ex.n_far[i] = 0;
    ex.mode[i] = 0;
    nt.n_act[i] = tab.n_act[s];
    nt.n_far[i] = tab.n_far[s];
    nt.mode[i] = 1;
  }
  const hipStream_t st = src_stream(h);
  const sa_stats keep = h->stats;
  sum_points(h, ex, h->na, h->stride_a, h->ax, h->ay, h->az, h->aq2, h->afx, h->afy, h->afz, h->afq2, h->arole,
             h->ax, h->ay, h->az, h->ax, true, h->stride_a, h->aT, h->aG, h->aLD);
  h->stats.pairs = keep.pairs;              // audit work is not part of the step's sum
  h->stats.pairs_near = keep.pairs_near;
  h->stats.pairs_net = keep.pairs_net;
  run_network(h, nt, h->na, h->apf, h->stride_a, h->anet);
  const int64_t n = h->na, sa_ = h->stride_a;
  std::vector<double> te((size_t)ex.count * sa_), tn((size_t)ex.count * 4 * sa_);
  hip_check(hipMemcpyAsync(te.data(), h->aT, te.size() * sizeof(double), hipMemcpyDeviceToHost, st),
            "download");
  hip_check(hipMemcpyAsync(tn.data(), h->anet, tn.size() * sizeof(double), hipMemcpyDeviceToHost, st),
            "download");
  hip_check(hipStreamSynchronize(st), "sync");
  for (int i = 0; i < ex.count; ++i) {
    double err = 0.0;
    for (int64_t q = 0; q < n; ++q)
      err = std::max(err, std::fabs(tn[(size_t)i * 4 * sa_ + q] - te[(size_t)i * sa_ + q]));
    if (!std::isfinite(err)) err = INFINITY;
    const bool fail = !(err <= h->m.opt.audit_tol);
    h->use_exact[ex.path[i]] = fail ? 1 : 0;
    h->stats.audits++;
    if (fail) h->stats.audit_failures++;
    h->stats.audit_max_err = std::max(h->stats.audit_max_err, err);
  }
}

// ---- one theta-step of a set of paths (at most kMaxBatch) -------------------------
// The paths may sit at different steps; their steps share one parity, which
// selects the state buffers (u^n, F^n read from one, u^{n+1}, F^{n+1} written
// to the other).
// verbose: host time between marks, added to h->host_us[section]
struct HostLap {
  sa_iga *h;
  std::chrono::steady_clock::time_point t;
  explicit HostLap(sa_iga *h_) : h(h_) {
    if (h->verbose) t = std::chrono::steady_clock::now();
  }
  void mark(int section) {
    if (!h->verbose) return;
    const auto n = std::chrono::steady_clock::now();
    h->host_us[section] += std::chrono::duration<double, std::micro>(n - t).count();
    t = n;
  }
};

void step_batch(sa_iga *h, std::vector<int> pids) {
  HostLap lap(h);
  const int count = (int)pids.size();
  const int cur = (int)(h->paths[pids[0]].step & 1), nxt = cur ^ 1;
  const int64_t nd = h->nd;
  sa::PathTab tab{};
  sa::SlotMap sm{};
  tab.count = sm.count = count;
  int n_net = 0;
  if (h->net) {
    // audits due at this step decide the far part of this step already
    sa::PathTab at{};
    at.count = count;
    std::vector<int> aud;
    for (int s = 0; s < count; ++s) {
      const int p = pids[s];
      const int64_t st1 = h->paths[p].step + 1;
      fill_slot(h, at, s, p, st1);
      // the first step with far sources, then every audit_every steps
      if (at.n_far[s] > 0 && (h->next_audit[p] < 0 || st1 >= h->next_audit[p])) {
        aud.push_back(s);
        h->next_audit[p] = st1 + h->m.opt.audit_every;
      }
    }
    audit_slots(h, at, aud);
    // paths on the network first: their slots index the network's output
    std::stable_partition(pids.begin(), pids.end(), [h](int p) { return !h->use_exact[p]; });
    for (int p : pids) n_net += h->use_exact[p] ? 0 : 1;
  }
  for (int s = 0; s < count; ++s) {
    const PathState &P = h->paths[pids[s]];
    if ((int)(P.step & 1) != cur) throw sa::SaError{SA_EINVAL, "internal: mixed step parity in a batch"};
    sm.path[s] = pids[s];
    fill_slot(h, tab, s, pids[s], P.step + 1);
    if (h->net) {
      // the other paths sum their far history as the precision form does
      // (FP32 terms in FP64 block sums)
      if (s < n_net) tab.mode[s] = 1;
    }
  }
  const double *net = nullptr;
  if (n_net > 0) {
    sa::PathTab nt = tab;
    nt.count = n_net;
    run_network(h, nt, h->nq, h->pf, h->stride, h->netf);
    net = h->netf;
    h->stats.net_steps += n_net;
  }
  // T~, grad T~ and load densities at every boundary point (Eqs. 7-8, 10-11)
  lap.mark(0);
  const hipStream_t as = post_stream(h);
  sum_points(h, tab, h->nq, h->stride, h->px, h->py, h->pz, h->pq2, h->fx, h->fy, h->fz, h->fq2, h->role,
             h->nx, h->ny, h->nz, h->wdS, false, h->stride, h->Tb, h->Gb, h->LD, net, h->stride, as, true);
  double *Vc = h->V[cur], *Vn = h->V[nxt], *Fc = h->Fb[cur], *Fn = h->Fb[nxt];
  lap.mark(1);
  if (h->overlap) {
    // F^{n+1} and the Dirichlet values of u^{n+1} overwrite F^{n-1} and
    // entries of u^{n-1}: wait until the right-hand side of step n of these
    // paths has read them
    int last = -1;
    for (int s = 0; s < count; ++s) last = std::max(last, h->path_rhs[pids[s]]);
    for (int s = 0; s < count; ++s) {
      const int e = h->path_rhs[pids[s]];
      if (e >= 0 && e != last) hip_check(hipStreamWaitEvent(as, h->ev_rhs[e], 0), "stream wait");
    }
    if (last >= 0) hip_check(hipStreamWaitEvent(as, h->ev_rhs[last], 0), "stream wait");
  }
  const bool dir_rhs = h->nD > 0 && (h->dir_exact || h->dir_fused);
  {
    StageScope s(h, SA_STAGE_LOAD, as);
    // F^{n+1} on the non-empty rows (Eq. 18), with the right-hand side of the
    // projection (Eq. 11) in the same launch
    if (dir_rhs)
      sa::launch_gather_rows2(as, sm, h->grows, Fn, nd, h->drows, h->bD, h->nDa, h->LD, h->stride);
    else
      sa::launch_gather_rows(as, sm, h->grows, h->LD, h->stride, Fn, nd, 0, nullptr, nullptr);
  }
  // Dirichlet values (Eq. 11), scattered into the Dirichlet DOFs of u^{n+1}
  if (h->nD > 0) {
    StageScope s(h, SA_STAGE_DIRICHLET, as);
    if (h->dir_direct) {
      sa::DirDirect a = h->ddir;
      a.xfull = Vn;
      sa::launch_dir_direct(as, sm, a);
    } else if (h->dir_exact) {
      sa::FusedPcg f = h->fd_dirp;
      f.scatter_out = Vn;
      sa::launch_fd_pass(as, sm, f, 0, false, false);
    } else if (h->dir_fused) {
      sa::DirArgs a = h->dargs;
      a.b = h->bD;
      a.vD = h->vD;
      a.xfull = Vn;
      a.xs = nd;
      a.status = next_status(h, count, 0);
      sa::launch_dirichlet(as, sm, a);
    } else {
      // generic projection solve (never overlapped: as is the main stream)
      for (int s = 0; s < count; ++s) {
        const int p = pids[s];
        sa::launch_gather(h->stream, h->dproj.nrow, h->dproj.rowptr, h->dproj.col, h->dproj.val,
                          h->LD + (int64_t)p * h->stride, h->bD + (int64_t)p * h->nDa);
        PcgSpec d;
        d.n = h->nD;
        d.stencil = false;
        d.csr = h->mdir.op();
        d.fd = h->m.opt.preconditioner == SA_PRECOND_FD && h->m.fd_dir_ok;
        d.fdop = h->fd_dir.op;
        d.invdiag = h->mdir_invdiag;
        d.x = path_vD(h, p);
        d.r = h->rD;
        d.z = h->zD;
        d.p = h->pDg;
        d.q = h->qD;
        d.n_part_b = sa::parts_for(h->nD);
        sa::launch_csr_init(h->stream, d.csr, h->bD + (int64_t)p * h->nDa, d.x, h->rD, h->part_b);
        double rr = 0;
        h->stats.dirichlet_iterations += pcg_run(h, d, &rr);
        sa::launch_scatter_dirichlet(h->stream, h->nD, h->dir_dofs, d.x, Vn + (int64_t)p * nd);
      }
    }
  }
  // the theta-step of these paths: on the solver stream
  lap.mark(2);
  const hipStream_t bsx = solve_stream(h);
  if (h->overlap) {
    const hipEvent_t e = h->ev_src[h->ev_next % (int64_t)h->ev_src.size()];
    hip_check(hipEventRecord(e, as), "event record");
    hip_check(hipStreamWaitEvent(bsx, e, 0), "stream wait");
  }
  // first iterate: u^n on the free DOFs (in the first pass of the
  // right-hand side on affine patches)
  if (!(h->pcg_fused && h->kron)) sa::launch_copy_free(bsx, sm, nd, h->free_mask, Vc, Vn);
  // theta-scheme (Eq. 20)
  const int ev_slot = (int)(h->ev_next % (int64_t)std::max<size_t>(h->ev_rhs.size(), 1));
  h->ev_next++;
  auto rhs_done = [&]() {
    if (!h->overlap) return;
    hip_check(hipEventRecord(h->ev_rhs[ev_slot], bsx), "event record");
    for (int s = 0; s < count; ++s) h->path_rhs[pids[s]] = ev_slot;
  };
  const bool checked = h->pcg_fused && h->kron && h->fd_exact && h->pcg_budget == 1 && h->zx_ok;
  if (h->pcg_fused) {
    {
      StageScope s(h, SA_STAGE_RHS, bsx);
      sa::SlArgs a{};
      a.nrow = nd;
      a.vs = nd;
      a.np = h->np_st;
      a.n0 = h->Aop.n[0];
      a.n1 = h->Aop.n[1];
      a.hw1 = h->Aop.hw[1];
      a.hw2 = h->Aop.hw[2];
      a.A = h->Aop.A;
      a.B = h->Bval;
      a.mask = h->free_mask;
      a.x = Vn;
      a.v = Vc;
      a.F1 = Fn;
      a.F0 = Fc;
      a.theta = h->m.opt.theta;
      a.out = h->r;
      a.part = h->part_b2;
      a.sc_w = h->sc;
      if (h->kron) {
        sa::KronArgs k = h->kargs;
        k.x = Vn;
        k.v = Vc;
        k.F1 = Fn;
        k.F0 = Fc;
        k.out = h->r;
        k.part = h->part_b2;
        k.sc = nullptr;
        k.sc_w = h->sc;
        k.init_x = 1;
        k.x_init = Vn;
        if (checked) {
          k.check = 1;
          sa::launch_theta_checked_rhs(bsx, sm, k, h->fp);
        } else {
          sa::launch_kron(bsx, sm, k, true);
        }
      } else {
        sa::launch_stencil_sl(bsx, sm, a, h->hw0, true);
      }
    }
    rhs_done();
    lap.mark(3);
    StageScope s(h, SA_STAGE_PCG, bsx);
    sa::FusedPcg f = h->fp;
    f.x = Vn;
    f.status = next_status(h, count, 1);
    sa::SlArgs ap{};
    ap.nrow = nd;
    ap.vs = nd;
    ap.np = h->np_st;
    ap.n0 = h->Aop.n[0];
    ap.n1 = h->Aop.n[1];
    ap.hw1 = h->Aop.hw[1];
    ap.hw2 = h->Aop.hw[2];
    ap.A = h->Aop.A;
    ap.mask = h->free_mask;
    ap.x = h->p;
    ap.out = h->q;
    ap.part = h->part_pq2;
    ap.sc = h->sc;
    sa::KronArgs kp = h->kargs;
    kp.x = h->p;
    kp.out = h->q;
    kp.part = h->part_pq2;
    kp.sc = h->sc;
    kp.sc_w = nullptr;
    auto apply = [&]() {
      if (h->kron) sa::launch_kron(bsx, sm, kp, false);
      else sa::launch_stencil_sl(bsx, sm, ap, h->hw0, false);
    };
    if (checked) {
      // x += P r; the first plane block also writes the record of the
      // previous step's residual check of each path that has one pending
      f.update_x = 1;
      f.check_mask = 0;
      for (int s = 0; s < count; ++s)
        if (h->chk_pending[pids[s]]) f.check_mask |= 1ull << s;
      f.part_chk = h->part_chk;
      f.np_chk = sa::zx_blocks(h->kargs.op);
      f.chk_rtol2 = h->force_rollback ? 0.0 : f.rtol2;   // forced: every check fails
      f.chk_bw2 = h->force_rollback ? 0.0 : f.bw2;
      sa::launch_theta_checked_solve(bsx, sm, f);
      for (int s = 0; s < count; ++s) h->chk_pending[pids[s]] = 1;
    } else {
      sa::launch_fd_pass(bsx, sm, f, 0, true, false);
      if (h->fd_exact && h->pcg_budget == 1 && h->force_rollback) {
        f.rtol2 = 0.0;   // no residual passes: the one-iteration pass fails
        f.bw2 = 0.0;
      }
      if (h->fd_exact) {
        // with the exact preconditioner the first iteration nearly always
        // converges: test |r| right after the update, and run the FD solve and
        // the new direction only for paths still going (the others exit at once)
        for (int k = 0; k < h->pcg_budget; ++k) {
          apply();
          sa::launch_pcg_last_update(bsx, sm, f, k);
          sa::launch_pcg_dir(bsx, sm, f, k, true);
          if (k + 1 < h->pcg_budget) {
            sa::launch_fd_pass(bsx, sm, f, k, false, false);
            sa::launch_pcg_dir(bsx, sm, f, k, false);
          }
        }
      } else {
        int k = 0, chunk = 4;
        for (;;) {
          for (int c = 0; c < chunk; ++c, ++k) {
            apply();
            sa::launch_fd_pass(bsx, sm, f, k, false, true);
            sa::launch_pcg_dir(bsx, sm, f, k, false);
          }
          hip_check(hipMemcpyAsync(h->h_sc, h->sc, h->S * sizeof(sa::PcgScalars), hipMemcpyDeviceToHost, bsx),
                    "status copy");
          hip_check(hipStreamSynchronize(bsx), "sync");
          bool all = true;
          for (int s = 0; s < count; ++s) {
            const sa::PcgScalars &st = h->h_sc[pids[s]];
            if (st.done == 2) throw sa::SaError{SA_ENOCONV, "PCG breakdown (operator not positive definite)"};
            if (st.done != 1) all = false;
          }
          if (all) break;
          if (k >= h->m.opt.pcg_max_iter) throw sa::SaError{SA_ENOCONV, "PCG did not converge within pcg_max_iter"};
          chunk = std::min(chunk * 2, 32);
        }
      }
    }
  } else {
    for (int s = 0; s < count; ++s) {
      const int p = pids[s];
      double *x = Vn + (int64_t)p * nd;
      {
        StageScope sc(h, SA_STAGE_RHS, h->stream);
        sa::launch_theta_init(h->stream, h->Aop, h->Bval, Vc + (int64_t)p * nd, Fn + (int64_t)p * nd,
                              Fc + (int64_t)p * nd, h->m.opt.theta, x, h->gr, h->part_b);
      }
      StageScope sc(h, SA_STAGE_PCG, h->stream);
      PcgSpec m;
      m.n = nd;
      m.stencil = true;
      m.st = h->Aop;
      m.fd = h->m.opt.preconditioner == SA_PRECOND_FD;
      m.fdop = h->fd_main.op;
      m.invdiag = h->A_invdiag;
      m.x = x;
      m.r = h->gr;
      m.z = h->gz;
      m.p = h->gp;
      m.q = h->gq;
      m.n_part_b = sa::parts_for(m.n);
      double rr = 0;
      const int it = pcg_run(h, m, &rr);
      h->stats.pcg_iterations += it;
      h->stats.pcg_last_iterations = it;
      h->stats.pcg_last_relres = rr;
    }
  }
  hip_check(hipGetLastError(), "kernel launch");
  for (int s = 0; s < count; ++s) h->paths[pids[s]].step++;
  h->stats.steps += count;
  lap.mark(4);
}

// K steps of the paths `pids` (one step parity, none finishing inside the
// block) with the source side once for the block (the blocked-source-side
// members of sa_iga): slot k L + l of the source launches is step k of path
// pids[l].  Same results, bit for bit, as K one-step calls.
void step_block(sa_iga *h, const std::vector<int> &pids, int K) {
  HostLap lap(h);
  const int L = (int)pids.size(), KL = K * L;
  if (L <= 0 || K <= 0 || KL > kBlockSlots) throw sa::SaError{SA_EINVAL, "internal: block size"};
  const int64_t nd = h->nd, st = h->stride, nDa = h->nDa;
  const int sb = h->blk_next;
  h->blk_next ^= 1;
  sa::PathTab tab{};
  tab.count = KL;
  for (int k = 0; k < K; ++k)
    for (int l = 0; l < L; ++l) {
      const PathState &P = h->paths[pids[l]];
      if ((P.step & 1) != (h->paths[pids[0]].step & 1) || P.step + K > P.n_steps)
        throw sa::SaError{SA_EINVAL, "internal: paths of a block"};
      fill_slot(h, tab, k * L + l, pids[l], P.step + 1 + k);
      if (tab.now[k * L + l] > h->age_max) throw sa::SaError{SA_EINVAL, "internal: block beyond the age tables"};
    }
  sa::SlotMap si{};   // slot s -> staging entry s
  si.count = KL;
  for (int s = 0; s < KL; ++s) si.path[s] = s;
  const hipStream_t as = post_stream(h);
  // staging set sb is free once the theta-steps of the block that used it last are done
  if (h->blk_live[sb]) hip_check(hipStreamWaitEvent(as, h->ev_blk_done[sb], 0), "stream wait");
  if (h->blk_mid_live) hip_check(hipStreamWaitEvent(src_stream(h), h->ev_blk_mid, 0), "stream wait");
  h->blk_mid_live = false;
  lap.mark(0);
  // T~, grad T~ and load densities of every step of the block (Eqs. 7-8, 10-11)
  sum_points(h, tab, h->nq, st, h->px, h->py, h->pz, h->pq2, h->fx, h->fy, h->fz, h->fq2, h->role, h->nx, h->ny,
             h->nz, h->wdS, true, st, h->bT[sb], h->bG[sb], h->bLD, nullptr, 0, as, true, L);
  lap.mark(1);
  {
    // F^{n+1..n+K} (Eq. 18) and the projection right-hand sides (Eq. 11)
    StageScope s(h, SA_STAGE_LOAD, as);
    if (h->nD > 0)
      sa::launch_gather_rows2(as, si, h->grows, h->bF[sb], nd, h->drows, h->bbD, nDa, h->bLD, st);
    else
      sa::launch_gather_rows(as, si, h->grows, h->bLD, st, h->bF[sb], nd, 0, nullptr, nullptr);
  }
  if (h->nD > 0) {
    StageScope s(h, SA_STAGE_DIRICHLET, as);
    sa::DirDirect a = h->ddir;
    a.b = h->bbD;
    a.vD = h->bvD[sb];
    a.vs = nDa;
    a.xfull = nullptr;   // scattered into u^{n+1} by its theta-step
    a.tmp = h->ddir.tmp ? h->btmp : nullptr;
    sa::launch_dir_direct(as, si, a);
  }
  const hipStream_t bsx = solve_stream(h);
  hip_check(hipEventRecord(h->ev_blk_src, as), "event record");
  hip_check(hipStreamWaitEvent(bsx, h->ev_blk_src, 0), "stream wait");
  lap.mark(2);
  sa::SlotMap sm{};
  sm.count = L;
  for (int l = 0; l < L; ++l) sm.path[l] = pids[l];
  const int par0 = (int)(h->paths[pids[0]].step & 1);
  // theta arguments of step k of the block (u^{n+k} in V[(n+k) & 1])
  auto step_args = [&](int k) {
    const int cur = (par0 + k) & 1, nxt = cur ^ 1;
    sa::KronArgs ka = h->kargs;
    ka.x = h->V[nxt];
    ka.v = h->V[cur];
    ka.F1 = h->bF[sb] + (int64_t)k * L * nd;
    ka.f1_slot = 1;
    ka.f1s = nd;
    if (k == 0) {
      ka.F0 = h->Fb[cur];
    } else {
      ka.F0 = h->bF[sb] + (int64_t)(k - 1) * L * nd;
      ka.f0_slot = 1;
      ka.f0s = nd;
    }
    ka.out = h->r;
    ka.part = h->part_b2;
    ka.sc = nullptr;
    ka.sc_w = h->sc;
    ka.init_x = 1;
    ka.x_init = h->V[nxt];
    ka.check = 1;
    if (h->nD > 0) {
      ka.dv = h->bvD[sb] + (int64_t)k * L * nDa;
      ka.dvs = nDa;
      ka.didx = h->didx;
    }
    return ka;
  };
  for (int k = 0; k < K; ++k) {
    const sa::KronArgs ka = step_args(k);
    {
      // theta-scheme right-hand side (Eq. 20), first iterate with the
      // Dirichlet values, and the residual check of the previous step (the
      // x pass of steps after the first ran fused with the previous solve)
      StageScope s(h, SA_STAGE_RHS, bsx);
      sa::launch_theta_checked_rhs(bsx, sm, ka, h->fp, k == 0);
    }
    lap.mark(3);
    {
      StageScope s(h, SA_STAGE_PCG, bsx);
      sa::FusedPcg f = h->fp;
      f.x = h->V[(par0 + k + 1) & 1];
      f.status = next_status(h, L, 1);
      f.update_x = 1;
      f.check_mask = 0;
      for (int l = 0; l < L; ++l)
        if (h->chk_pending[pids[l]]) f.check_mask |= 1ull << l;
      f.part_chk = h->part_chk;
      f.np_chk = sa::zx_blocks(h->kargs.op);
      f.chk_rtol2 = h->force_rollback ? 0.0 : f.rtol2;
      f.chk_bw2 = h->force_rollback ? 0.0 : f.bw2;
      sa::launch_theta_checked_solve(bsx, sm, f, k + 1 == K);
      if (k + 1 < K) sa::launch_xbwd_x(bsx, sm, f, step_args(k + 1));
    }
    for (int l = 0; l < L; ++l) {
      h->chk_pending[pids[l]] = 1;
      h->paths[pids[l]].step++;
    }
    h->stats.steps += L;
    if (h->blk_overlap < K && k + 1 == std::max(1, K - h->blk_overlap)) {
      hip_check(hipEventRecord(h->ev_blk_mid, bsx), "event record");
      h->blk_mid_live = true;
    }
    lap.mark(4);
  }
  // the block's last F, Dirichlet values, T~ and grad T~ into the paths' state
  const int fin = (int)(h->paths[pids[0]].step & 1);
  const int64_t last = (int64_t)(K - 1) * L;
  sa::CopyJob jobs[4];
  int nj = 0;
  jobs[nj++] = sa::CopyJob{h->bF[sb] + last * nd, h->Fb[fin], nd, nd, nd};
  jobs[nj++] = sa::CopyJob{h->bT[sb] + last * st, h->Tb, st, st, st};
  jobs[nj++] = sa::CopyJob{h->bG[sb] + last * 3 * st, h->Gb, 3 * st, 3 * st, 3 * st};
  if (h->nD > 0) jobs[nj++] = sa::CopyJob{h->bvD[sb] + last * nDa, h->vD, nDa, nDa, nDa};
  sa::launch_copy_jobs(bsx, sm, jobs, nj);
  hip_check(hipEventRecord(h->ev_blk_done[sb], bsx), "event record");
  h->blk_live[sb] = true;
  lap.mark(4);
}

// the residual checks of checked updates still pending at the end of a call:
// A u^n from u^n alone (in V[n & 1]), against the stored right-hand side,
// per parity of the paths' steps
void flush_checks(sa_iga *h) {
  std::vector<int> ids[2];
  for (int p = 0; p < (int)h->chk_pending.size(); ++p)
    if (h->chk_pending[p]) ids[h->paths[p].step & 1].push_back(p);
  if (ids[0].empty() && ids[1].empty()) return;
  const hipStream_t bsx = solve_stream(h);
  StageScope sc(h, SA_STAGE_PCG, bsx);
  const double rt = h->force_rollback ? 0.0 : h->fp.rtol2, bw = h->force_rollback ? 0.0 : h->fp.bw2;
  for (int par = 0; par < 2; ++par)
    for (size_t i0 = 0; i0 < ids[par].size(); i0 += sa::kMaxBatch) {
      const size_t i1 = std::min(ids[par].size(), i0 + (size_t)sa::kMaxBatch);
      sa::SlotMap sm{};
      sm.count = (int)(i1 - i0);
      for (size_t i = i0; i < i1; ++i) sm.path[i - i0] = ids[par][i];
      sa::KronArgs k = h->kargs;
      k.v = h->V[par];
      k.check = 1;
      k.check_only = 1;
      k.sc = nullptr;
      k.sc_w = nullptr;
      sa::launch_kron(bsx, sm, k, true);
      sa::launch_check_status(bsx, sm, h->part_chk, h->np_st, rt, bw, next_status(h, sm.count, 1));
    }
  std::fill(h->chk_pending.begin(), h->chk_pending.end(), 0);
}

// advance every live path by one step: launches of at most kMaxBatch paths,
// grouped by the parity of their steps
void step_all(sa_iga *h) {
  std::vector<int> ids[2];
  for (int p = 0; p < (int)h->paths.size(); ++p)
    if (h->paths[p].step < h->paths[p].n_steps) ids[h->paths[p].step & 1].push_back(p);
  for (int par = 0; par < 2; ++par) {
    const auto &v = ids[par];
    const size_t nb = (v.size() + sa::kMaxBatch - 1) / sa::kMaxBatch;
    for (size_t b = 0; b < nb; ++b) {
      // equal shares: 65 paths go as 33 + 32, not 64 + 1
      const size_t i0 = v.size() * b / nb, i1 = v.size() * (b + 1) / nb;
      step_batch(h, std::vector<int>(v.begin() + i0, v.begin() + i1));
    }
  }
}

std::vector<float> to_float(const std::vector<double> &v) {
  std::vector<float> f(v.size());
  for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
  return f;
}

void upload_fd(sa_iga *h, const sa::FdData &F, DevFd &D) {
  D.op = sa::FdOp{};
  for (int d = 0; d < 3; ++d) {
    D.op.n[d] = F.n[d];
    D.op.lo[d] = F.lo[d];
    D.op.m[d] = F.m[d];
    D.op.U[d] = dev_upload(h->owned, F.U[d], h->stream);
  }
  D.op.inv_diag = dev_upload(h->owned, F.inv_diag, h->stream);
  const size_t nb = F.inv_diag.size();
  D.op.t1 = dev_alloc<double>(h->owned, nb);
  D.op.t2 = dev_alloc<double>(h->owned, nb);
}

DevCsr upload_csr(sa_iga *h, const sa::Csr &C) {
  DevCsr d;
  d.nrow = C.nrow;
  d.rowptr = dev_upload(h->owned, C.rowptr, h->stream);
  d.col = dev_upload(h->owned, C.col, h->stream);
  d.val = dev_upload(h->owned, C.val, h->stream);
  return d;
}

template <class T>
T *dev_zeros(sa_iga *h, size_t n) {
  T *p = dev_alloc<T>(h->owned, n);
  hip_check(hipMemsetAsync(p, 0, std::max<size_t>(n, 1) * sizeof(T), h->stream), "memset");
  return p;
}

// splitmix64: fixed pseudo-random sequences (audit subset, operator checks)
uint64_t splitmix64(uint64_t &x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// y = cM (M2 x M1 x M0) x + c0 (M2 x M1 x K0) x + c1 (M2 x K1 x M0) x + c2 (K2 x M1 x M0) x
// with dense 1-D factors (host check of the matrix-free device operator)
void kron_apply_host(const int n[3], const std::vector<double> *M1, const std::vector<double> *K1, double cM,
                     const double c[3], const std::vector<double> &x, std::vector<double> &y) {
  const int64_t N = (int64_t)n[0] * n[1] * n[2];
  const int64_t st[3] = {1, n[0], (int64_t)n[0] * n[1]};
  auto pass = [&](int d, const std::vector<double> &F, const std::vector<double> &in, std::vector<double> &out) {
    out.assign(N, 0.0);
    for (int64_t r = 0; r < N; ++r) {
      const int i = (int)((r / st[d]) % n[d]);
      double s = 0.0;
      for (int j = 0; j < n[d]; ++j) s += F[(size_t)i * n[d] + j] * in[r + (int64_t)(j - i) * st[d]];
      out[r] = s;
    }
  };
  std::vector<double> t0, t1, a, b, c1v, s(N), w(N), z0, z1;
  pass(0, M1[0], x, t0);
  pass(0, K1[0], x, t1);
  pass(1, M1[1], t0, a);
  pass(1, M1[1], t1, b);
  pass(1, K1[1], t0, c1v);
  for (int64_t r = 0; r < N; ++r) {
    s[r] = cM * a[r] + c[0] * b[r] + c[1] * c1v[r];
    w[r] = c[2] * a[r];
  }
  pass(2, M1[2], s, z0);
  pass(2, K1[2], w, z1);
  y.resize(N);
  for (int64_t r = 0; r < N; ++r) y[r] = z0[r] + z1[r];
}

// matrix-free A and B when the Kronecker form reproduces the assembled A
void build_kron(sa_iga *h) {
  const sa::Model &m = h->m;
  const int n[3] = {m.P.n[0], m.P.n[1], m.P.n[2]};
  const double th = m.opt.theta;
  const double cM = m.mat.rho * m.mat.cp * m.mean_detJ / m.dt;
  double cA[3], cB[3];
  for (int d = 0; d < 3; ++d) {
    cA[d] = th * m.mat.k * m.mean_metric[d];
    cB[d] = -(1.0 - th) * m.mat.k * m.mean_metric[d];
  }
  const int64_t N = h->nd;
  std::vector<double> x(N), y, ym(N), yk(N);
  uint64_t st = 0x243f6a8885a308d3ull;
  for (int64_t i = 0; i < N; ++i) x[i] = (double)(splitmix64(st) >> 11) / 9007199254740992.0 - 0.5;
  kron_apply_host(n, m.M1, m.K1, cM, cA, x, y);
  m.M.apply(x.data(), ym.data());
  m.K.apply(x.data(), yk.data());
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const double ya = ym[i] / m.dt + th * yk[i];
    num = std::max(num, std::fabs(y[i] - ya));
    den = std::max(den, std::fabs(ya));
  }
  if (!(den > 0 && num <= 1e-12 * den)) return;
  sa::KronArgs &k = h->kargs;
  k = sa::KronArgs{};
  for (int d = 0; d < 3; ++d) {
    const int nd = n[d], p = m.P.b[d].p, w = 2 * p + 1;
    std::vector<double> Mb((size_t)nd * w, 0.0), Kb((size_t)nd * w, 0.0);
    for (int i = 0; i < nd; ++i)
      for (int kk = 0; kk < w; ++kk) {
        const int j = i - p + kk;
        if (j < 0 || j >= nd) continue;
        Mb[(size_t)i * w + kk] = m.M1[d][(size_t)i * nd + j];
        Kb[(size_t)i * w + kk] = m.K1[d][(size_t)i * nd + j];
      }
    k.op.n[d] = nd;
    k.op.p[d] = p;
    k.op.Mb[d] = dev_upload(h->owned, Mb, h->stream);
    k.op.Kb[d] = dev_upload(h->owned, Kb, h->stream);
    k.op.cA[d] = cA[d];
    k.op.cB[d] = cB[d];
  }
  k.op.cM = cM;
  k.nrow = N;
  k.vs = N;
  k.np = h->np_st;
  k.mask = h->free_mask;
  k.theta = th;
  h->zx_ok = sa::zx_fits(n[0]);
  const bool chk = h->fd_exact && h->zx_ok;
  k.ts = (chk ? 10 : 8) * N;
  k.t = dev_zeros<double>(h, (size_t)h->S * k.ts);
  if (chk) {
    h->bprev = dev_zeros<double>(h, (size_t)h->S * N);
    h->part_chk = dev_zeros<double>(h, (size_t)h->S * 3 * std::max<int64_t>(h->np_st, sa::zx_blocks(k.op)));
    k.bprev = h->bprev;
    k.part_chk = h->part_chk;
  }
  h->chk_pending.assign((size_t)h->S, 0);
  h->kron = true;
}

// network inputs (box, point features, source bins) for every object; the
// weights, buffers and audit points of the surrogate form
void build_network_state(sa_iga *h, const sa_patch *patch, const sa_scan_path *scan) {
  const sa::Model &m = h->m;
  const int64_t nctrl = (int64_t)patch->n_ctrl[0] * patch->n_ctrl[1] * patch->n_ctrl[2];
  for (int d = 0; d < 3; ++d) {
    h->box_lo[d] = INFINITY;
    h->box_hi[d] = -INFINITY;
  }
  for (int64_t i = 0; i < nctrl; ++i)
    for (int d = 0; d < 3; ++d) {
      h->box_lo[d] = std::min(h->box_lo[d], patch->ctrl_xyzw[4 * i + d]);
      h->box_hi[d] = std::max(h->box_hi[d], patch->ctrl_xyzw[4 * i + d]);
    }
  const sa::BoundaryTables &bt = m.bt;
  std::vector<float> pf((size_t)bt.nq * sa::kMlpPoint);
  for (int64_t q = 0; q < bt.nq; ++q)
    for (int d = 0; d < 3; ++d) {
      const double ext = h->box_hi[d] - h->box_lo[d];
      pf[q * 6 + d] = (float)(ext > 0 ? 2.0 * (bt.x[3 * q + d] - h->box_lo[d]) / ext - 1.0 : 0.0);
      pf[q * 6 + 3 + d] = (float)bt.nrm[3 * q + d];
    }
  h->pf = dev_upload(h->owned, pf, h->stream);
  const int64_t N = scan->src_offset[scan->n_paths];
  std::vector<int8_t> sb(std::max<int64_t>(N, 1), 0);
  for (int64_t i = 0; i < N; ++i) {
    int idx[3];
    for (int d = 0; d < 3; ++d) {
      const double ext = h->box_hi[d] - h->box_lo[d];
      const double u = ext > 0 ? std::floor(4.0 * (scan->xyz[3 * i + d] - h->box_lo[d]) / ext) : 0.0;
      idx[d] = u < 0 ? 0 : (u > 3 ? 3 : (int)u);
    }
    sb[i] = (int8_t)(idx[0] + 4 * idx[1] + 16 * idx[2]);
  }
  h->sbin = dev_upload(h->owned, sb, h->stream);
  h->bins = dev_zeros<float>(h, (size_t)sa::kMaxBatch * sa::kMlpBins);
  if (m.opt.precision != SA_PREC_SURROGATE) return;

  h->net = true;
  const float *wb = m.opt.surrogate_weights;
  h->net_T = wb[0];
  h->net_G = wb[1];
  h->net_E = wb[2];
  std::vector<float> w(wb + 3, wb + 3 + sa::kNetParams);
  h->nw = dev_upload(h->owned, w, h->stream);
  const int64_t off[3] = {sa::MlpLayout::W2, sa::MlpLayout::W3, sa::MlpLayout::W4};
  for (int l = 0; l < 3; ++l) {
    h->nWb[l] = dev_alloc<sa::bf16_t>(h->owned, (size_t)sa::kMlpHid * sa::kMlpHid);
    sa::launch_to_bf16(h->stream, (int64_t)sa::kMlpHid * sa::kMlpHid, h->nw + off[l], h->nWb[l]);
  }
  h->nW3p = dev_alloc<sa::bf16_t>(h->owned, (size_t)sa::kMlpHid * sa::kMlpHid);
  h->nW4p = dev_alloc<sa::bf16_t>(h->owned, (size_t)sa::kMlpHid * sa::kMlpHid);
  sa::launch_net_permute(h->stream, h->nWb[1], h->nW3p);
  sa::launch_net_permute(h->stream, h->nWb[2], h->nW4p);
  h->net_fused = sa::net_fused_lds() + 1024 <= h->lds_per_block && sa::net_fused_prepare() &&
                 !std::getenv("SA_IGA_NET_LAYERWISE");
  h->cvec = dev_zeros<float>(h, (size_t)sa::kMaxBatch * sa::kMlpHid);
  h->netf = dev_zeros<double>(h, (size_t)sa::kMaxBatch * 4 * h->stride);
  h->net_rows = std::min<int64_t>(131072, (int64_t)sa::kMaxBatch * h->stride);
  h->hA = dev_alloc<sa::bf16_t>(h->owned, (size_t)h->net_rows * sa::kMlpHid);
  h->hB = dev_alloc<sa::bf16_t>(h->owned, (size_t)h->net_rows * sa::kMlpHid);
  // no path uses the network before an audit has passed
  h->use_exact.assign(h->paths.size(), 1);
  h->next_audit.assign(h->paths.size(), -1);
  // audit points: ceil(audit_frac nq) of the boundary points, drawn once
  const int64_t nq = bt.nq;
  h->na = std::min<int64_t>(nq, std::max<int64_t>(1, (int64_t)std::ceil(m.opt.audit_frac * (double)nq)));
  std::vector<int64_t> perm(nq);
  for (int64_t i = 0; i < nq; ++i) perm[i] = i;
  uint64_t st = 0x5a17a0d17ull;
  for (int64_t i = 0; i < h->na; ++i) {
    const int64_t j = i + (int64_t)(splitmix64(st) % (uint64_t)(nq - i));
    std::swap(perm[i], perm[j]);
  }
  std::sort(perm.begin(), perm.begin() + h->na);
  h->stride_a = (h->na + 63) / 64 * 64;
  std::vector<double> x(h->na), y(h->na), z(h->na), q2(h->na);
  std::vector<float> apf((size_t)h->na * 6);
  for (int64_t i = 0; i < h->na; ++i) {
    const int64_t q = perm[i];
    x[i] = bt.x[3 * q] - m.P.center[0];
    y[i] = bt.x[3 * q + 1] - m.P.center[1];
    z[i] = bt.x[3 * q + 2] - m.P.center[2];
    q2[i] = x[i] * x[i] + y[i] * y[i] + z[i] * z[i];
    for (int j = 0; j < 6; ++j) apf[i * 6 + j] = pf[q * 6 + j];
  }
  h->ax = dev_upload(h->owned, x, h->stream);
  h->ay = dev_upload(h->owned, y, h->stream);
  h->az = dev_upload(h->owned, z, h->stream);
  h->aq2 = dev_upload(h->owned, q2, h->stream);
  h->afx = dev_upload(h->owned, to_float(x), h->stream);
  h->afy = dev_upload(h->owned, to_float(y), h->stream);
  h->afz = dev_upload(h->owned, to_float(z), h->stream);
  h->afq2 = dev_upload(h->owned, to_float(q2), h->stream);
  h->arole = dev_upload(h->owned, std::vector<int8_t>(h->na, (int8_t)SA_FACE_SOURCE_PLANE), h->stream);
  h->apf = dev_upload(h->owned, apf, h->stream);
  h->aT = dev_zeros<double>(h, (size_t)sa::kMaxBatch * h->stride_a);
  h->aG = dev_zeros<double>(h, (size_t)sa::kMaxBatch * 3 * h->stride_a);
  h->aLD = dev_zeros<double>(h, (size_t)sa::kMaxBatch * h->stride_a);
  h->anet = dev_zeros<double>(h, (size_t)sa::kMaxBatch * 4 * h->stride_a);
  hip_check(hipStreamSynchronize(h->stream), "sync");
  hip_check(hipGetLastError(), "kernel launch");
}

// Faces whose boundary points form a grid along Cartesian axes: the points of
// face f are stored as off + b * na + a (a the faster parametric direction of
// the face, Gauss points within elements), so the check is that coordinate
// ax_a depends on a only, ax_b on b only and ax_n is constant, each within
// 1e-14 of the patch size (a few units in the last place).
void build_tensor_faces(sa_iga *h) {
  const sa::Model &m = h->m;
  const sa::BoundaryTables &bt = m.bt;
  const sa::PatchData &P = m.P;
  std::vector<sa::TFace> faces;
  std::vector<int32_t> tiles, gen;
  std::vector<double> coords;
  std::vector<std::pair<size_t, size_t>> where;   // per tensor face: offsets of sa, sb in coords
  double ext = 0.0;
  for (int64_t q = 0; q < bt.nq; ++q)
    for (int c = 0; c < 3; ++c) ext = std::max(ext, std::fabs(bt.x[3 * q + c] - P.center[c]));
  const double tol = 1e-14 * std::max(ext, 1e-300);
  const bool allow = !std::getenv("SA_IGA_NO_TENSOR");
  for (int f = 0; f < 6; ++f) {
    const int64_t off = bt.face_off[f], n = bt.face_off[f + 1] - off;
    if (n <= 0) continue;
    const int d = f / 2, pa = (d == 0) ? 1 : 0, pb = (d == 2) ? 1 : 2;
    const int na = P.b[pa].n_el() * P.qf, nb = P.b[pb].n_el() * P.qf;
    auto X = [&](int64_t q, int c) { return bt.x[3 * q + c] - P.center[c]; };
    bool ok = allow && (int64_t)na * nb == n && na > 1 && nb > 1;
    int ax[3] = {-1, -1, -1};   // a, b, n
    if (ok) {
      // the normal axis: the coordinate with the smallest spread over the face
      double spread[3];
      for (int c = 0; c < 3; ++c) {
        double lo = X(off, c), hi = lo;
        for (int64_t q = off; q < off + n; ++q) {
          lo = std::min(lo, X(q, c));
          hi = std::max(hi, X(q, c));
        }
        spread[c] = hi - lo;
      }
      ax[2] = (int)(std::min_element(spread, spread + 3) - spread);
      // along a (first row) the coordinate that moves most
      double best = -1.0;
      for (int c = 0; c < 3; ++c) {
        if (c == ax[2]) continue;
        const double v = std::fabs(X(off + na - 1, c) - X(off, c));
        if (v > best) { best = v; ax[0] = c; }
      }
      ax[1] = 3 - ax[0] - ax[2];
      const double sn = X(off, ax[2]);
      for (int b = 0; b < nb && ok; ++b)
        for (int a = 0; a < na && ok; ++a) {
          const int64_t q = off + (int64_t)b * na + a;
          ok = std::fabs(X(q, ax[0]) - X(off + a, ax[0])) <= tol && std::fabs(X(q, ax[1]) - X(off + (int64_t)b * na, ax[1])) <= tol &&
               std::fabs(X(q, ax[2]) - sn) <= tol;
        }
    }
    if (!ok) {
      for (int64_t q = off; q < off + n; ++q) gen.push_back((int32_t)q);
      continue;
    }
    sa::TFace F{};
    F.na = na;
    F.nb = nb;
    F.ax_a = ax[0];
    F.ax_b = ax[1];
    F.ax_n = ax[2];
    F.off = off;
    F.sn = X(off, ax[2]);
    where.push_back({coords.size(), coords.size() + (size_t)na});
    for (int a = 0; a < na; ++a) coords.push_back(X(off + a, ax[0]));
    for (int b = 0; b < nb; ++b) coords.push_back(X(off + (int64_t)b * na, ax[1]));
    const int fi = (int)faces.size();
    faces.push_back(F);
    for (int b0 = 0; b0 < nb; b0 += sa::kTensorTile)
      for (int a0 = 0; a0 < na; a0 += sa::kTensorTile) {
        tiles.push_back(fi);
        tiles.push_back(b0);
        tiles.push_back(a0);
        tiles.push_back(0);
      }
  }
  if (faces.empty()) return;
  const double *dc = dev_upload(h->owned, coords, h->stream);
  for (size_t i = 0; i < faces.size(); ++i) {
    faces[i].sa = dc + where[i].first;
    faces[i].sb = dc + where[i].second;
  }
  std::vector<uint8_t> raw(faces.size() * sizeof(sa::TFace));
  std::memcpy(raw.data(), faces.data(), raw.size());
  h->tens = sa::TensorArgs{};
  h->tens.faces = (const sa::TFace *)dev_upload(h->owned, raw, h->stream);
  h->tens.tiles = (const int4 *)dev_upload(h->owned, tiles, h->stream);
  h->tens.n_tiles = (int)(tiles.size() / 4);
  h->tens.sx = h->sx;
  h->tens.sy = h->sy;
  h->tens.sz = h->sz;
  {
    // workgroups per compute unit of the sum: with one path, room is left
    // for the solver kernels that run beside it (two per unit); a batch is
    // dominated by its sum, which then takes the whole device (eight per
    // unit, more than fit at once)
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, h->device), "device properties");
    const char *g = std::getenv("SA_IGA_SUM_GROUPS_PER_CU");
    const char *gb = std::getenv("SA_IGA_SUM_GROUPS_PER_CU_BATCH");
    h->tens.max_groups = (int)((g ? std::max(0.0, std::atof(g)) : 2.0) * prop.multiProcessorCount);
    h->n_cu = prop.multiProcessorCount;
    h->sum_groups_per_cu_batch = gb ? std::max(0, std::atoi(gb)) : 8;
    h->tens.max_groups_batch = h->sum_groups_per_cu_batch * prop.multiProcessorCount;
    // a blocked call's sum: one workgroup per work item (they retire often,
    // so the solver kernels beside the sum get compute units), three per
    // compute unit (no LDS padding: its registers allow three)
    const char *bg = std::getenv("SA_IGA_BLOCK_SUM_GROUPS_PER_CU");
    const char *pad = std::getenv("SA_IGA_BLOCK_SUM_LDS_PAD");
    h->blk_groups = (int)((bg ? std::max(0.0, std::atof(bg)) : 0.0) * prop.multiProcessorCount);
    h->blk_pad = pad ? std::max(0, std::min(96 * 1024, std::atoi(pad))) : 0;
    if (h->blk_pad > 0 && !sa::sum_tensor_prepare(h->blk_pad)) h->blk_pad = 0;
    // launches of several paths per step: LDS padding that leaves two per
    // compute unit and room for the theta-step kernels beside the sum
    const char *bpad = std::getenv("SA_IGA_BATCH_SUM_LDS_PAD");
    h->tens.lds_pad = bpad ? std::max(0, std::min(96 * 1024, std::atoi(bpad))) : 10000;
    if (h->tens.lds_pad > 0 && !sa::sum_tensor_prepare(std::max(h->tens.lds_pad, h->blk_pad))) h->tens.lds_pad = 0;
  }
  h->n_gen = (int64_t)gen.size();
  h->n_tfaces = (int)faces.size();
  if (!gen.empty()) h->gen_idx = dev_upload(h->owned, gen, h->stream);
  h->use_tensor = true;
  hip_check(hipStreamSynchronize(h->stream), "sync");
}

// Three streams per device, shared by every object and kept until the
// process ends: the solves (an object's own stream), the sums and the
// post-processing.  Hardware queues are few (four per process by default);
// streams per object would make the objects' streams share queues, and two
// streams of one object on one queue would run its overlapped steps in queue
// order.  Objects stepped one after the other lose nothing by sharing.
struct DeviceStreams {
  hipStream_t solve = nullptr, sum = nullptr, post = nullptr;
};

const DeviceStreams &device_streams(int device) {
  static std::mutex mu;
  static std::map<int, DeviceStreams> pool;
  std::lock_guard<std::mutex> lock(mu);
  auto it = pool.find(device);
  if (it != pool.end()) return it->second;
  DeviceStreams d;
  hip_check(hipStreamCreateWithFlags(&d.solve, hipStreamNonBlocking), "stream");
  hip_check(hipStreamCreateWithFlags(&d.sum, hipStreamNonBlocking), "stream");
  hip_check(hipStreamCreateWithFlags(&d.post, hipStreamNonBlocking), "stream");
  return pool.emplace(device, d).first->second;
}

// inverse of a dense SPD matrix (row-major, n x n) by Gauss-Jordan
// elimination with partial pivoting; false if a pivot vanishes
bool invert_dense(std::vector<double> &a, int n) {
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
    if (!(std::fabs(a[(size_t)piv * n + c]) > 0.0)) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[(size_t)piv * n + k], a[(size_t)c * n + k]);
        std::swap(inv[(size_t)piv * n + k], inv[(size_t)c * n + k]);
      }
    const double d = 1.0 / a[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      a[(size_t)c * n + k] *= d;
      inv[(size_t)c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
      }
    }
  }
  a.swap(inv);
  return true;
}

// The trace mass matrix of a single DIRICHLET face whose surface measure and
// weights factor over its two parametric directions (the annular bottom face
// of the quarter annulus: dS = r r'(xi1) theta'(xi0) dxi0 dxi1, weights along
// the arc only) is a Kronecker product A (x) B of two 1-D matrices.  The
// factors are read off the assembled matrix (A from the rows of the first
// layer along b, B from those of the first point along a, scaled by their
// common entry) and every entry is checked; the projection (Eq. 11) is then
// solved exactly by the dense inverses, A^{-1} (x) B^{-1}.
void try_kronecker_trace_mass(sa_iga *h) {
  const sa::Model &m = h->m;
  int nf = 0, face = -1;
  for (int f = 0; f < 6; ++f)
    if (m.P.role[f] == SA_FACE_DIRICHLET) {
      nf++;
      face = f;
    }
  if (nf != 1 || std::getenv("SA_IGA_NO_KRON_DIRICHLET")) return;
  const int d = face / 2, da = (d == 0) ? 1 : 0, db = (d == 2) ? 1 : 2;
  const int na = m.P.n[da], nb = m.P.n[db];
  if ((int64_t)na * nb != h->nD) return;
  const sa::Csr &M = m.mass_dir;
  auto entry = [&](int64_t r, int64_t c) {
    for (int64_t e = M.rowptr[r]; e < M.rowptr[r + 1]; ++e)
      if (M.col[e] == c) return M.val[e];
    return 0.0;
  };
  const double piv = entry(0, 0);
  if (!(piv > 0.0)) return;
  std::vector<double> A((size_t)na * na), B((size_t)nb * nb);
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < na; ++j) A[(size_t)i * na + j] = entry(i, j) / piv;
  for (int k = 0; k < nb; ++k)
    for (int l = 0; l < nb; ++l) B[(size_t)k * nb + l] = entry((int64_t)na * k, (int64_t)na * l);
  double worst = 0.0, big = 0.0;
  int64_t nnz_ab = 0;
  for (int64_t r = 0; r < h->nD; ++r)
    for (int64_t e = M.rowptr[r]; e < M.rowptr[r + 1]; ++e) {
      const int64_t c = M.col[e];
      const double v = A[(size_t)(r % na) * na + (c % na)] * B[(size_t)(r / na) * nb + (c / na)];
      worst = std::max(worst, std::fabs(M.val[e] - v));
      big = std::max(big, std::fabs(M.val[e]));
    }
  for (double a : A)
    if (a != 0.0) nnz_ab++;
  int64_t nnz_b = 0;
  for (double b : B)
    if (b != 0.0) nnz_b++;
  nnz_ab *= nnz_b;
  // every product entry must be an assembled entry (the matrix's pattern)
  if (!(big > 0.0) || worst > 1e-13 * big || nnz_ab != M.rowptr[h->nD]) return;
  if (!invert_dense(A, na) || !invert_dense(B, nb)) return;
  if (!(sa::dir_direct_lds(na, nb) + 1024 <= h->lds_per_block && sa::dir_direct_prepare(sa::dir_direct_lds(na, nb))))
    return;
  const int64_t S = h->S;
  sa::DirDirect &a = h->ddir;
  a.na = na;
  a.nb = nb;
  a.Ia = dev_upload(h->owned, A, h->stream);
  a.Ib = dev_upload(h->owned, B, h->stream);
  a.inv_area = 1.0;
  a.b = h->bD;
  a.vD = h->vD;
  a.vs = h->nDa;
  a.dofs = h->dir_dofs;
  a.xs = h->nd;
  a.tmp = dev_zeros<double>(h, (size_t)S * na * nb);
  h->dir_direct = true;
  h->dir_exact = true;   // the projection right-hand side goes with the load gather
}

void build_object(sa_iga *h, const sa_patch *patch, const sa_material *mat, const sa_scan_path *scan) {
  sa::Model &m = h->m;
  // device and stream
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) throw sa::SaError{SA_EDEVICE, "no HIP device"};
  hip_check(hipGetDevice(&h->device), "get device");
  hipDeviceProp_t prop;
  hip_check(hipGetDeviceProperties(&prop, h->device), "device properties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    throw sa::SaError{SA_EDEVICE, std::string("device is ") + prop.gcnArchName + ", built for gfx950"};
  const DeviceStreams &ds = device_streams(h->device);
  // the fixed scratch area's device address, taken once per device (nullptr:
  // the allocation-free evaluation reports an error)
  h->scratch = sa::noalloc_scratch(h->device);
  h->own_stream = ds.solve;
  h->stream = h->own_stream;
  h->lds_per_block = prop.sharedMemPerBlock;

  // model set-up (host)
  sa::load_patch(patch, m.P);
  m.mat = *mat;
  m.dt = scan->dt;
  sa::assemble_volume(m);
  sa::build_boundary(m);
  sa::build_fd(m);
  const int64_t nd = m.P.ndof;
  h->nd = nd;
  const double th = m.opt.theta;
  const int S = scan->n_paths;
  h->S = S;

  // theta-scheme stencils A = M/dt + theta K, B = M/dt - (1-theta) K
  {
    std::vector<double> A(m.M.val.size()), B(m.M.val.size());
    for (size_t i = 0; i < A.size(); ++i) {
      A[i] = m.M.val[i] / m.dt + th * m.K.val[i];
      B[i] = m.M.val[i] / m.dt - (1.0 - th) * m.K.val[i];
    }
    h->Aop = sa::StencilOp{};
    for (int d = 0; d < 3; ++d) { h->Aop.n[d] = m.M.n[d]; h->Aop.hw[d] = m.M.hw[d]; }
    h->Aop.n_off = m.M.n_off;
    h->Aop.nrow = nd;
    h->Aop.A = dev_upload(h->owned, A, h->stream);
    h->Bval = dev_upload(h->owned, B, h->stream);
    std::vector<uint8_t> fm(m.free_mask.begin(), m.free_mask.end());
    h->free_mask = dev_upload(h->owned, fm, h->stream);
    h->Aop.free_mask = h->free_mask;
    std::vector<double> jd(nd, 0.0);
    const int o0 = m.M.off_index(0, 0, 0);
    for (int64_t i = 0; i < nd; ++i)
      if (m.free_mask[i]) jd[i] = 1.0 / A[(size_t)o0 * nd + i];
    h->A_invdiag = dev_upload(h->owned, jd, h->stream);
    hip_check(hipStreamSynchronize(h->stream), "sync");
    // an exact FD solve (affine axis-aligned patch) needs no convergence loop
    h->fd_exact = m.opt.preconditioner == SA_PRECOND_FD &&
                  sa::fd_inverse_defect(m.fd_main, m.M, A, m.free_mask) < 1e-10;
    // |A|_inf over the free rows: scale of the attainable residual
    double anorm = 0.0;
    for (int64_t i = 0; i < nd; ++i) {
      if (!m.free_mask[i]) continue;
      double rs = 0.0;
      for (int o = 0; o < m.M.n_off; ++o) rs += std::fabs(A[(size_t)o * nd + i]);
      anorm = std::max(anorm, rs);
    }
    const double bw = 64.0 * 2.220446049250313e-16 * anorm;
    h->bw2 = bw * bw;
  }
  upload_fd(h, m.fd_main, h->fd_main);
  if (m.fd_dir_ok) upload_fd(h, m.fd_dir, h->fd_dir);

  // boundary tables (centred coordinates)
  const sa::BoundaryTables &bt = m.bt;
  h->nq = bt.nq;
  h->stride = (bt.nq + 63) / 64 * 64;
  {
    std::vector<double> x(bt.nq), y(bt.nq), z(bt.nq), q2(bt.nq), nx(bt.nq), ny(bt.nq), nz(bt.nq);
    for (int64_t i = 0; i < bt.nq; ++i) {
      x[i] = bt.x[3 * i] - m.P.center[0];
      y[i] = bt.x[3 * i + 1] - m.P.center[1];
      z[i] = bt.x[3 * i + 2] - m.P.center[2];
      q2[i] = x[i] * x[i] + y[i] * y[i] + z[i] * z[i];
      nx[i] = bt.nrm[3 * i];
      ny[i] = bt.nrm[3 * i + 1];
      nz[i] = bt.nrm[3 * i + 2];
    }
    h->px = dev_upload(h->owned, x, h->stream);
    h->py = dev_upload(h->owned, y, h->stream);
    h->pz = dev_upload(h->owned, z, h->stream);
    h->pq2 = dev_upload(h->owned, q2, h->stream);
    h->fx = dev_upload(h->owned, to_float(x), h->stream);
    h->fy = dev_upload(h->owned, to_float(y), h->stream);
    h->fz = dev_upload(h->owned, to_float(z), h->stream);
    h->fq2 = dev_upload(h->owned, to_float(q2), h->stream);
    h->nx = dev_upload(h->owned, nx, h->stream);
    h->ny = dev_upload(h->owned, ny, h->stream);
    h->nz = dev_upload(h->owned, nz, h->stream);
    h->wdS = dev_upload(h->owned, bt.wdS, h->stream);
    h->role = dev_upload(h->owned, bt.role, h->stream);
    hip_check(hipStreamSynchronize(h->stream), "sync");
  }
  h->load = upload_csr(h, m.load);
  h->dproj = upload_csr(h, m.dproj);
  h->mdir = upload_csr(h, m.mass_dir);
  h->nD = (int64_t)m.dir_dofs.size();
  h->nDa = std::max<int64_t>(h->nD, 1);
  h->dir_dofs = dev_upload(h->owned, m.dir_dofs, h->stream);
  {
    std::vector<double> jd(h->nDa, 1.0);
    for (int64_t j = 0; j < h->nD; ++j)
      for (int64_t e = m.mass_dir.rowptr[j]; e < m.mass_dir.rowptr[j + 1]; ++e)
        if (m.mass_dir.col[e] == j) jd[j] = 1.0 / m.mass_dir.val[e];
    h->mdir_invdiag = dev_upload(h->owned, jd, h->stream);
  }

  // sources (centred)
  const int64_t N = scan->src_offset[scan->n_paths];
  {
    std::vector<double> x(N), y(N), z(N), E(N);
    h->h_tick.assign(scan->tick, scan->tick + N);
    for (int64_t i = 0; i < N; ++i) {
      x[i] = scan->xyz[3 * i] - m.P.center[0];
      y[i] = scan->xyz[3 * i + 1] - m.P.center[1];
      z[i] = scan->xyz[3 * i + 2] - m.P.center[2];
      E[i] = scan->energy[i];
    }
    h->sx = dev_upload(h->owned, x, h->stream);
    h->sy = dev_upload(h->owned, y, h->stream);
    h->sz = dev_upload(h->owned, z, h->stream);
    h->sE = dev_upload(h->owned, E, h->stream);
    h->stick = dev_upload(h->owned, h->h_tick, h->stream);
    hip_check(hipStreamSynchronize(h->stream), "sync");
  }
  h->ns = scan->sources_per_step;
  h->delta = scan->dt / scan->sources_per_step;
  h->rc = mat->rho * mat->cp;
  h->alpha = mat->k / h->rc;
  h->shift = scan->spot_radius * scan->spot_radius / (8.0 * h->alpha);
  h->tau_ticks = (int64_t)std::floor(m.opt.tau_near / h->delta + 1e-9);
  for (int p = 0; p < S; ++p)
    if (scan->src_offset[p + 1] - scan->src_offset[p] > 2000000000)
      throw sa::SaError{SA_EINVAL, "a path holds more than 2e9 sources"};
  h->c64 = dev_alloc<double>(h->owned, (size_t)std::max<int64_t>(N, 1) * sa::kCoefStride);
  h->c32 = dev_alloc<float>(h->owned, (size_t)std::max<int64_t>(N, 1) * sa::kCoefStride);
  build_tensor_faces(h);
  if (h->use_tensor) {
    // Eq. 8 coefficients of the tensor sum by source age: with
    // D(a) = a delta + r^2/(8 alpha), c = -1/(4 alpha D) and
    // ln A = ln(s E) - ln(rho c_p (4 pi alpha D)^{3/2}); the age runs to the
    // last step of the longest path
    int64_t steps = 0;
    for (int p = 0; p < S; ++p) steps = std::max<int64_t>(steps, scan->n_steps[p]);
    h->age_max = steps * h->ns;
    std::vector<double> ac((size_t)h->age_max + 1), al((size_t)h->age_max + 1), le((size_t)std::max<int64_t>(N, 1));
    for (int64_t a = 0; a <= h->age_max; ++a) {
      const double D = (double)a * h->delta + h->shift;
      ac[a] = -1.0 / (4.0 * h->alpha * D);
      al[a] = -std::log(h->rc * std::pow(4.0 * M_PI * h->alpha * D, 1.5));
    }
    for (int64_t i = 0; i < N; ++i) le[i] = std::log(m.opt.kernel_scale * scan->energy[i]);
    h->tens.tick = h->stick;
    h->tens.age_c = dev_upload(h->owned, ac, h->stream);
    h->tens.age_l = dev_upload(h->owned, al, h->stream);
    h->tens.src_le = dev_upload(h->owned, le, h->stream);
    hip_check(hipStreamSynchronize(h->stream), "sync");
  }

  // per-path state: u = T0 (v = 0), F = 0, Dirichlet values 0
  h->paths.resize(S);
  for (int p = 0; p < S; ++p) {
    PathState &P = h->paths[p];
    P.src0 = scan->src_offset[p];
    P.src1 = scan->src_offset[p + 1];
    P.n_steps = scan->n_steps[p];
    P.step = 0;
  }
  for (int b = 0; b < 2; ++b) {
    h->V[b] = dev_zeros<double>(h, (size_t)S * nd);
    h->Fb[b] = dev_zeros<double>(h, (size_t)S * nd);
  }
  h->vD = dev_zeros<double>(h, (size_t)S * h->nDa);
  h->bD = dev_zeros<double>(h, (size_t)S * h->nDa);
  h->pD = dev_zeros<double>(h, (size_t)S * h->nDa);
  h->Tb = dev_zeros<double>(h, (size_t)S * h->stride);
  h->Gb = dev_zeros<double>(h, (size_t)S * 3 * h->stride);
  h->LD = dev_zeros<double>(h, (size_t)S * h->stride);
  h->sc = dev_zeros<sa::PcgScalars>(h, S);
  h->sc_dir = dev_zeros<sa::PcgScalars>(h, S);
  hip_check(hipHostMalloc((void **)&h->h_sc, (size_t)S * sizeof(sa::PcgScalars), hipHostMallocDefault), "pinned");
  // generic solver work vectors
  h->gr = dev_zeros<double>(h, nd);
  h->gz = dev_zeros<double>(h, nd);
  h->gp = dev_zeros<double>(h, nd);
  h->gq = dev_zeros<double>(h, nd);
  h->rD = dev_zeros<double>(h, h->nDa);
  h->zD = dev_zeros<double>(h, h->nDa);
  h->pDg = dev_zeros<double>(h, h->nDa);
  h->qD = dev_zeros<double>(h, h->nDa);
  h->part_b = dev_zeros<double>(h, 1024);
  h->part_rz = dev_zeros<double>(h, 1024);
  h->part_pq = dev_zeros<double>(h, 1024);
  h->part_rr = dev_zeros<double>(h, 1024);
  h->sc_gen = dev_zeros<sa::PcgScalars>(h, 1);
  ensure_part(h, (int64_t)5 * h->stride * 16);

  // load gather over non-empty rows
  {
    std::vector<int32_t> rows;
    std::vector<int64_t> rp(1, 0);
    std::vector<int32_t> cl;
    std::vector<double> vl;
    for (int64_t A = 0; A < nd; ++A) {
      if (m.load.rowptr[A + 1] == m.load.rowptr[A]) continue;
      rows.push_back((int32_t)A);
      for (int64_t e = m.load.rowptr[A]; e < m.load.rowptr[A + 1]; ++e) {
        cl.push_back(m.load.col[e]);
        vl.push_back(m.load.val[e]);
      }
      rp.push_back((int64_t)cl.size());
    }
    h->grows.nrows = (int64_t)rows.size();
    h->grows.rows = dev_upload(h->owned, rows, h->stream);
    h->grows.rowptr = dev_upload(h->owned, rp, h->stream);
    h->grows.col = dev_upload(h->owned, cl, h->stream);
    h->grows.val = dev_upload(h->owned, vl, h->stream);
  }
  // Dirichlet projection: direct Kronecker solve, one-workgroup PCG, or generic
  if (h->nD > 0) {
    std::vector<int32_t> iota(h->nD);
    for (int64_t j = 0; j < h->nD; ++j) iota[j] = (int32_t)j;
    h->drows.nrows = h->nD;
    h->drows.rows = dev_upload(h->owned, iota, h->stream);
    h->drows.rowptr = h->dproj.rowptr;
    h->drows.col = h->dproj.col;
    h->drows.val = h->dproj.val;
    if (m.opt.preconditioner == SA_PRECOND_FD && m.fd_dir_ok) {
      // exactness of the Kronecker solve for the trace mass matrix
      const int64_t n = h->nD;
      std::vector<double> y(n), zz(n);
      uint64_t st = 0x2545f4914f6cdd1dull;
      for (int64_t i = 0; i < n; ++i) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        y[i] = (double)(st >> 11) / 9007199254740992.0 - 0.5;
      }
      sa::fd_apply_host(m.fd_dir, y.data(), zz.data(), n);
      double num = 0, den = 0;
      for (int64_t j = 0; j < n; ++j) {
        double sum = 0;
        for (int64_t e = m.mass_dir.rowptr[j]; e < m.mass_dir.rowptr[j + 1]; ++e)
          sum += m.mass_dir.val[e] * zz[m.mass_dir.col[e]];
        num = std::max(num, std::fabs(sum - y[j]));
        den = std::max(den, std::fabs(y[j]));
      }
      const int dm[3] = {m.fd_dir.m[0], m.fd_dir.m[1], 1};
      h->dir_exact = den > 0 && num / den < 1e-10 && sa::fused_fits(dm) &&
                     sa::fd_plane_lds(dm) + 1024 <= h->lds_per_block;
      if (h->dir_exact) {
        sa::FusedPcg &f = h->fd_dirp;
        f = sa::FusedPcg{};
        for (int d = 0; d < 3; ++d) {
          f.n[d] = dm[d];
          f.lo[d] = 0;
          f.m[d] = dm[d];
        }
        f.U0 = h->fd_dir.op.U[0];
        f.U1 = h->fd_dir.op.U[1];
        f.U2 = h->fd_dir.op.U[2];
        f.inv = h->fd_dir.op.inv_diag;
        f.r = h->bD;
        f.z = h->vD;
        f.p = h->pD;
        f.vs = h->nDa;
        f.t = dev_zeros<double>(h, (size_t)S * h->nD);
        f.ts = h->nD;
        f.sc = h->sc_dir;
        f.scatter_idx = h->dir_dofs;
        f.sos = nd;
        // with a constant scaling the solve is inv (U1 U1^T x U0 U0^T): two dense passes
        const int na = dm[0], nb = dm[1];
        if (sa::dir_direct_lds(na, nb) + 1024 <= h->lds_per_block &&
            sa::dir_direct_prepare(sa::dir_direct_lds(na, nb))) {
          std::vector<double> Ia((size_t)na * na), Ib((size_t)nb * nb);
          const auto &U0 = m.fd_dir.U[0], &U1 = m.fd_dir.U[1];
          for (int i = 0; i < na; ++i)
            for (int j = 0; j < na; ++j) {
              double acc = 0.0;
              for (int q = 0; q < na; ++q) acc += U0[(size_t)i * na + q] * U0[(size_t)j * na + q];
              Ia[(size_t)i * na + j] = acc;
            }
          for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) {
              double acc = 0.0;
              for (int q = 0; q < nb; ++q) acc += U1[(size_t)i * nb + q] * U1[(size_t)j * nb + q];
              Ib[(size_t)i * nb + j] = acc;
            }
          sa::DirDirect &a = h->ddir;
          a.na = na;
          a.nb = nb;
          a.Ia = dev_upload(h->owned, Ia, h->stream);
          a.Ib = dev_upload(h->owned, Ib, h->stream);
          a.inv_area = m.fd_dir.inv_diag[0];
          a.b = h->bD;
          a.vD = h->vD;
          a.vs = h->nDa;
          a.dofs = h->dir_dofs;
          a.xs = nd;
          a.tmp = dev_zeros<double>(h, (size_t)S * na * nb);
          h->dir_direct = true;
        }
      }
    }
    if (!h->dir_exact) try_kronecker_trace_mass(h);
    if (!h->dir_exact && sa::dirichlet_fits(h->nD)) {
      sa::DirArgs &a = h->dargs;
      a = sa::DirArgs{};
      a.nD = (int)h->nD;
      a.mrow = h->mdir.rowptr;
      a.mcol = h->mdir.col;
      a.mval = h->mdir.val;
      a.fd = (m.opt.preconditioner == SA_PRECOND_FD && m.fd_dir_ok) ? 1 : 0;
      a.na = m.fd_dir_ok ? m.fd_dir.m[0] : 0;
      a.nb = m.fd_dir_ok ? m.fd_dir.m[1] : 0;
      a.Ua = a.fd ? h->fd_dir.op.U[0] : nullptr;
      a.Ub = a.fd ? h->fd_dir.op.U[1] : nullptr;
      a.inv = a.fd ? h->fd_dir.op.inv_diag : nullptr;
      a.jacobi = h->mdir_invdiag;
      a.dofs = h->dir_dofs;
      a.rtol2 = m.opt.pcg_rtol * m.opt.pcg_rtol;
      a.max_iter = m.opt.pcg_max_iter;
      a.u_in_lds = a.fd ? 1 : 0;
      if (sa::dirichlet_lds(a) + 1024 > h->lds_per_block) a.u_in_lds = 0;
      h->dir_fused = sa::dirichlet_lds(a) + 1024 <= h->lds_per_block;
    }
  }
  // fused PCG on the box of free DOFs
  h->hw0 = m.M.hw[0];
  const auto &FM = m.fd_main;
  const size_t plane_lds = sa::fd_plane_lds(FM.m);
  h->pcg_fused = m.opt.preconditioner == SA_PRECOND_FD && sa::fused_fits(FM.m) &&
                 plane_lds + 1024 <= h->lds_per_block && m.M.hw[2] <= 7 && m.M.hw[0] <= 6;
  h->np_st = sa::stencil_blocks(nd);
  if (h->pcg_fused) {
    h->r = dev_zeros<double>(h, (size_t)S * nd);
    h->z = dev_zeros<double>(h, (size_t)S * nd);
    h->p = dev_zeros<double>(h, (size_t)S * nd);
    h->q = dev_zeros<double>(h, (size_t)S * nd);
    sa::FusedPcg &f = h->fp;
    f = sa::FusedPcg{};
    for (int d = 0; d < 3; ++d) {
      f.n[d] = FM.n[d];
      f.lo[d] = FM.lo[d];
      f.m[d] = FM.m[d];
    }
    f.U0 = h->fd_main.op.U[0];
    {
      const int mm = FM.m[0];
      std::vector<double> ut((size_t)mm * mm);
      for (int i = 0; i < mm; ++i)
        for (int j = 0; j < mm; ++j) ut[(size_t)j * mm + i] = FM.U[0][(size_t)i * mm + j];
      f.U0T = dev_upload(h->owned, ut, h->stream);
    }
    f.U1 = h->fd_main.op.U[1];
    f.U2 = h->fd_main.op.U[2];
    f.inv = h->fd_main.op.inv_diag;
    f.r = h->r;
    f.z = h->z;
    f.p = h->p;
    f.q = h->q;
    f.vs = nd;
    h->nbox = (int64_t)FM.m[0] * FM.m[1] * FM.m[2];
    h->t_box = dev_zeros<double>(h, (size_t)S * h->nbox);
    f.t = h->t_box;
    f.ts = h->nbox;
    f.np_rz = FM.m[1] * FM.m[2];
    h->np_fd = f.np_rz;
    h->part_rz2 = dev_zeros<double>(h, (size_t)S * 2 * f.np_rz);
    h->part_rrs = dev_zeros<double>(h, (size_t)S * f.np_rz);
    f.part_rz = h->part_rz2;
    f.part_rr = h->part_rrs;
    h->part_pq2 = dev_zeros<double>(h, (size_t)S * h->np_st);
    h->part_b2 = dev_zeros<double>(h, (size_t)S * h->np_st);
    f.part_pq = h->part_pq2;
    f.np_pq = h->np_st;
    f.part_b = h->part_b2;
    f.np_b = h->np_st;
    f.rtol2 = m.opt.pcg_rtol * m.opt.pcg_rtol;
    f.part_xx = dev_zeros<double>(h, (size_t)S * f.np_rz);
    f.bw2 = h->bw2;
    f.sc = h->sc;
  }
  if (h->pcg_fused) build_kron(h);
  build_network_state(h, patch, scan);
  h->m.opt.surrogate_weights = nullptr;   // copied; the caller's array is not kept
  h->status_cap = 8192;
  h->d_status = dev_zeros<sa::SolveStatus>(h, h->status_cap);
  // overlapped steps: the source side on a stream of its own (default
  // priority, like every stream here). Only with the fused solvers, whose
  // work buffers the two sides do not share.
  h->overlap = h->pcg_fused && (h->nD == 0 || h->dir_direct || h->dir_exact || h->dir_fused) &&
               !std::getenv("SA_IGA_SERIAL");
  h->force_rollback = std::getenv("SA_IGA_FORCE_ROLLBACK") != nullptr;
  if (const char *e = std::getenv("SA_IGA_PCG_BUDGET"))   // 2: the two-iteration form from the start (tests)
    h->pcg_budget = std::atoi(e) >= 2 ? 2 : 1;
  for (int b = 0; b < 2; ++b) {
    hip_check(hipEventCreateWithFlags(&h->ev_sum[b], hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&h->ev_part[b], hipEventDisableTiming), "event");
  }
  if (h->overlap) {
    h->ss = ds.sum;
    h->ps = ds.post;
    hip_check(hipEventCreateWithFlags(&h->ev_start, hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&h->ev_end, hipEventDisableTiming), "event");
    // batches per step: at most two parity groups of ceil(S / kMaxBatch) batches each
    const size_t ring = 2 * (2 * (size_t)((S + sa::kMaxBatch - 1) / sa::kMaxBatch) + 2);
    h->ev_src.resize(ring, nullptr);
    h->ev_rhs.resize(ring, nullptr);
    for (size_t i = 0; i < ring; ++i) {
      hip_check(hipEventCreateWithFlags(&h->ev_src[i], hipEventDisableTiming), "event");
      hip_check(hipEventCreateWithFlags(&h->ev_rhs[i], hipEventDisableTiming), "event");
    }
    h->path_rhs.assign(S, -1);
  }
  // the blocked source side: the matrix-core sum with age tables alone, no
  // network, the checked one-application theta-step, exact Dirichlet data
  h->blk_ok = h->overlap && h->pcg_fused && h->kron && h->zx_ok && h->fd_exact && h->use_tensor && h->n_gen == 0 && !h->net &&
              (h->nD == 0 || h->dir_direct) && h->age_max >= 0 && !std::getenv("SA_IGA_NO_BLOCK");
  if (h->blk_ok && h->nD > 0) {
    std::vector<int32_t> di((size_t)nd, -1);
    for (int64_t i = 0; i < h->nD; ++i) di[(size_t)h->m.dir_dofs[i]] = (int32_t)i;
    for (int64_t r = 0; r < nd; ++r)
      if (!h->m.free_mask[r] && di[r] < 0) h->blk_ok = false;
    if (h->blk_ok) h->didx = dev_upload(h->owned, di, h->stream);
  }
  if (h->blk_ok) {
    const size_t KL = kBlockSlots, st = (size_t)h->stride;
    for (int b = 0; b < 2; ++b) {
      h->bF[b] = dev_zeros<double>(h, KL * nd);   // rows the load vector never touches stay zero
      h->bT[b] = dev_zeros<double>(h, KL * st);
      h->bG[b] = dev_zeros<double>(h, KL * 3 * st);
      h->bvD[b] = dev_zeros<double>(h, KL * h->nDa);
      hip_check(hipEventCreateWithFlags(&h->ev_blk_done[b], hipEventDisableTiming), "event");
    }
    h->bLD = dev_zeros<double>(h, KL * st);
    h->bbD = dev_zeros<double>(h, KL * h->nDa);
    if (h->nD > 0 && h->ddir.tmp) h->btmp = dev_zeros<double>(h, KL * (size_t)h->ddir.na * h->ddir.nb);
    hip_check(hipEventCreateWithFlags(&h->ev_blk_src, hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&h->ev_blk_mid, hipEventDisableTiming), "event");
    if (const char *e = std::getenv("SA_IGA_BLOCK_SUM_OVERLAP")) h->blk_overlap = std::max(0, std::atoi(e));
    if (const char *e = std::getenv("SA_IGA_BLOCK_STEPS")) h->blk_steps = std::max(1, std::min(kBlockSlots, std::atoi(e)));
  }
  hip_check(hipStreamSynchronize(h->stream), "sync");
  h->verbose = std::getenv("SA_IGA_VERBOSE") != nullptr;
  if (h->verbose)
    std::fprintf(stderr,
                 "[sa_iga] paths %d ndof %lld nq %lld nD %lld | lds/block %zu | dirichlet: exact %d direct %d one-wg %d | "
                 "theta-step: fused %d fd-exact %d budget %d kron %d | tensor tiles %d, generic points %lld | "
                 "blocked source side %d\n",
                 S, (long long)nd, (long long)h->nq, (long long)h->nD, h->lds_per_block, (int)h->dir_exact, (int)h->dir_direct,
                 (int)h->dir_fused, (int)h->pcg_fused, (int)h->fd_exact, h->pcg_budget, (int)h->kron,
                 h->use_tensor ? h->tens.n_tiles : 0, (long long)(h->use_tensor ? h->n_gen : h->nq), (int)h->blk_ok);
}

// parametric query points -> device CSR rows of basis values (and gradients)
struct EvalTables {
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> R, gx, gy, gz;
  std::vector<double> x;  // physical points [n][3]
};

EvalTables eval_tables(const sa::PatchData &P, int64_t n, const double *xi) {
  EvalTables t;
  t.rowptr.assign(1, 0);
  t.x.resize(3 * n);
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
    const double (&J)[3][3] = pe.J;
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double id = 1.0 / det, Ji[3][3];
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
      t.col.push_back((int32_t)pe.idx[l]);
      t.R.push_back(pe.R[l]);
      double g[3];
      for (int c = 0; c < 3; ++c) g[c] = pe.dR[l][0] * Ji[0][c] + pe.dR[l][1] * Ji[1][c] + pe.dR[l][2] * Ji[2][c];
      t.gx.push_back(g[0]);
      t.gy.push_back(g[1]);
      t.gz.push_back(g[2]);
    }
    t.rowptr.push_back((int64_t)t.col.size());
    for (int c = 0; c < 3; ++c) t.x[3 * i + c] = pe.x[c];
  }
  return t;
}

// temporary device buffers freed at scope exit
struct TempBufs {
  std::vector<void *> v;
  template <class T>
  T *alloc(size_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw sa::SaError{SA_ENOMEM, "hipMalloc"};
    v.push_back(p);
    return (T *)p;
  }
  template <class T>
  T *up(const std::vector<T> &h, hipStream_t st) {
    T *p = alloc<T>(h.size());
    if (!h.empty()) hip_check(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st), "upload");
    return p;
  }
  ~TempBufs() {
    for (void *p : v) (void)hipFree(p);
  }
};

// T~ and grad T~ of path p at time step*dt at n physical points (host in),
// into device arrays dT [stride] and dG [3][stride] that tb owns, on the
// object's stream; returns the stride
int64_t source_field_dev(sa_iga *h, TempBufs &tb, int p, int64_t step, int64_t n, const double *x, double **pT,
                         double **pG) {
  const int64_t stride = (n + 63) / 64 * 64;
  std::vector<double> cx(n), cy(n), cz(n), q2(n);
  for (int64_t i = 0; i < n; ++i) {
    cx[i] = x[3 * i] - h->m.P.center[0];
    cy[i] = x[3 * i + 1] - h->m.P.center[1];
    cz[i] = x[3 * i + 2] - h->m.P.center[2];
    q2[i] = cx[i] * cx[i] + cy[i] * cy[i] + cz[i] * cz[i];
  }
  double *dx = tb.up(cx, h->stream), *dy = tb.up(cy, h->stream), *dz = tb.up(cz, h->stream),
         *dq = tb.up(q2, h->stream);
  float *fx = tb.up(to_float(cx), h->stream), *fy = tb.up(to_float(cy), h->stream),
        *fz = tb.up(to_float(cz), h->stream), *fq = tb.up(to_float(q2), h->stream);
  std::vector<int8_t> roles(n, (int8_t)SA_FACE_SOURCE_PLANE);
  int8_t *drole = tb.up(roles, h->stream);
  double *dT = tb.alloc<double>(stride), *dg = tb.alloc<double>(3 * stride), *dld = tb.alloc<double>(stride);
  sa::PathTab tab{};
  tab.count = 1;
  fill_slot(h, tab, 0, p, step);
  const sa_stats keep = h->stats;
  sum_points(h, tab, n, stride, dx, dy, dz, dq, fx, fy, fz, fq, drole, dx, dy, dz, dx, true, stride, dT, dg,
             dld);
  h->stats.pairs = keep.pairs;
  h->stats.pairs_near = keep.pairs_near;
  *pT = dT;
  *pG = dg;
  return stride;
}

// T~ and grad T~ of path p at time step*dt at n physical points (host in / host out)
void source_field_host(sa_iga *h, int p, int64_t step, int64_t n, const double *x, double *T, double *grad) {
  if (n <= 0) return;
  TempBufs tb;
  double *dT = nullptr, *dg = nullptr;
  const int64_t stride = source_field_dev(h, tb, p, step, n, x, &dT, &dg);
  hip_check(hipMemcpyAsync(T, dT, n * sizeof(double), hipMemcpyDeviceToHost, h->stream), "download");
  if (grad)
    for (int c = 0; c < 3; ++c)
      hip_check(hipMemcpyAsync(grad + c * n, dg + c * stride, n * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                "download");
  hip_check(hipStreamSynchronize(h->stream), "sync");
  hip_check(hipGetLastError(), "kernel launch");
}

// Plan of the source-field sum for n query points in the slot of `tab`, its
// chunks lengthened (far chunks kept multiples of the FP32 record block)
// until there are at most max_chunks of them (0: no limit).
sa::SumPlan query_plan(sa_iga *h, const sa::PathTab &tab, int64_t n, int max_chunks) {
  const int64_t n_act = tab.n_act[0], n_far = tab.n_far[0];
  sa::SumPlan pl = make_plan(h, n, 1, n_far, n_act - n_far);
  while (max_chunks > 0 && pl.n_chunks_far + pl.n_chunks_near > max_chunks) {
    if (pl.n_chunks_far >= pl.n_chunks_near) {
      pl.chunk_far *= 2;
      pl.n_chunks_far = (int)((n_far + pl.chunk_far - 1) / pl.chunk_far);
    } else {
      pl.chunk_near *= 2;
      pl.n_chunks_near = (int)((n_act - n_far + pl.chunk_near - 1) / pl.chunk_near);
    }
  }
  return pl;
}

// T [n] and grad [3][n] (may be NULL) = T~ and grad T~ at the device points
// x [n][3] for the slot of `tab` with plan pl, every intermediate in the
// layout L; enqueued on the object's stream, no allocation, no wait
void source_field_in(sa_iga *h, const sa::PathTab &tab, sa::SumPlan pl, int64_t n, const double *x, double *T,
                     double *grad, const sa::NoAllocLayout &L) {
  if (n <= 0) return;
  const hipStream_t st = h->stream;
  const int64_t n_act = tab.n_act[0];
  const int nch = pl.n_chunks_far + pl.n_chunks_near;
  pl.nq = n;
  pl.part_stride = L.stride;
  sa::launch_noalloc_points(st, n, x, h->m.P.center, L);
  if (n_act > 0) {
    sa::CoeffParams cp{h->delta, h->shift, h->alpha, h->rc, h->m.opt.kernel_scale};
    sa::launch_coeff(st, tab, n_act, h->stick, h->sx, h->sy, h->sz, h->sE, cp, h->c64, h->c32);
  }
  if (nch > 0)
    sa::launch_sum(st, pl, tab, L.px, L.py, L.pz, L.pq2, L.fx, L.fy, L.fz, L.fq2, h->c64, h->c32, L.part);
  // query points: role SOURCE_PLANE, so the normals and weights are not read
  sa::launch_finalize(st, tab, true, n, nch, L.stride, L.part, L.px, L.py, L.pz, L.px, L.py, L.pz, L.px, L.role,
                      h->m.mat.k, n, T, grad ? grad : L.G, L.ld, nullptr, 0);
  hip_check(hipGetLastError(), "kernel launch");
}

// T~ and grad T~ of path p at time step*dt at n <= kNoAllocMaxPoints
// physical points, device arrays in and out, with the fixed scratch area for
// everything else: enqueued on the object's stream, no allocation, no wait.
// The source history is cut into at most kNoAllocMaxChunks chunks (the
// chunks of a call with more sources are longer than those of
// source_field_host, so the sums agree to rounding, not bitwise).
void source_field_noalloc(sa_iga *h, int p, int64_t step, int64_t n, const double *x, double *T, double *grad) {
  if (n <= 0) return;
  sa::PathTab tab{};
  tab.count = 1;
  fill_slot(h, tab, 0, p, step);
  const sa::SumPlan pl = query_plan(h, tab, n, sa::kNoAllocMaxChunks);
  const int nch = pl.n_chunks_far + pl.n_chunks_near;
  const sa::NoAllocLayout L = sa::noalloc_layout(h->scratch, n, std::max(nch, 1));
  if (L.bytes > sa::kNoAllocScratchBytes) throw sa::SaError{SA_EINVAL, "internal: scratch layout too large"};
  source_field_in(h, tab, pl, n, x, T, grad, L);
}

// the object's device-query workspace, at least `bytes` (grown after the
// work queued on its streams has finished)
void *query_workspace(sa_iga *h, size_t bytes) {
  if (bytes <= h->evw_bytes) return h->evw;
  sync_all(h);
  const size_t cap = std::max(bytes, 2 * h->evw_bytes);
  if (h->evw) {
    hip_check(hipFree(h->evw), "free");
    h->owned.erase(std::find(h->owned.begin(), h->owned.end(), h->evw));
    h->evw = nullptr;
    h->evw_bytes = 0;
  }
  h->evw = dev_alloc<unsigned char>(h->owned, cap);
  h->evw_bytes = cap;
  return h->evw;
}

// the patch geometry on the device, uploaded once
const sa::GeoDev &geometry_on_device(sa_iga *h) {
  if (h->geo_ready) return h->geo;
  const sa::PatchData &P = h->m.P;
  for (int d = 0; d < 3; ++d) {
    h->geo.t[d] = dev_upload(h->owned, P.b[d].t, h->stream);
    h->geo.p[d] = P.b[d].p;
    h->geo.n[d] = P.b[d].n;
  }
  h->geo.ctrl = dev_upload(h->owned, P.ctrl, h->stream);
  h->geo_ready = true;
  return h->geo;
}

int path_index(sa_iga *h, int32_t path) {
  if (path < 0 || path >= (int32_t)h->paths.size()) throw sa::SaError{SA_ERANGE, "path index out of range"};
  return path;
}

constexpr uint64_t kMagic = 0x5341494741434b33ull;  // checkpoint tag (with the audit state)

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// n_steps steps of every live path, overlapped where the object allows it;
// returns when they are complete (the status records checked)
void run_steps(sa_iga *h, int32_t n_steps) {
  struct InStep {
    sa_iga *h;
    explicit InStep(sa_iga *h_) : h(h_) { h->in_step = true; }
    ~InStep() { h->in_step = false; }
  };
  {
    InStep guard(h);
    if (h->overlap) {
      // the source side starts after everything queued so far
      hip_check(hipEventRecord(h->ev_start, h->stream), "event record");
      hip_check(hipStreamWaitEvent(h->ss, h->ev_start, 0), "stream wait");
      hip_check(hipStreamWaitEvent(h->ps, h->ev_start, 0), "stream wait");
      std::fill(h->path_rhs.begin(), h->path_rhs.end(), -1);
    }
    const auto t0 = std::chrono::steady_clock::now();
    // a call of one path (or a few at one step parity) runs in blocks of up
    // to kBlockSlots / paths steps
    std::vector<int> live;
    int64_t rem = INT64_MAX;
    for (int p = 0; p < (int)h->paths.size(); ++p)
      if (h->paths[p].step < h->paths[p].n_steps) live.push_back(p);
    bool blocked = h->blk_ok && h->pcg_budget == 1 && !live.empty() && 2 * (int)live.size() <= h->blk_steps;
    for (int p : live) blocked = blocked && (h->paths[p].step & 1) == (h->paths[live[0]].step & 1);
    for (int32_t s = 0; s < n_steps;) {
      if (!blocked) {
        step_all(h);
        ++s;
        continue;
      }
      live.clear();
      rem = INT64_MAX;
      for (int p = 0; p < (int)h->paths.size(); ++p)
        if (h->paths[p].step < h->paths[p].n_steps) {
          live.push_back(p);
          rem = std::min<int64_t>(rem, h->paths[p].n_steps - h->paths[p].step);
        }
      if (live.empty()) break;
      const int K = (int)std::min<int64_t>({rem, (int64_t)(n_steps - s), (int64_t)(h->blk_steps / (int)live.size())});
      step_block(h, live, K);
      s += K;
    }
    flush_checks(h);
    h->stats.host_enqueue_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (h->verbose && n_steps > 0) {
      const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
      std::fprintf(stderr,
                   "[sa_iga] %d steps enqueued in %.1f us per step (slots %.1f, sum %.1f, load+Dirichlet %.1f, "
                   "rhs %.1f, solve %.1f)\n",
                   n_steps, us / n_steps, h->host_us[0] / n_steps, h->host_us[1] / n_steps,
                   h->host_us[2] / n_steps, h->host_us[3] / n_steps, h->host_us[4] / n_steps);
      for (double &x : h->host_us) x = 0.0;
    }
    if (h->overlap) {
      hip_check(hipEventRecord(h->ev_end, h->ss), "event record");
      hip_check(hipStreamWaitEvent(h->stream, h->ev_end, 0), "stream wait");
      hip_check(hipEventRecord(h->ev_end, h->ps), "event record");
      hip_check(hipStreamWaitEvent(h->stream, h->ev_end, 0), "stream wait");
    }
  }
  check_statuses(h);
  sync_all(h);
  collect_timing(h);
}

// after a failed run_steps: drain the streams, drop pending records
void abandon_steps(sa_iga *h);

// the per-path state a call changes: kept on the device while the steps run
// with one PCG iteration
struct HostState {
  std::vector<int64_t> steps;
  sa_stats stats{};
  std::vector<uint8_t> use_exact;
  std::vector<int64_t> next_audit;
};

void save_state(sa_iga *h, HostState &c) {
  const size_t S = (size_t)h->S, nd = (size_t)h->nd, nDa = (size_t)h->nDa;
  double *src[5] = {h->V[0], h->V[1], h->Fb[0], h->Fb[1], h->vD};
  const size_t n[5] = {S * nd, S * nd, S * nd, S * nd, S * nDa};
  if (h->ckpt.empty())
    for (int b = 0; b < 5; ++b) h->ckpt.push_back(dev_alloc<double>(h->owned, n[b]));
  for (int b = 0; b < 5; ++b)
    hip_check(hipMemcpyAsync(h->ckpt[b], src[b], n[b] * sizeof(double), hipMemcpyDeviceToDevice, h->stream), "copy");
  c.steps.resize(h->paths.size());
  for (size_t p = 0; p < h->paths.size(); ++p) c.steps[p] = h->paths[p].step;
  c.stats = h->stats;
  c.use_exact = h->use_exact;
  c.next_audit = h->next_audit;
}

void restore_state(sa_iga *h, const HostState &c) {
  const size_t S = (size_t)h->S, nd = (size_t)h->nd, nDa = (size_t)h->nDa;
  double *dst[5] = {h->V[0], h->V[1], h->Fb[0], h->Fb[1], h->vD};
  const size_t n[5] = {S * nd, S * nd, S * nd, S * nd, S * nDa};
  for (int b = 0; b < 5; ++b)
    hip_check(hipMemcpyAsync(dst[b], h->ckpt[b], n[b] * sizeof(double), hipMemcpyDeviceToDevice, h->stream), "copy");
  hip_check(hipStreamSynchronize(h->stream), "sync");
  for (size_t p = 0; p < h->paths.size(); ++p) h->paths[p].step = c.steps[p];
  h->stats = c.stats;
  h->use_exact = c.use_exact;
  h->next_audit = c.next_audit;
  std::fill(h->chk_pending.begin(), h->chk_pending.end(), 0);
}

// run_steps with one PCG iteration per theta-step where that is the budget;
// if a step needed more, the state goes back to the call's start and the
// steps run again with two
void run_steps_checked(sa_iga *h, int32_t n_steps) {
  if (!(h->fd_exact && h->pcg_budget == 1) || n_steps <= 0) {
    run_steps(h, n_steps);
    return;
  }
  HostState c;
  save_state(h, c);
  try {
    run_steps(h, n_steps);
  } catch (const BudgetExceeded &) {
    abandon_steps(h);
    restore_state(h, c);
    h->pcg_budget = 2;
    h->force_rollback = false;
    h->stats.rollbacks++;
    run_steps(h, n_steps);
  }
}

void abandon_steps(sa_iga *h) {
  if (h->ss) (void)hipStreamSynchronize(h->ss);
  if (h->ps) (void)hipStreamSynchronize(h->ps);
  (void)hipStreamSynchronize(h->stream);
  h->status_kind.clear();
  std::fill(h->chk_pending.begin(), h->chk_pending.end(), 0);
  try {
    collect_timing(h);
  } catch (...) {
  }
}

extern "C" {

int sa_iga_default_options(sa_solver_options *opt) {
  if (!opt) return set_error(SA_EINVAL, "NULL options");
  std::memset(opt, 0, sizeof(*opt));
  opt->theta = 0.5;
  opt->kernel_scale = 1.0;
  opt->precision = SA_PREC_FP64;
  opt->tau_near = 2e-4;
  opt->pcg_rtol = 1e-13;
  opt->pcg_max_iter = 2000;
  opt->preconditioner = SA_PRECOND_FD;
  opt->audit_every = 50;
  opt->audit_frac = 0.01;
  opt->audit_tol = 0.5;
  return SA_OK;
}

int sa_iga_setup(const sa_patch *patch, const sa_material *mat, const sa_scan_path *scan, sa_iga **out) {
  if (out) *out = nullptr;
  return guarded([&]() -> int {
    if (!out) throw sa::SaError{SA_EINVAL, "NULL output pointer"};
    sa_solver_options opt;
    sa_iga_default_options(&opt);
    if (scan && scan->opt) opt = *scan->opt;
    sa::validate_inputs(patch, mat, scan, opt);
    std::unique_ptr<sa_iga> h(new sa_iga());
    h->m.opt = opt;
    build_object(h.get(), patch, mat, scan);
    *out = h.release();
    return SA_OK;
  });
}

int sa_iga_step(sa_iga *h, int32_t n_steps) {
  return guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    if (n_steps < 0) throw sa::SaError{SA_EINVAL, "n_steps must be >= 0"};
    if (h->sticky) throw sa::SaError{SA_ESTATE, "object is in an error state (load a checkpoint)"};
    try {
      run_steps_checked(h, n_steps);
    } catch (const sa::SaError &e) {
      if (e.code == SA_ENOCONV) h->sticky = 1;
      abandon_steps(h);
      throw;
    }
    return SA_OK;
  });
}

int sa_iga_get_step(sa_iga *h, int32_t path, int64_t *step) {
  return guarded([&]() -> int {
    if (!h || !step) throw sa::SaError{SA_EINVAL, "NULL argument"};
    *step = h->paths[path_index(h, path)].step;
    return SA_OK;
  });
}

int sa_iga_eval_source_field(sa_iga *h, int32_t path, int64_t step, int64_t n, const double *x, double *T,
                             double *grad) {
  return guarded([&]() -> int {
    if (!h || (n > 0 && (!x || !T))) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (n < 0 || step < 0) throw sa::SaError{SA_EINVAL, "negative size or step"};
    source_field_host(h, path_index(h, path), step, n, x, T, grad);
    return SA_OK;
  });
}

int sa_iga_eval_source_field_noalloc(sa_iga *h, int32_t path, int64_t step, int64_t n, const double *x, double *T,
                                     double *grad) {
  return guarded([&]() -> int {
    if (!h || (n > 0 && (!x || !T))) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (n < 0 || step < 0) throw sa::SaError{SA_EINVAL, "negative size or step"};
    if (n > sa::kNoAllocMaxPoints) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "%lld points: the allocation-free evaluation takes at most %lld per call",
                    (long long)n, (long long)sa::kNoAllocMaxPoints);
      throw sa::SaError{SA_EINVAL, msg};
    }
    const int p = path_index(h, path);
    if (n == 0) return SA_OK;
    if (!h->scratch) throw sa::SaError{SA_EDEVICE, "the device scratch area is not available"};
    source_field_noalloc(h, p, step, n, x, T, grad);
    return SA_OK;
  });
}

int sa_iga_heat_loss(sa_iga *h, int32_t path, int32_t face, int32_t edge_face, int32_t quad, int64_t *n_pts,
                     double *x, double *normal, double *ds, double *q_tilde, double *q_hat, double *integrals) {
  return guarded([&]() -> int {
    if (!h || !n_pts) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (face < 0 || face > 5 || edge_face < 0 || edge_face > 5 || face / 2 == edge_face / 2)
      throw sa::SaError{SA_EINVAL, "face and edge_face must be parametric faces 0..5 that meet along an edge"};
    if (quad < 1 || quad > 16) throw sa::SaError{SA_EINVAL, "quad must be 1..16"};
    const int p = path_index(h, path);
    const sa::PatchData &P = h->m.P;
    const int d = face / 2, de = edge_face / 2, e = 3 - d - de;
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
    EvalTables t = eval_tables(P, n, xi.data());
    const hipStream_t st = h->stream;
    TempBufs tb;
    double *dT = nullptr, *dG = nullptr;
    const int64_t gs = source_field_dev(h, tb, p, h->paths[p].step, n, t.x.data(), &dT, &dG);
    int64_t *rp = tb.up(t.rowptr, st);
    int32_t *cl = tb.up(t.col, st);
    double *gx = tb.up(t.gx, st), *gy = tb.up(t.gy, st), *gz = tb.up(t.gz, st);
    double *dn = tb.up(nrm, st), *dds = tb.up(dsv, st);
    double *out = tb.alloc<double>((size_t)4 * n + 2);
    sa::launch_heat_loss(st, n, rp, cl, gx, gy, gz, path_v(h, p), dG, gs, dn, dds, h->m.mat.k, out, out + n,
                         out + 2 * n, out + 3 * n, out + 4 * n);
    hip_check(hipGetLastError(), "kernel launch");
    std::vector<double> hv((size_t)4 * n + 2);
    hip_check(hipMemcpyAsync(hv.data(), out, hv.size() * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    hip_check(hipStreamSynchronize(st), "sync");
    if (x) std::memcpy(x, t.x.data(), (size_t)3 * n * sizeof(double));
    if (normal) std::memcpy(normal, nrm.data(), (size_t)3 * n * sizeof(double));
    if (ds) std::memcpy(ds, dsv.data(), (size_t)n * sizeof(double));
    if (q_tilde) std::memcpy(q_tilde, hv.data(), (size_t)n * sizeof(double));
    if (q_hat) std::memcpy(q_hat, hv.data() + n, (size_t)n * sizeof(double));
    if (integrals) {
      integrals[0] = hv[(size_t)4 * n];
      integrals[1] = hv[(size_t)4 * n + 1];
    }
    *n_pts = n;
    return SA_OK;
  });
}

int sa_iga_eval_temperature_at(sa_iga *h, int32_t path, int64_t n, const double *x, double *T, double *gradT,
                               double *xi_out) {
  return guarded([&]() -> int {
    if (!h || (n > 0 && (!x || !T))) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (n < 0) throw sa::SaError{SA_EINVAL, "negative size"};
    const int p = path_index(h, path);
    if (n == 0) return SA_OK;
    const sa::PatchData &P = h->m.P;
    // element centres (parametric and physical), built once per object
    if (h->el_centre.empty()) sa::element_centres(P, h->el_centre, h->el_xi);
    const double tol = sa::locate_tolerance(P);
    std::vector<double> xi((size_t)3 * n);
    std::vector<int64_t> inside;
    std::vector<double> xin;
    for (int64_t i = 0; i < n; ++i) {
      if (sa::locate_point(P, h->el_centre, h->el_xi, x + 3 * i, tol, &xi[3 * i])) {
        inside.push_back(i);
        for (int c = 0; c < 3; ++c) xin.push_back(xi[3 * i + c]);
      } else {
        for (int c = 0; c < 3; ++c) xi[3 * i + c] = NAN;
      }
    }
    const int64_t m = (int64_t)inside.size();
    std::vector<double> Ti((size_t)m), Gi((size_t)3 * m);
    if (m > 0) {
      const int rc = sa_iga_eval_temperature(h, p, m, xin.data(), Ti.data(), Gi.data());
      if (rc != SA_OK) throw sa::SaError{rc, sa_iga_last_error()};
    }
    for (int64_t i = 0; i < n; ++i) {
      T[i] = NAN;
      if (gradT)
        for (int c = 0; c < 3; ++c) gradT[3 * i + c] = NAN;
    }
    for (int64_t k = 0; k < m; ++k) {
      const int64_t i = inside[k];
      T[i] = Ti[k];
      if (gradT)
        for (int c = 0; c < 3; ++c) gradT[3 * i + c] = Gi[3 * k + c];
    }
    if (xi_out) std::memcpy(xi_out, xi.data(), xi.size() * sizeof(double));
    return SA_OK;
  });
}

int sa_iga_eval_temperature(sa_iga *h, int32_t path, int64_t n, const double *xi, double *T, double *gradT) {
  return guarded([&]() -> int {
    if (!h || (n > 0 && (!xi || !T))) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (n < 0) throw sa::SaError{SA_EINVAL, "negative size"};
    const int p = path_index(h, path);
    if (n == 0) return SA_OK;
    EvalTables t = eval_tables(h->m.P, n, xi);
    std::vector<double> Tt(n), Gt(3 * n);
    source_field_host(h, p, h->paths[p].step, n, t.x.data(), Tt.data(), Gt.data());
    TempBufs tb;
    int64_t *rp = tb.up(t.rowptr, h->stream);
    int32_t *cl = tb.up(t.col, h->stream);
    double *vals[4] = {tb.up(t.R, h->stream), tb.up(t.gx, h->stream), tb.up(t.gy, h->stream), tb.up(t.gz, h->stream)};
    double *out = tb.alloc<double>(4 * n);
    for (int k = 0; k < 4; ++k) sa::launch_csr_eval(h->stream, n, rp, cl, vals[k], path_v(h, p), out + k * n);
    std::vector<double> hv(4 * n);
    hip_check(hipMemcpyAsync(hv.data(), out, 4 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream), "download");
    hip_check(hipStreamSynchronize(h->stream), "sync");
    for (int64_t i = 0; i < n; ++i) {
      T[i] = h->m.mat.T0 + hv[i] + Tt[i];
      if (gradT)
        for (int c = 0; c < 3; ++c) gradT[3 * i + c] = hv[(c + 1) * n + i] + Gt[c * n + i];
    }
    return SA_OK;
  });
}

int sa_iga_get_boundary_fields(sa_iga *h, int32_t path, double *T_gp, double *grad_gp, double *F, double *du) {
  return guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    const int p = path_index(h, path);
    const int64_t nq = h->nq, nd = h->nd;
    if (T_gp) hip_check(hipMemcpyAsync(T_gp, path_T(h, p), nq * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                        "download");
    if (grad_gp)
      for (int c = 0; c < 3; ++c)
        hip_check(hipMemcpyAsync(grad_gp + c * nq, path_G(h, p) + c * h->stride, nq * sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream),
                  "download");
    if (F) hip_check(hipMemcpyAsync(F, path_F(h, p), nd * sizeof(double), hipMemcpyDeviceToHost, h->stream), "download");
    if (du) hip_check(hipMemcpyAsync(du, path_v(h, p), nd * sizeof(double), hipMemcpyDeviceToHost, h->stream), "download");
    hip_check(hipStreamSynchronize(h->stream), "sync");
    return SA_OK;
  });
}

int sa_iga_eval_temperature_device(sa_iga *h, int32_t path, int64_t n, const double *xi, double *T,
                                   double *gradT) {
  return guarded([&]() -> int {
    if (!h || (n > 0 && (!xi || !T))) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (n < 0) throw sa::SaError{SA_EINVAL, "negative size"};
    const int p = path_index(h, path);
    if (n == 0) return SA_OK;
    const sa::GeoDev &g = geometry_on_device(h);
    sa::PathTab tab{};
    tab.count = 1;
    fill_slot(h, tab, 0, p, h->paths[p].step);
    const sa::SumPlan pl = query_plan(h, tab, n, 0);
    const int nch = std::max(pl.n_chunks_far + pl.n_chunks_near, 1);
    const size_t sum_bytes = sa::noalloc_layout(nullptr, n, nch).bytes;
    // after the sum's area: x [n][3], Th [n], Gh [3][n], Tt [n], Gt [3][n]
    const size_t vec = ((size_t)n * sizeof(double) + 255) / 256 * 256;
    unsigned char *base = (unsigned char *)query_workspace(h, sum_bytes + 11 * vec);
    const sa::NoAllocLayout L = sa::noalloc_layout(base, n, nch);
    double *x = (double *)(base + sum_bytes), *Th = (double *)(base + sum_bytes + 3 * vec),
           *Gh = (double *)(base + sum_bytes + 4 * vec), *Tt = (double *)(base + sum_bytes + 7 * vec),
           *Gt = (double *)(base + sum_bytes + 8 * vec);
    sa::launch_eval_hat(h->stream, n, xi, g, path_v(h, p), x, Th, Gh);
    source_field_in(h, tab, pl, n, x, Tt, Gt, L);
    sa::launch_eval_combine(h->stream, n, h->m.mat.T0, Th, Gh, Tt, Gt, T, gradT);
    hip_check(hipGetLastError(), "kernel launch");
    return SA_OK;
  });
}

int sa_iga_get_boundary_fields_device(sa_iga *h, int32_t path, double *T_gp, double *grad_gp, double *F,
                                      double *du) {
  return guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    const int p = path_index(h, path);
    const int64_t nq = h->nq, nd = h->nd;
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (T_gp) hip_check(hipMemcpyAsync(T_gp, path_T(h, p), nq * sizeof(double), k, h->stream), "copy");
    if (grad_gp)
      for (int c = 0; c < 3; ++c)
        hip_check(hipMemcpyAsync(grad_gp + c * nq, path_G(h, p) + c * h->stride, nq * sizeof(double), k, h->stream),
                  "copy");
    if (F) hip_check(hipMemcpyAsync(F, path_F(h, p), nd * sizeof(double), k, h->stream), "copy");
    if (du) hip_check(hipMemcpyAsync(du, path_v(h, p), nd * sizeof(double), k, h->stream), "copy");
    return SA_OK;
  });
}

int sa_iga_get_boundary_points(sa_iga *h, double *x, double *normal, double *wdS) {
  return guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    const auto &bt = h->m.bt;
    if (x) std::memcpy(x, bt.x.data(), bt.x.size() * sizeof(double));
    if (normal) std::memcpy(normal, bt.nrm.data(), bt.nrm.size() * sizeof(double));
    if (wdS) std::memcpy(wdS, bt.wdS.data(), bt.wdS.size() * sizeof(double));
    return SA_OK;
  });
}

int sa_iga_apply_operator(sa_iga *h, int32_t which, const double *x, double *y) {
  return guarded([&]() -> int {
    if (!h || !x || !y) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (which == 0) h->m.M.apply(x, y);
    else if (which == 1) h->m.K.apply(x, y);
    else throw sa::SaError{SA_EINVAL, "which must be 0 (M) or 1 (K)"};
    return SA_OK;
  });
}

int sa_iga_autotune(sa_iga *h, int32_t reps, int32_t *points_per_lane, int32_t *waves_per_group,
                    double *ms_per_step) {
  return guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    if (reps < 1) throw sa::SaError{SA_EINVAL, "reps must be >= 1"};
    if (h->sticky) throw sa::SaError{SA_ESTATE, "object is in an error state (load a checkpoint)"};
    auto &o = h->m.opt;
    bool any = false;
    for (const PathState &P : h->paths) any = any || (P.n_steps > 1 && P.src1 > P.src0);
    double best_ms = 0.0;
    if (any) {
      // the state the trial steps overwrite, kept on the device
      const int S = h->S;
      const int64_t nd = h->nd;
      struct Saved {
        double *dst;
        size_t n;
      };
      const Saved arr[] = {{h->V[0], (size_t)S * nd},        {h->V[1], (size_t)S * nd},
                           {h->Fb[0], (size_t)S * nd},       {h->Fb[1], (size_t)S * nd},
                           {h->vD, (size_t)S * h->nDa},      {h->Tb, (size_t)S * h->stride},
                           {h->Gb, (size_t)S * 3 * h->stride}, {h->LD, (size_t)S * h->stride}};
      TempBufs tb;
      std::vector<double *> keep;
      for (const Saved &a : arr) {
        double *c = tb.alloc<double>(a.n);
        hip_check(hipMemcpyAsync(c, a.dst, a.n * sizeof(double), hipMemcpyDeviceToDevice, h->stream), "copy");
        keep.push_back(c);
      }
      std::vector<int64_t> steps(S);
      for (int p = 0; p < S; ++p) steps[p] = h->paths[p].step;
      const sa_stats stats = h->stats;
      const std::vector<uint8_t> use_exact = h->use_exact;
      const std::vector<int64_t> next_audit = h->next_audit;
      const int keep_timing = o.timing;
      auto restore = [&]() {
        for (int p = 0; p < S; ++p) h->paths[p].step = steps[p];
        h->stats = stats;
        h->use_exact = use_exact;
        h->next_audit = next_audit;
        o.timing = keep_timing;
        for (size_t k = 0; k < keep.size(); ++k)
          hip_check(hipMemcpyAsync(arr[k].dst, keep[k], arr[k].n * sizeof(double), hipMemcpyDeviceToDevice,
                                   h->stream),
                    "copy");
        hip_check(hipStreamSynchronize(h->stream), "sync");
      };
      // every shape runs one untimed and `reps` timed steps of all paths
      // from the middle of their scans, through the whole step pipeline
      static const int kP[3] = {1, 2, 4}, kW[4] = {1, 2, 4, 8};
      double best = -1.0;
      int bp = 2, bw = 4;
      o.timing = 0;
      // with every boundary point on a tensor face the pair-by-pair kernel
      // does not run: one shape is timed, for the time per step
      const bool moot = h->use_tensor && h->n_gen == 0;
      try {
        for (int P : kP)
          for (int w : kW) {
            if (moot && (P != bp || w != bw)) continue;
            o.points_per_lane = P;
            o.waves_per_group = w;
            for (int p = 0; p < S; ++p)
              h->paths[p].step = std::max<int64_t>(0, h->paths[p].n_steps / 2 - 1 - reps);
            run_steps_checked(h, 1);
            const auto t0 = std::chrono::steady_clock::now();
            run_steps_checked(h, reps);
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (best < 0 || ms < best) {
              best = ms;
              bp = P;
              bw = w;
            }
          }
        o.points_per_lane = bp;
        o.waves_per_group = bw;
        // the matrix-core sum's launch shape (tensor faces): for launches of
        // four paths or more the workgroups per compute unit of its grid;
        // for a blocked call its LDS padding (how many of its workgroups
        // share a compute unit with the solver kernels beside it) and the
        // block length.  Neither changes how the histories are chunked, so
        // results stay bitwise the same.
        if (h->use_tensor && S >= 4) {
          // workgroups per compute unit, then the LDS padding that leaves
          // compute units to the theta-step kernels beside the sum
          static const int kG[4] = {8, 4, 6, 12}, kBp[3] = {10000, 0, 38000};
          int bg = h->sum_groups_per_cu_batch, bbp = h->tens.lds_pad;
          double bt = -1.0, base = -1.0;
          auto time_shape = [&]() {
            for (int p = 0; p < S; ++p)
              h->paths[p].step = std::max<int64_t>(0, h->paths[p].n_steps / 2 - 1 - reps);
            run_steps_checked(h, 1);
            const auto t0 = std::chrono::steady_clock::now();
            run_steps_checked(h, reps);
            return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
          };
          for (int g : kG) {
            h->tens.max_groups_batch = g * h->n_cu;
            const double ms = time_shape();
            if (base < 0) {
              base = bt = ms;
              bg = g;
            } else if (ms < 0.97 * base && ms < bt) {
              bt = ms;
              bg = g;
            }
          }
          h->tens.max_groups_batch = bg * h->n_cu;
          const double base_g = bt;
          for (int pad : kBp) {
            if (pad == bbp || !sa::sum_tensor_prepare(pad)) continue;
            h->tens.lds_pad = pad;
            const double ms = time_shape();
            if (ms < 0.97 * base_g && ms < bt) {
              bt = ms;
              bbp = pad;
            }
          }
          h->sum_groups_per_cu_batch = bg;
          h->tens.lds_pad = bbp;
          best = bt;
        }
        if (h->use_tensor && h->blk_ok && S <= 4) {
          // short blocked steps time noisily, and the sum's share of a step
          // grows along a scan: each shape is timed at a quarter, half and
          // three quarters of every path's scan, the better of two runs of
          // 48 steps at each, and the set-up shape (the first) is left only
          // for one at least 3 % faster
          static const int kPad[3] = {0, 10000, 38000}, kBs[2] = {8, 4};
          const int rb = std::max(reps, 48);
          int bpad = h->blk_pad, bbs = h->blk_steps;
          double bt = -1.0, base = -1.0;
          const bool big_pad = sa::sum_tensor_prepare(38000);
          for (int pad : kPad)
            for (int bs : kBs) {
              if ((pad > 0 && !big_pad) || 2 * S > bs) continue;
              h->blk_pad = pad;
              h->blk_steps = bs;
              double ms = 0.0;
              for (int q = 1; q <= 3; ++q) {
                double mq = -1.0;
                for (int rep = 0; rep < 2; ++rep) {
                  for (int p = 0; p < S; ++p)
                    h->paths[p].step = std::max<int64_t>(0, h->paths[p].n_steps * q / 4 - 1 - rb);
                  run_steps_checked(h, bs);
                  const auto t0 = std::chrono::steady_clock::now();
                  run_steps_checked(h, rb);
                  const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                                       .count() * reps / rb;
                  mq = mq < 0 ? t : std::min(mq, t);
                }
                ms += mq / 3.0;
              }
              if (base < 0) {
                base = bt = ms;
                bpad = pad;
                bbs = bs;
              } else if (ms < 0.97 * base && ms < bt) {
                bt = ms;
                bpad = pad;
                bbs = bs;
              }
            }
          if (bt >= 0) {
            h->blk_pad = bpad;
            h->blk_steps = bbs;
            best = bt;
          }
        }
      } catch (...) {
        abandon_steps(h);
        restore();
        throw;
      }
      restore();
      best_ms = best / reps;
    }
    if (points_per_lane) *points_per_lane = o.points_per_lane ? o.points_per_lane : 2;
    if (waves_per_group) *waves_per_group = o.waves_per_group ? o.waves_per_group : 4;
    if (ms_per_step) *ms_per_step = best_ms;
    return SA_OK;
  });
}

int sa_iga_set_timing(sa_iga *h, int32_t on) {
  return guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    h->m.opt.timing = on ? 1 : 0;
    return SA_OK;
  });
}

int sa_iga_get_info(sa_iga *h, sa_info *info) {
  return guarded([&]() -> int {
    if (!h || !info) throw sa::SaError{SA_EINVAL, "NULL argument"};
    std::memset(info, 0, sizeof(*info));
    for (int d = 0; d < 3; ++d) info->n_ctrl[d] = h->m.P.n[d];
    info->n_dof = h->nd;
    info->n_bpts = h->nq;
    for (int f = 0; f < 7; ++f) info->face_offset[f] = h->m.bt.face_off[f];
    info->n_paths = (int32_t)h->paths.size();
    info->n_sources = (int64_t)h->h_tick.size();
    info->blocked_steps = h->blk_ok ? h->blk_steps : 1;
    info->sum_groups_per_cu_batch = h->use_tensor ? h->sum_groups_per_cu_batch : 0;
    info->block_lds_pad = h->blk_ok ? h->blk_pad : 0;
    info->batch_lds_pad = h->use_tensor ? h->tens.lds_pad : 0;
    info->n_dirichlet = h->nD;
    info->tensor_faces = h->use_tensor ? h->n_tfaces : 0;
    info->generic_points = h->use_tensor ? h->n_gen : h->nq;
    return SA_OK;
  });
}

int sa_iga_get_stats(sa_iga *h, sa_stats *stats) {
  return guarded([&]() -> int {
    if (!h || !stats) throw sa::SaError{SA_EINVAL, "NULL argument"};
    *stats = h->stats;
    return SA_OK;
  });
}

int sa_iga_reset_stats(sa_iga *h) {
  return guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    h->stats = sa_stats{};
    return SA_OK;
  });
}

int sa_iga_save(sa_iga *h, void *buf, size_t *len) {
  return guarded([&]() -> int {
    if (!h || !len) throw sa::SaError{SA_EINVAL, "NULL argument"};
    const int64_t nd = h->nd, nDa = h->nDa, nq = h->nq;
    const size_t per = 3 * sizeof(int64_t) + (2 * nd + nDa + 4 * nq) * sizeof(double);
    const size_t need = 4 * sizeof(uint64_t) + h->paths.size() * per;
    if (!buf) {
      *len = need;
      return SA_OK;
    }
    if (*len < need) throw sa::SaError{SA_EINVAL, "checkpoint buffer too small"};
    char *b = (char *)buf;
    uint64_t hdr[4] = {kMagic, (uint64_t)h->paths.size(), (uint64_t)nd, (uint64_t)nDa};
    std::memcpy(b, hdr, sizeof(hdr));
    b += sizeof(hdr);
    for (int p = 0; p < (int)h->paths.size(); ++p) {
      // step, then the surrogate form's audit state (1, -1 without a network)
      const int64_t rec[3] = {h->paths[p].step, h->net ? (int64_t)h->use_exact[p] : 1,
                              h->net ? h->next_audit[p] : -1};
      std::memcpy(b, rec, sizeof(rec));
      b += sizeof(rec);
      hip_check(hipMemcpyAsync(b, path_v(h, p), nd * sizeof(double), hipMemcpyDeviceToHost, h->stream), "download");
      b += nd * sizeof(double);
      hip_check(hipMemcpyAsync(b, path_F(h, p), nd * sizeof(double), hipMemcpyDeviceToHost, h->stream), "download");
      b += nd * sizeof(double);
      hip_check(hipMemcpyAsync(b, path_vD(h, p), nDa * sizeof(double), hipMemcpyDeviceToHost, h->stream), "download");
      b += nDa * sizeof(double);
      hip_check(hipMemcpyAsync(b, path_T(h, p), nq * sizeof(double), hipMemcpyDeviceToHost, h->stream), "download");
      b += nq * sizeof(double);
      for (int c = 0; c < 3; ++c) {
        hip_check(hipMemcpyAsync(b, path_G(h, p) + c * h->stride, nq * sizeof(double), hipMemcpyDeviceToHost,
                                 h->stream),
                  "download");
        b += nq * sizeof(double);
      }
    }
    hip_check(hipStreamSynchronize(h->stream), "sync");
    *len = need;
    return SA_OK;
  });
}

int sa_iga_load(sa_iga *h, const void *buf, size_t len) {
  return guarded([&]() -> int {
    if (!h || !buf) throw sa::SaError{SA_EINVAL, "NULL argument"};
    const int64_t nd = h->nd, nDa = h->nDa, nq = h->nq;
    const size_t per = 3 * sizeof(int64_t) + (2 * nd + nDa + 4 * nq) * sizeof(double);
    const size_t need = 4 * sizeof(uint64_t) + h->paths.size() * per;
    if (len < need) throw sa::SaError{SA_EINVAL, "checkpoint too short"};
    const char *b = (const char *)buf;
    uint64_t hdr[4];
    std::memcpy(hdr, b, sizeof(hdr));
    if (hdr[0] != kMagic || hdr[1] != h->paths.size() || hdr[2] != (uint64_t)nd || hdr[3] != (uint64_t)nDa)
      throw sa::SaError{SA_EINVAL, "checkpoint does not match this object"};
    b += sizeof(hdr);
    for (auto &P : h->paths) {
      int64_t rec[3];
      std::memcpy(rec, b, sizeof(rec));
      if (rec[0] < 0 || rec[0] > P.n_steps) throw sa::SaError{SA_EINVAL, "checkpoint step out of range"};
      if ((rec[1] != 0 && rec[1] != 1) || rec[2] < -1) throw sa::SaError{SA_EINVAL, "checkpoint audit state invalid"};
      b += per;
    }
    b = (const char *)buf + sizeof(hdr);
    for (int p = 0; p < (int)h->paths.size(); ++p) {
      int64_t rec[3];
      std::memcpy(rec, b, sizeof(rec));
      b += sizeof(rec);
      h->paths[p].step = rec[0];
      if (h->net) {
        h->use_exact[p] = (uint8_t)rec[1];
        h->next_audit[p] = rec[2];
      }
      hip_check(hipMemcpyAsync(path_v(h, p), b, nd * sizeof(double), hipMemcpyHostToDevice, h->stream), "upload");
      b += nd * sizeof(double);
      hip_check(hipMemcpyAsync(path_F(h, p), b, nd * sizeof(double), hipMemcpyHostToDevice, h->stream), "upload");
      b += nd * sizeof(double);
      hip_check(hipMemcpyAsync(path_vD(h, p), b, nDa * sizeof(double), hipMemcpyHostToDevice, h->stream), "upload");
      b += nDa * sizeof(double);
      hip_check(hipMemcpyAsync(path_T(h, p), b, nq * sizeof(double), hipMemcpyHostToDevice, h->stream), "upload");
      b += nq * sizeof(double);
      for (int c = 0; c < 3; ++c) {
        hip_check(hipMemcpyAsync(path_G(h, p) + c * h->stride, b, nq * sizeof(double), hipMemcpyHostToDevice,
                                 h->stream),
                  "upload");
        b += nq * sizeof(double);
      }
    }
    hip_check(hipStreamSynchronize(h->stream), "sync");
    h->sticky = 0;
    return SA_OK;
  });
}

int sa_iga_far_field(sa_iga *h, int32_t path, int64_t step, double e_scale, float *X, double *T, double *grad) {
  return guarded([&]() -> int {
    if (!h || !T || !grad) throw sa::SaError{SA_EINVAL, "NULL argument"};
    if (step < 0) throw sa::SaError{SA_EINVAL, "negative step"};
    if (!(e_scale > 0) || !std::isfinite(e_scale)) throw sa::SaError{SA_EINVAL, "e_scale must be positive"};
    const int p = path_index(h, path);
    const PathState &P = h->paths[p];
    const int64_t now = step * h->ns;
    auto b = h->h_tick.begin() + P.src0, e = h->h_tick.begin() + P.src1;
    const int64_t a = (int64_t)(std::upper_bound(b, e, now) - b);
    const int64_t f = std::min<int64_t>(a, (int64_t)(std::lower_bound(b, b + a, now - h->tau_ticks) - b));
    sa::PathTab ex{};
    ex.count = 1;
    ex.path[0] = p;
    ex.src0[0] = P.src0;
    ex.now[0] = now;
    ex.n_act[0] = (int32_t)f;                 // the far sources, all in FP64
    ex.n_far[0] = 0;
    ex.mode[0] = 0;
    const sa_stats keep = h->stats;
    // T and grad written directly in the caller's layout (slot 0, stride n_bpts)
    sum_points(h, ex, h->nq, h->stride, h->px, h->py, h->pz, h->pq2, h->fx, h->fy, h->fz, h->fq2, h->role,
               h->nx, h->ny, h->nz, h->wdS, true, h->nq, T, grad, h->LD, nullptr, 0, nullptr, true);
    h->stats.pairs = keep.pairs;
    h->stats.pairs_near = keep.pairs_near;
    if (X) {
      sa::PathTab ft = ex;
      ft.n_far[0] = (int32_t)f;
      sa::launch_far_bins(h->stream, ft, h->sbin, h->sE, e_scale, h->bins);
      sa::launch_net_inputs(h->stream, h->nq, h->pf, h->bins, X);
    }
    hip_check(hipStreamSynchronize(h->stream), "sync");
    hip_check(hipGetLastError(), "kernel launch");
    return SA_OK;
  });
}

int sa_iga_set_stream(sa_iga *h, void *hip_stream) {
  return guarded([&]() -> int {
    if (!h) throw sa::SaError{SA_EINVAL, "NULL object"};
    sync_all(h);
    h->stream = hip_stream ? (hipStream_t)hip_stream : h->own_stream;
    return SA_OK;
  });
}

const char *sa_iga_last_error(void) { return g_last_error.c_str(); }

void sa_iga_destroy(sa_iga *h) { delete h; }

}  // extern "C"
