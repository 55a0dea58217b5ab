// gfx950 kernels of the semi-analytical IGA thermal model.
//
//  * k_coeff     per-step source coefficients (Eq. 8 with the finite-spot
//                shift): FP64 records for every active source, FP32 base-2
//                records for the far (old) ones.
//  * k_sum       the point-source superposition (Eq. 7) at the boundary
//                quadrature points.  Points live in lanes (P per lane),
//                sources are wave-uniform and stream through scalar loads;
//                each workgroup column sums one chunk of the source history.
//  * k_finalize  fixed-order reduction of the chunk partials, gradient, and
//                the per-point load densities of Eqs. 10-11 and 18.
//  * k_gather    transpose-CSR gathers (load vector, projection rhs).
//  * stencil / CSR operators, Jacobi and fast-diagonalisation
//                preconditioners and the PCG steps for the theta-scheme
//                (Eq. 20); every PCG kernel is a no-op once the device flag
//                says the solve has converged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "kernels.h"

namespace sa {

constexpr int kBlock = 256;
constexpr int kMaxParts = 1024;

int parts_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  return (int)(g > kMaxParts ? kMaxParts : g);
}

// ---------------------------------------------------------------------------
// FP64 exponential: Cody-Waite reduction a = k ln2 + r (|r| <= ln2/2, two-part
// ln2), degree-13 Taylor polynomial of e^r (truncation < 5e-18 relative),
// scaling by 2^k with ldexp (underflows to 0 below the subnormal range).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_f64(double a) {
  a = fmax(a, -1080.0);
  const double kInvLn2 = 1.4426950408889634;
  const double kShift = 6755399441055744.0;       // 1.5 * 2^52
  const double kLn2Hi = 6.93147180369123816490e-01;
  const double kLn2Lo = 1.90821492927058770002e-10;
  const double t = fma(a, kInvLn2, kShift);
  const double kf = t - kShift;
  double r = fma(kf, -kLn2Hi, a);
  r = fma(kf, -kLn2Lo, r);
  double p = 1.0 / 6227020800.0;                  // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  const int k = __double2loint(t);                 // low word of t holds rint(a / ln2)
  return __builtin_ldexp(p, k);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// sum over the block; every thread gets the result
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[kBlock / 64];
  __shared__ double tot;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    tot = s;
  }
  __syncthreads();
  return tot;
}

// fixed-order sum of partials[0..n) by one block
__device__ __forceinline__ double reduce_parts(const double *part, int n) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  return block_sum(s);
}

// ---------------------------------------------------------------------------
// source coefficients
// ---------------------------------------------------------------------------
__global__ void k_coeff(PathTab tab, const int64_t *__restrict__ tick, const double *__restrict__ sx,
                        const double *__restrict__ sy, const double *__restrict__ sz,
                        const double *__restrict__ E, CoeffParams cp, double *__restrict__ c64,
                        float *__restrict__ c32) {
  const int slot = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= tab.n_act[slot]) return;
  const int64_t i = tab.src0[slot] + j;
  const double D = (double)(tab.now[slot] - tick[i]) * cp.delta + cp.shift;
  const double c = -1.0 / (4.0 * cp.alpha * D);
  const double x = sx[i], y = sy[i], z = sz[i];
  const double amp = cp.scale * E[i] / (cp.rc * pow(4.0 * M_PI * cp.alpha * D, 1.5));
  const double K = c * (x * x + y * y + z * z) + log(amp);
  double *o = c64 + i * kCoefStride;
  o[0] = c;
  o[1] = -2.0 * c * x;
  o[2] = -2.0 * c * y;
  o[3] = -2.0 * c * z;
  o[4] = K;
  o[5] = log(amp);
  o[6] = 0.0;
  o[7] = 0.0;
  if (j < tab.n_far[slot]) {
    // FP32 record in base 2, relative to the origin o of its aligned block of
    // kTile32 sources (the block's first source, rounded to FP32): the
    // exponent c |x - o|^2 + u'.(x - o) + K' then cancels little for the
    // points near the block, where its terms matter
    const int64_t ib = tab.src0[slot] + (j & ~(int64_t)(kTile32 - 1));
    const float ofx = (float)sx[ib], ofy = (float)sy[ib], ofz = (float)sz[ib];
    const double rx = x - (double)ofx, ry = y - (double)ofy, rz = z - (double)ofz;
    const double l2e = 1.4426950408889634;
    float *f = c32 + i * kCoefStride;
    f[0] = (float)(c * l2e);
    f[1] = (float)(-2.0 * c * rx * l2e);
    f[2] = (float)(-2.0 * c * ry * l2e);
    f[3] = (float)(-2.0 * c * rz * l2e);
    f[4] = (float)((c * (rx * rx + ry * ry + rz * rz) + log(amp)) * l2e);
    f[5] = ofx;
    f[6] = ofy;
    f[7] = ofz;
  }
}

void launch_coeff(hipStream_t st, const PathTab &tab, int64_t max_act, const int64_t *tick, const double *sx,
                  const double *sy, const double *sz, const double *E, const CoeffParams &cp,
                  double *c64, float *c32) {
  if (max_act <= 0 || tab.count <= 0) return;
  dim3 g((unsigned)((max_act + kBlock - 1) / kBlock), (unsigned)tab.count);
  hipLaunchKernelGGL(k_coeff, g, dim3(kBlock), 0, st, tab, tick, sx, sy, sz, E, cp, c64, c32);
}

// ---------------------------------------------------------------------------
// kernel sum on tensor faces (matrix cores)
//
// On a face whose points form the grid (sa[a], sb[b], sn) along Cartesian
// axes, the Gaussian of Eq. 8 factorises over the axes:
//   A e^{c |x - x_i|^2} = L_i[b] R_i[a],  L = A e^{c (sb - x_ib)^2 + c (sn - x_in)^2},
//                                         R = e^{c (sa - x_ia)^2},
// and its gradient A e^{c r^2} 2c (x - x_i) has the components
//   along a: L (2c da R),  along b: (2c db L) R,  along n: (2c dn L) R.
// Over the sources of a chunk the four sums at the points of a 32 x 32 tile
// are therefore matrix products [b x i] [i x a] on the matrix cores, with the
// operands formed in the lanes (one exponential per row or column and source
// instead of one per pair), the chunk's sources staged in LDS 256 at a time.
// Far chunks: FP32 operands (coordinates relative to the tile) and
// accumulation over 128 sources, then FP64 (32 x 32 x 2 steps); near chunks:
// FP64 (16 x 16 x 4 steps).  The operand layouts are given at each kind of
// item (checked on the device).
// ---------------------------------------------------------------------------
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx16 __attribute__((ext_vector_type(16)));

constexpr int kStage = 256;   // sources staged in LDS at a time

// Shared by the two kinds of work item (tile, chunk, slot): the chunk's
// source range, the source arrays along the face's axes, and the loads of
// one source's data (coefficients and position), issued a block ahead.
struct ItemSrc {
  int slot, lo, hi;
  int64_t s0, now;
  const double *c64, *pa, *pb, *pn;
};

__device__ __forceinline__ ItemSrc item_sources(const TensorArgs &ta, const PathTab &tab, const TFace &F, int slot,
                                                int lo, int hi) {
  ItemSrc r;
  r.slot = slot;
  r.lo = lo;
  r.hi = hi;
  r.s0 = tab.src0[slot];
  r.now = tab.now[slot];
  r.c64 = ta.c64 + r.s0 * kCoefStride;
  r.pa = (F.ax_a == 0 ? ta.sx : (F.ax_a == 1 ? ta.sy : ta.sz)) + r.s0;
  r.pb = (F.ax_b == 0 ? ta.sx : (F.ax_b == 1 ? ta.sy : ta.sz)) + r.s0;
  r.pn = (F.ax_n == 0 ? ta.sx : (F.ax_n == 1 ? ta.sy : ta.sz)) + r.s0;
  return r;
}

struct SrcRegs {
  double c, lnA, xa, xb, xn;
};

__device__ __forceinline__ void fetch_source(const TensorArgs &ta, const ItemSrc &is, int blk, SrcRegs &v) {
  const int i = blk + (int)threadIdx.x;
  if (i < is.hi) {
    if (ta.age_c) {
      const int64_t a = is.now - ta.tick[is.s0 + i];
      v.c = ta.age_c[a];
      v.lnA = ta.src_le[is.s0 + i] + ta.age_l[a];
    } else {
      v.c = is.c64[(int64_t)i * kCoefStride];
      v.lnA = is.c64[(int64_t)i * kCoefStride + 5];
    }
    v.xa = is.pa[i];
    v.xb = is.pb[i];
    v.xn = is.pn[i];
  }
}

// Far item: FP32 32 x 32 x 2 matrix-core steps.  The workgroup's tile is
// 32 x 32 points (rows b, columns a); each wave takes a quarter of every
// staged block of 512 sources (2 sources per step, 64 steps) for the whole
// tile, so every L row and R column value is formed once per source.  After
// each block the waves' FP32 sums (128 sources each) go to LDS and every
// thread adds the four of each of its 16 outputs, in wave order, to its FP64
// accumulators (the same summation at every launch shape).  Staged record
// per source (base 2, coordinates relative to the tile's first point, where
// they are small for the sources near the tile, the ones that matter):
// c log2 e, x_a - o_a, x_b - o_b, 2 c dn | (ln A + c dn^2) log2 e, 2 c.
// Layout of a 32 x 32 x 2 step: lane l holds A[l % 32][l / 32] and
// B[l / 32][l % 32]; element r of lane l is D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
constexpr int kFarPad = 36;                              // LDS column stride of the wave sums (floats)
constexpr int kFarSumBytes = 4 * 2 * 32 * kFarPad * 4;   // 4 waves x 2 kinds x 32 columns (one pass)
constexpr int kStageFar = 512;                          // far items: sources staged at a time (128 per wave)
constexpr int kTensorLds = kStageFar * 32 + kFarSumBytes;   // far: records + wave sums; near: 5 kStage doubles
static_assert(kTensorLds >= 5 * kStage * 8, "near items stage 5 doubles per source");

__device__ __forceinline__ void tensor_far(const TensorArgs &ta, const PathTab &tab, int item, int n_chunks_far,
                                           int n_chunks, int chunk_far, unsigned char *lds) {
  float4 (*srf)[2] = (float4(*)[2])lds;
  float *wsum = (float *)(lds + kStageFar * 32);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 31, k = lane >> 5;
  const int tile = item % ta.n_tiles;
  const int ck = (item / ta.n_tiles) % n_chunks_far;
  const int slot = item / (ta.n_tiles * n_chunks_far);
  const int4 tl = ta.tiles[tile];
  const TFace F = ta.faces[tl.x];
  const int lo = ck * chunk_far;
  const int e = lo + chunk_far < tab.n_far[slot] ? lo + chunk_far : tab.n_far[slot];
  const ItemSrc is = item_sources(ta, tab, F, slot, lo, tab.mode[slot] ? lo : e);
  const int bi = tl.y + i, ai = tl.z + i;
  const bool vb = bi < F.nb, va = ai < F.na;
  const double ob = F.sb[tl.y], oa = F.sa[tl.z];
  const float sbr = (float)(F.sb[vb ? bi : tl.y] - ob), sar = (float)(F.sa[va ? ai : tl.z] - oa);
  const bool full_tile = tl.y + 32 <= F.nb && tl.z + 32 <= F.na;
  // this thread's outputs: column rc, rows rr .. rr + 3, of each sum
  const int rc = threadIdx.x & 31, rr = 4 * (threadIdx.x >> 5);
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  fx16 accf[4];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int r = 0; r < 16; ++r) accf[g][r] = 0.f;
  const double l2e = 1.4426950408889634;
  // each thread stages two sources of a block: t and t + 256
  SrcRegs nx0{0.0, 0.0, 0.0, 0.0, 0.0}, nx1{0.0, 0.0, 0.0, 0.0, 0.0};
  auto stage = [&](const SrcRegs &v, int t) {
    const double c = v.c, dn = F.sn - v.xn;
    const double base = fma(c * dn, dn, v.lnA);
    srf[t][0] = make_float4((float)(c * l2e), (float)(v.xa - oa), (float)(v.xb - ob), (float)(2.0 * c * dn));
    srf[t][1] = make_float4((float)(base * l2e), (float)(2.0 * c), 0.f, 0.f);
  };
  if (is.lo < is.hi) {
    fetch_source(ta, is, is.lo, nx0);
    fetch_source(ta, is, is.lo + kStage, nx1);
  }
  for (int blk = is.lo; blk < is.hi; blk += kStageFar) {
    const int n_in = is.hi - blk < kStageFar ? is.hi - blk : kStageFar;
    __syncthreads();
    if ((int)threadIdx.x < n_in) stage(nx0, threadIdx.x);
    if ((int)threadIdx.x + kStage < n_in) stage(nx1, threadIdx.x + kStage);
    if (blk + kStageFar < is.hi) {
      fetch_source(ta, is, blk + kStageFar, nx0);
      fetch_source(ta, is, blk + kStageFar + kStage, nx1);
    }
    __syncthreads();
    if (n_in == kStageFar && full_tile) {
      const int w0 = 128 * wave;
      // every source and every point valid: no masks
#pragma unroll
      for (int st = 0; st < 64; ++st) {
        const int t = w0 + 2 * st + k;
        const float4 u0 = srf[t][0], u1 = srf[t][1];
        const float cl = u0.x, xa = u0.y, xb = u0.z, tn = u0.w, base = u1.x, c2 = u1.y;
        const float db = sbr - xb, da = sar - xa;
        const float L0 = __builtin_amdgcn_exp2f(fmaf(cl, db * db, base));
        const float Lb = L0 * (c2 * db);
        const float Ln = L0 * tn;
        const float R0 = __builtin_amdgcn_exp2f(cl * (da * da));
        const float Ra = R0 * (c2 * da);
        accf[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(L0, R0, accf[0], 0, 0, 0);
        accf[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(L0, Ra, accf[1], 0, 0, 0);
        accf[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(Lb, R0, accf[2], 0, 0, 0);
        accf[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(Ln, R0, accf[3], 0, 0, 0);
      }
    } else {
      // a part block: its source pairs spread evenly over the waves; the
      // sources past the block and the points past the face contribute zeros
      const int pairs = (n_in + 1) / 2, per = (pairs + 3) / 4;
      const int p0 = wave * per, p1 = p0 + per < pairs ? p0 + per : pairs;
      for (int st = p0; st < p1; ++st) {
        int t = 2 * st + k;
        const bool vi = t < n_in;
        t = vi ? t : n_in - 1;
        const float4 u0 = srf[t][0], u1 = srf[t][1];
        const float cl = u0.x, xa = u0.y, xb = u0.z, tn = u0.w, base = u1.x, c2 = u1.y;
        const float db = sbr - xb, da = sar - xa;
        const float el = __builtin_amdgcn_exp2f(fmaf(cl, db * db, base));
        const float L0 = (vi && vb) ? el : 0.f;
        const float Lb = L0 * (c2 * db);
        const float Ln = L0 * tn;
        const float er = __builtin_amdgcn_exp2f(cl * (da * da));
        const float R0 = va ? er : 0.f;
        const float Ra = R0 * (c2 * da);
        accf[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(L0, R0, accf[0], 0, 0, 0);
        accf[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(L0, Ra, accf[1], 0, 0, 0);
        accf[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(Lb, R0, accf[2], 0, 0, 0);
        accf[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(Ln, R0, accf[3], 0, 0, 0);
      }
    }
    // fold, two sums at a time: the waves' FP32 sums into LDS ([wave][sum]
    // [column][row], 4 consecutive rows per lane and element group), then
    // each thread's outputs in FP64, wave 0 first
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h) __syncthreads();
#pragma unroll
      for (int gg = 0; gg < 2; ++gg) {
        const int g = 2 * h + gg;
#pragma unroll
        for (int m = 0; m < 4; ++m)
          *(float4 *)(wsum + ((wave * 2 + gg) * 32 + i) * kFarPad + 8 * m + 4 * k) =
              make_float4(accf[g][4 * m], accf[g][4 * m + 1], accf[g][4 * m + 2], accf[g][4 * m + 3]);
#pragma unroll
        for (int r = 0; r < 16; ++r) accf[g][r] = 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int gg = 0; gg < 2; ++gg) {
        const int g = 2 * h + gg;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const float4 v = *(const float4 *)(wsum + ((w * 2 + gg) * 32 + rc) * kFarPad + rr);
          acc[4 * g] += (double)v.x;
          acc[4 * g + 1] += (double)v.y;
          acc[4 * g + 2] += (double)v.z;
          acc[4 * g + 3] += (double)v.w;
        }
      }
    }
  }
  // a wave's threads write 32 consecutive points of each of two rows
  double *o = ta.part + ((int64_t)slot * n_chunks + ck) * 5 * ta.stride;
  const int64_t S = ta.stride;
  const int ac = tl.z + rc;
  if (ac < F.na) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int br = tl.y + rr + r;
      if (br >= F.nb) continue;
      const int64_t q = F.off + (int64_t)br * F.na + ac;
      o[q] = acc[r];
      o[S + q] = 0.0;
      o[(2 + F.ax_a) * S + q] = acc[4 + r];
      o[(2 + F.ax_b) * S + q] = acc[8 + r];
      o[(2 + F.ax_n) * S + q] = acc[12 + r];
    }
  }
  __syncthreads();   // the staged sources and sums of this item are no longer read
}

// Near item of a short chunk (under 256 sources): FP64 16 x 16 x 4
// matrix-core steps, the four waves on the four 16 x 16 blocks of the tile
// (each forms the exponentials of its block's rows and columns), 4 sources
// per step.  Staged per source: c,
// x_a, x_b, 2 c dn, ln A + c dn^2.  Element r of lane l of a step is
// D[4 r + l / 16][l % 16].
__device__ __forceinline__ void tensor_near_blocks(const TensorArgs &ta, const PathTab &tab, int item, int n_chunks_far,
                                            int n_chunks, int chunk_near, unsigned char *lds) {
  double(*src)[kStage] = (double(*)[kStage])lds;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, k = lane >> 4;
  const int n_kind = n_chunks - n_chunks_far;
  const int tile = item % ta.n_tiles;
  const int ck = (item / ta.n_tiles) % n_kind;
  const int slot = item / (ta.n_tiles * n_kind);
  const int4 tl = ta.tiles[tile];
  const TFace F = ta.faces[tl.x];
  // this wave's 16 x 16 block of the tile: rows b, columns a
  const int b0 = tl.y + 16 * (wave >> 1), a0 = tl.z + 16 * (wave & 1);
  const int lo = tab.n_far[slot] + ck * chunk_near;
  const ItemSrc is = item_sources(ta, tab, F, slot, lo,
                                  lo + chunk_near < tab.n_act[slot] ? lo + chunk_near : tab.n_act[slot]);
  const int bi = b0 + j, ai = a0 + j;
  const bool vb = bi < F.nb, va = ai < F.na;
  const double sb = F.sb[vb ? bi : 0], sa = F.sa[va ? ai : 0];
  dx4 acc[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) acc[g] = dx4{0.0, 0.0, 0.0, 0.0};
  SrcRegs nx{0.0, 0.0, 0.0, 0.0, 0.0};
  if (is.lo < is.hi) fetch_source(ta, is, is.lo, nx);
  for (int blk = is.lo; blk < is.hi; blk += kStage) {
    const int n_in = is.hi - blk < kStage ? is.hi - blk : kStage;
    __syncthreads();
    if ((int)threadIdx.x < n_in) {
      const double c = nx.c, dn = F.sn - nx.xn;
      src[0][threadIdx.x] = c;
      src[1][threadIdx.x] = nx.xa;
      src[2][threadIdx.x] = nx.xb;
      src[3][threadIdx.x] = 2.0 * c * dn;
      src[4][threadIdx.x] = fma(c * dn, dn, nx.lnA);
    }
    if (blk + kStage < is.hi) fetch_source(ta, is, blk + kStage, nx);
    __syncthreads();
    const int n_steps = (n_in + 3) / 4;
    for (int st = 0; st < n_steps; ++st) {
      int t = 4 * st + k;
      const bool vi = t < n_in;
      t = vi ? t : n_in - 1;
      const double c = src[0][t], xa = src[1][t], xb = src[2][t], tn = src[3][t], base = src[4][t];
      const double db = sb - xb, da = sa - xa;
      const double e = exp_f64(fma(c * db, db, base));
      const double L0 = (vi && vb) ? e : 0.0;
      const double Lb = L0 * (2.0 * c * db);
      const double Ln = L0 * tn;
      const double r = exp_f64(c * da * da);
      const double R0 = va ? r : 0.0;
      const double Ra = R0 * (2.0 * c * da);
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(L0, R0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(L0, Ra, acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(Lb, R0, acc[2], 0, 0, 0);
      acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ln, R0, acc[3], 0, 0, 0);
    }
  }
  double *o = ta.part + ((int64_t)slot * n_chunks + n_chunks_far + ck) * 5 * ta.stride;
  const int64_t S = ta.stride;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int br = b0 + 4 * r + k;
    if (br >= F.nb || !va) continue;
    const int64_t q = F.off + (int64_t)br * F.na + ai;
    o[q] = acc[0][r];
    o[S + q] = 0.0;
    o[(2 + F.ax_a) * S + q] = acc[1][r];
    o[(2 + F.ax_b) * S + q] = acc[2][r];
    o[(2 + F.ax_n) * S + q] = acc[3][r];
  }
  __syncthreads();   // the staged sources of this item are no longer read
}

// Near item of a long chunk: FP64 16 x 16 x 4 matrix-core steps, 4 sources
// per step.  The four waves split every staged block of 256 sources (64 each); a wave forms
// the L values of the tile's 32 rows and the R values of its 32 columns for
// its sources (two of each per lane) and runs the 16 products of the four
// 16 x 16 blocks and four sums, so every exponential is formed once per
// source and row or column.  At the end of the item the waves' sums are
// added in wave order through LDS.  Staged per source: c, x_a, x_b, 2 c dn,
// ln A + c dn^2.  Element r of lane l of a step is D[4 r + l / 16][l % 16].
constexpr int kNearRed = 4 * 32 * 32;   // doubles: the waves' sums of one kind for the tile
__device__ __forceinline__ void tensor_near_split(const TensorArgs &ta, const PathTab &tab, int item, int n_chunks_far,
                                            int n_chunks, int chunk_near, unsigned char *lds) {
  double(*src)[kStage] = (double(*)[kStage])lds;
  double *red = (double *)(lds + 5 * kStage * 8);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, k = lane >> 4;
  const int n_kind = n_chunks - n_chunks_far;
  const int tile = item % ta.n_tiles;
  const int ck = (item / ta.n_tiles) % n_kind;
  const int slot = item / (ta.n_tiles * n_kind);
  const int4 tl = ta.tiles[tile];
  const TFace F = ta.faces[tl.x];
  const int lo = tab.n_far[slot] + ck * chunk_near;
  const ItemSrc is = item_sources(ta, tab, F, slot, lo,
                                  lo + chunk_near < tab.n_act[slot] ? lo + chunk_near : tab.n_act[slot]);
  // rows b (two halves) and columns a (two halves) of this lane
  bool vb[2], va[2];
  double sb[2], sa[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int bi = tl.y + 16 * h + j, ai = tl.z + 16 * h + j;
    vb[h] = bi < F.nb;
    va[h] = ai < F.na;
    sb[h] = F.sb[vb[h] ? bi : 0];
    sa[h] = F.sa[va[h] ? ai : 0];
  }
  dx4 acc[4][4];   // [block 2 bh + ah][sum]
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[q][g] = dx4{0.0, 0.0, 0.0, 0.0};
  SrcRegs nx{0.0, 0.0, 0.0, 0.0, 0.0};
  if (is.lo < is.hi) fetch_source(ta, is, is.lo, nx);
  for (int blk = is.lo; blk < is.hi; blk += kStage) {
    const int n_in = is.hi - blk < kStage ? is.hi - blk : kStage;
    __syncthreads();
    if ((int)threadIdx.x < n_in) {
      const double c = nx.c, dn = F.sn - nx.xn;
      src[0][threadIdx.x] = c;
      src[1][threadIdx.x] = nx.xa;
      src[2][threadIdx.x] = nx.xb;
      src[3][threadIdx.x] = 2.0 * c * dn;
      src[4][threadIdx.x] = fma(c * dn, dn, nx.lnA);
    }
    if (blk + kStage < is.hi) fetch_source(ta, is, blk + kStage, nx);
    __syncthreads();
    const int s0 = 64 * wave, s1 = s0 + 64 < n_in ? s0 + 64 : n_in;
    for (int st = s0; st < s1; st += 4) {
      int t = st + k;
      const bool vi = t < s1;
      t = vi ? t : s1 - 1;
      const double c = src[0][t], xa = src[1][t], xb = src[2][t], tn = src[3][t], base = src[4][t];
      double L0[2], Lb[2], Ln[2], R0[2], Ra[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double db = sb[h] - xb, da = sa[h] - xa;
        const double e = exp_f64(fma(c * db, db, base));
        L0[h] = (vi && vb[h]) ? e : 0.0;
        Lb[h] = L0[h] * (2.0 * c * db);
        Ln[h] = L0[h] * tn;
        const double r = exp_f64(c * da * da);
        R0[h] = va[h] ? r : 0.0;
        Ra[h] = R0[h] * (2.0 * c * da);
      }
#pragma unroll
      for (int bh = 0; bh < 2; ++bh)
#pragma unroll
        for (int ah = 0; ah < 2; ++ah) {
          dx4(&a4)[4] = acc[2 * bh + ah];
          a4[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(L0[bh], R0[ah], a4[0], 0, 0, 0);
          a4[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(L0[bh], Ra[ah], a4[1], 0, 0, 0);
          a4[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(Lb[bh], R0[ah], a4[2], 0, 0, 0);
          a4[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ln[bh], R0[ah], a4[3], 0, 0, 0);
        }
    }
  }
  // the waves' sums, one kind at a time, added in wave order: thread t then
  // holds the 4 consecutive points 4 t .. 4 t + 3 of the tile (row-major)
  double out[4][4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    __syncthreads();
#pragma unroll
    for (int bh = 0; bh < 2; ++bh)
#pragma unroll
      for (int ah = 0; ah < 2; ++ah)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          red[wave * 1024 + (16 * bh + 4 * r + k) * 32 + 16 * ah + j] = acc[2 * bh + ah][g][r];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = 4 * threadIdx.x + e;
      out[g][e] = ((red[idx] + red[1024 + idx]) + red[2048 + idx]) + red[3072 + idx];
    }
  }
  double *o = ta.part + ((int64_t)slot * n_chunks + n_chunks_far + ck) * 5 * ta.stride;
  const int64_t S = ta.stride;
  const int row = (4 * threadIdx.x) >> 5, col0 = (4 * threadIdx.x) & 31;
  const int br = tl.y + row;
  if (br < F.nb) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ac = tl.z + col0 + e;
      if (ac >= F.na) break;
      const int64_t q = F.off + (int64_t)br * F.na + ac;
      o[q] = out[0][e];
      o[S + q] = 0.0;
      o[(2 + F.ax_a) * S + q] = out[1][e];
      o[(2 + F.ax_b) * S + q] = out[2][e];
      o[(2 + F.ax_n) * S + q] = out[3][e];
    }
  }
  __syncthreads();   // the staged sources and sums of this item are no longer read
}

// The far items (FP32), slot by slot in the order of the path table (longest
// far history first), taken in turn by the workgroups of a grid sized to
// leave room on the compute units (at most 168 registers: three waves per
// SIMD); then, in a launch of their own (fewer registers), the near items
// (FP64) with the same LDS per workgroup.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_sum_tensor_far(
    TensorArgs ta, PathTab tab, int n_chunks_far, int n_chunks, int chunk_far) {
  __shared__ __align__(16) unsigned char lds[kTensorLds];
  const int n_items = ta.n_tiles * n_chunks_far * tab.count;
  for (int item = blockIdx.x; item < n_items; item += gridDim.x)
    tensor_far(ta, tab, item, n_chunks_far, n_chunks, chunk_far, lds);
}

constexpr int kNearLds = 5 * kStage * 8;                      // staged sources
constexpr int kNearSplitLds = kNearLds + kNearRed * 8;        // + the waves' sums of one kind
static_assert(kNearSplitLds <= kTensorLds, "the near kernels' LDS within the far kernel's footprint");
constexpr int kNearSplitMin = kStage;   // chunks of at least this many sources: the split kernel

__global__ __launch_bounds__(256) void k_sum_tensor_near(TensorArgs ta, PathTab tab, int n_chunks_far, int n_chunks,
                                                         int chunk_near) {
  __shared__ __align__(16) unsigned char lds[kNearLds];
  const int n_items = ta.n_tiles * (n_chunks - n_chunks_far) * tab.count;
  for (int item = blockIdx.x; item < n_items; item += gridDim.x)
    tensor_near_blocks(ta, tab, item, n_chunks_far, n_chunks, chunk_near, lds);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_sum_tensor_near_split(
    TensorArgs ta, PathTab tab, int n_chunks_far, int n_chunks, int chunk_near) {
  __shared__ __align__(16) unsigned char lds[kNearSplitLds];
  const int n_items = ta.n_tiles * (n_chunks - n_chunks_far) * tab.count;
  for (int item = blockIdx.x; item < n_items; item += gridDim.x)
    tensor_near_split(ta, tab, item, n_chunks_far, n_chunks, chunk_near, lds);
}

void launch_sum_tensor(hipStream_t st, const SumPlan &pl, const PathTab &tab, const TensorArgs &a) {
  if (a.n_tiles <= 0 || tab.count <= 0) return;
  const int nch = pl.n_chunks_far + pl.n_chunks_near;
  const int cap = tab.count >= 4 ? a.max_groups_batch : a.max_groups;
  auto grid = [&](int64_t items) { return (unsigned)(cap > 0 && items > cap ? cap : items); };
  const int64_t far_items = (int64_t)a.n_tiles * pl.n_chunks_far * tab.count;
  const int64_t near_items = (int64_t)a.n_tiles * pl.n_chunks_near * tab.count;
  if (far_items > 0)
    hipLaunchKernelGGL(k_sum_tensor_far, dim3(grid(far_items)), dim3(256), (size_t)a.lds_pad, st, a, tab,
                       pl.n_chunks_far, nch, pl.chunk_far);
  // near items: long chunks (the FP64 form) on the source-split kernel,
  // short ones (the recent sources of the FP32 form) on the block kernel
  if (near_items > 0) {
    if (pl.chunk_near >= kNearSplitMin)
      hipLaunchKernelGGL(k_sum_tensor_near_split, dim3(grid(near_items)), dim3(256),
                         (size_t)(a.lds_pad + kTensorLds - kNearSplitLds), st, a, tab, pl.n_chunks_far, nch,
                         pl.chunk_near);
    else
      hipLaunchKernelGGL(k_sum_tensor_near, dim3(grid(near_items)), dim3(256),
                         (size_t)(a.lds_pad + kTensorLds - kNearLds), st, a, tab, pl.n_chunks_far, nch, pl.chunk_near);
  }
}

// the allowance only grows (per device), so a later object asking for less
// never takes room from the launches of one set up before it
bool sum_tensor_prepare(int lds_pad) {
  static std::mutex mu;
  static int granted[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lk(mu);
  if (lds_pad <= granted[dev]) return true;
  if (hipFuncSetAttribute((const void *)k_sum_tensor_far, hipFuncAttributeMaxDynamicSharedMemorySize, lds_pad) !=
          hipSuccess ||
      hipFuncSetAttribute((const void *)k_sum_tensor_near, hipFuncAttributeMaxDynamicSharedMemorySize,
                          lds_pad + kTensorLds - kNearLds) != hipSuccess ||
      hipFuncSetAttribute((const void *)k_sum_tensor_near_split, hipFuncAttributeMaxDynamicSharedMemorySize,
                          lds_pad + kTensorLds - kNearSplitLds) != hipSuccess)
    return false;
  granted[dev] = lds_pad;
  return true;
}

// ---------------------------------------------------------------------------
// kernel sum
// ---------------------------------------------------------------------------
struct SumArgs {
  const double *px, *py, *pz, *pq2;
  const float *fx, *fy, *fz, *fq2;
  const double *c64;
  const float *c32;
  double *part;
  int64_t nq, stride;
  int n_chunks_far, n_chunks, chunk_far, chunk_near;
  const int32_t *qidx;    // optional point indices (nq of them)
};


template <int P>
__global__ __launch_bounds__(512) void k_sum(SumArgs a, PathTab tab) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * (64 * P) + lane;
  const int chunk = blockIdx.y;
  const int slot = blockIdx.z;
  const int n_far = tab.n_far[slot], n_act = tab.n_act[slot];
  const double *c64 = a.c64 + tab.src0[slot] * kCoefStride;
  const float *c32 = a.c32 + tab.src0[slot] * kCoefStride;
  double x[P], y[P], z[P], q2[P];
  int64_t qq[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    int64_t q = base + 64 * j;
    q = q < a.nq ? q : a.nq - 1;
    q = a.qidx ? a.qidx[q] : q;
    qq[j] = q;
    x[j] = a.px[q];
    y[j] = a.py[q];
    z[j] = a.pz[q];
    q2[j] = a.pq2[q];
  }
  double s0[P], s1[P], sx[P], sy[P], sz[P];
#pragma unroll
  for (int j = 0; j < P; ++j) s0[j] = s1[j] = sx[j] = sy[j] = sz[j] = 0.0;

  if (chunk < a.n_chunks_far) {
    const int lo = chunk * a.chunk_far;
    const int hi = tab.mode[slot] ? lo : (lo + a.chunk_far < n_far ? lo + a.chunk_far : n_far);
    float xf[P], yf[P], zf[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      xf[j] = a.fx[qq[j]];
      yf[j] = a.fy[qq[j]];
      zf[j] = a.fz[qq[j]];
    }
    const double ln2 = 0.6931471805599453;
    // tiles are the aligned blocks of the FP32 records (lo is a multiple of kTile32)
    for (int t0 = lo; t0 < hi; t0 += kTile32) {
      const int t1 = t0 + kTile32 < hi ? t0 + kTile32 : hi;
      const float *ob = c32 + (int64_t)t0 * kCoefStride;
      const float ox = ob[5], oy = ob[6], oz = ob[7];
      float rxf[P], ryf[P], rzf[P], qf[P];
      float f0[P], f1[P], fx_[P], fy_[P], fz_[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        rxf[j] = xf[j] - ox;
        ryf[j] = yf[j] - oy;
        rzf[j] = zf[j] - oz;
        qf[j] = fmaf(rxf[j], rxf[j], fmaf(ryf[j], ryf[j], rzf[j] * rzf[j]));
        f0[j] = f1[j] = fx_[j] = fy_[j] = fz_[j] = 0.0f;
      }
      // unrolled so that the scalar loads of the next records are in flight
#pragma unroll 8
      for (int i = t0; i < t1; ++i) {
        const float *c = c32 + (int64_t)i * kCoefStride;
        const float cc = c[0], ux = c[1], uy = c[2], uz = c[3], K = c[4];
#pragma unroll
        for (int j = 0; j < P; ++j) {
          float arg = fmaf(cc, qf[j], K);
          arg = fmaf(ux, rxf[j], arg);
          arg = fmaf(uy, ryf[j], arg);
          arg = fmaf(uz, rzf[j], arg);
          const float e = __builtin_amdgcn_exp2f(arg);
          f0[j] += e;
          f1[j] = fmaf(e, cc, f1[j]);
          fx_[j] = fmaf(e, ux, fx_[j]);
          fy_[j] = fmaf(e, uy, fy_[j]);
          fz_[j] = fmaf(e, uz, fz_[j]);
        }
      }
      // back to the centred form grad = 2 x S1 + S_u of the partials:
      // sum e u = sum e u' - 2 o sum e c
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const double g1 = (double)f1[j];
        s0[j] += (double)f0[j];
        s1[j] += ln2 * g1;
        sx[j] += ln2 * ((double)fx_[j] - 2.0 * (double)ox * g1);
        sy[j] += ln2 * ((double)fy_[j] - 2.0 * (double)oy * g1);
        sz[j] += ln2 * ((double)fz_[j] - 2.0 * (double)oz * g1);
      }
    }
  } else {
    const int c = chunk - a.n_chunks_far;
    const int lo = n_far + c * a.chunk_near;
    const int hi = lo + a.chunk_near < n_act ? lo + a.chunk_near : n_act;
    for (int i = lo; i < hi; ++i) {
      const double *cr = c64 + (int64_t)i * kCoefStride;
      const double cc = cr[0], ux = cr[1], uy = cr[2], uz = cr[3], K = cr[4];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        double arg = fma(cc, q2[j], K);
        arg = fma(ux, x[j], arg);
        arg = fma(uy, y[j], arg);
        arg = fma(uz, z[j], arg);
        const double e = exp_f64(arg);
        s0[j] += e;
        s1[j] = fma(e, cc, s1[j]);
        sx[j] = fma(e, ux, sx[j]);
        sy[j] = fma(e, uy, sy[j]);
        sz[j] = fma(e, uz, sz[j]);
      }
    }
  }
  double *o = a.part + ((int64_t)slot * a.n_chunks + chunk) * 5 * a.stride;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    if (base + 64 * j < a.nq) {
      const int64_t q = qq[j];
      o[q] = s0[j];
      o[a.stride + q] = s1[j];
      o[2 * a.stride + q] = sx[j];
      o[3 * a.stride + q] = sy[j];
      o[4 * a.stride + q] = sz[j];
    }
  }
}

void launch_sum(hipStream_t st, const SumPlan &pl, const PathTab &tab, const double *px, const double *py,
                const double *pz, const double *pq2, const float *fx, const float *fy, const float *fz,
                const float *fq2, const double *c64, const float *c32, double *part, const int32_t *qidx) {
  const int nch = pl.n_chunks_far + pl.n_chunks_near;
  if (nch <= 0 || pl.nq <= 0 || tab.count <= 0) return;
  SumArgs a{px, py, pz, pq2, fx, fy, fz, fq2, c64, c32, part, pl.nq, pl.part_stride,
            pl.n_chunks_far, nch, pl.chunk_far, pl.chunk_near, qidx};
  const int64_t per_block = (int64_t)64 * pl.points_per_lane * pl.waves;
  dim3 g((unsigned)((pl.nq + per_block - 1) / per_block), (unsigned)nch, (unsigned)tab.count);
  dim3 b(64 * pl.waves);
  switch (pl.points_per_lane) {
    case 1: hipLaunchKernelGGL(k_sum<1>, g, b, 0, st, a, tab); break;
    case 2: hipLaunchKernelGGL(k_sum<2>, g, b, 0, st, a, tab); break;
    default: hipLaunchKernelGGL(k_sum<4>, g, b, 0, st, a, tab); break;
  }
}

__global__ void k_finalize(PathTab tab, int by_slot, int64_t nq, int n_chunks, int64_t stride,
                           const double *__restrict__ part, const double *__restrict__ px,
                           const double *__restrict__ py, const double *__restrict__ pz,
                           const double *__restrict__ nx, const double *__restrict__ ny,
                           const double *__restrict__ nz, const double *__restrict__ wdS,
                           const int8_t *__restrict__ role, double kcond, int64_t ostride,
                           double *__restrict__ Tb, double *__restrict__ gb, double *__restrict__ ldb,
                           const double *__restrict__ net, int64_t net_stride) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int slot = blockIdx.y;
  const int64_t oi = by_slot ? slot : tab.path[slot];
  double s0 = 0, s1 = 0, sx = 0, sy = 0, sz = 0;
  const double *pb = part + (int64_t)slot * n_chunks * 5 * stride;
  for (int c = 0; c < n_chunks; ++c) {
    const double *o = pb + (int64_t)c * 5 * stride;
    s0 += o[q];
    s1 += o[stride + q];
    sx += o[2 * stride + q];
    sy += o[3 * stride + q];
    sz += o[4 * stride + q];
  }
  double g0 = fma(2.0 * px[q], s1, sx);
  double g1 = fma(2.0 * py[q], s1, sy);
  double g2 = fma(2.0 * pz[q], s1, sz);
  if (net && tab.mode[slot]) {
    const double *nf = net + (int64_t)slot * 4 * net_stride + q;
    s0 += nf[0];
    g0 += nf[net_stride];
    g1 += nf[2 * net_stride];
    g2 += nf[3 * net_stride];
  }
  double *T = Tb + oi * ostride, *g = gb + oi * 3 * ostride, *ld = ldb + oi * ostride;
  T[q] = s0;
  g[q] = g0;
  g[ostride + q] = g1;
  g[2 * ostride + q] = g2;
  const int r = role[q];
  double d = 0.0;
  if (r == 0) d = -kcond * (g0 * nx[q] + g1 * ny[q] + g2 * nz[q]) * wdS[q];
  else if (r == 1) d = -s0 * wdS[q];
  ld[q] = d;
}

// net heat-loss rate at edge points (Sec. 3.1): grad T^ from the CSR rows of
// basis gradients and the control values u, q~ = -k grad T~ . n,
// q^ = -k grad T^ . n, and the integrands |q~ + q^| ds, |q~| ds
__global__ void k_heat_loss(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            const double *__restrict__ gx, const double *__restrict__ gy,
                            const double *__restrict__ gz, const double *__restrict__ u,
                            const double *__restrict__ G, int64_t gstride, const double *__restrict__ nrm,
                            const double *__restrict__ ds, double kcond, double *__restrict__ qt,
                            double *__restrict__ qh, double *__restrict__ fnet, double *__restrict__ ftil) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const double w = u[col[e]];
    g0 = fma(gx[e], w, g0);
    g1 = fma(gy[e], w, g1);
    g2 = fma(gz[e], w, g2);
  }
  const double n0 = nrm[3 * i], n1 = nrm[3 * i + 1], n2 = nrm[3 * i + 2];
  const double a = -kcond * (G[i] * n0 + G[gstride + i] * n1 + G[2 * gstride + i] * n2);
  const double b = -kcond * (g0 * n0 + g1 * n1 + g2 * n2);
  qt[i] = a;
  qh[i] = b;
  fnet[i] = fabs(a + b) * ds[i];
  ftil[i] = fabs(a) * ds[i];
}

// out[0] = sum a[0..n), out[1] = sum b[0..n) by one block in a fixed order
__global__ void k_sum_pair(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                           double *__restrict__ out) {
  double sa = 0.0, sb = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    sa += a[i];
    sb += b[i];
  }
  sa = block_sum(sa);
  sb = block_sum(sb);
  if (threadIdx.x == 0) {
    out[0] = sa;
    out[1] = sb;
  }
}

void launch_heat_loss(hipStream_t st, int64_t n, const int64_t *rowptr, const int32_t *col, const double *gx,
                      const double *gy, const double *gz, const double *u, const double *G, int64_t gstride,
                      const double *nrm, const double *ds, double kcond, double *qt, double *qh, double *fnet,
                      double *ftil, double *integrals) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_heat_loss, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, rowptr, col,
                     gx, gy, gz, u, G, gstride, nrm, ds, kcond, qt, qh, fnet, ftil);
  hipLaunchKernelGGL(k_sum_pair, dim3(1), dim3(kBlock), 0, st, n, fnet, ftil, integrals);
}

void launch_finalize(hipStream_t st, const PathTab &tab, bool by_slot, int64_t nq, int n_chunks,
                     int64_t part_stride, const double *part, const double *px, const double *py,
                     const double *pz, const double *nx, const double *ny, const double *nz, const double *wdS,
                     const int8_t *role, double kcond, int64_t ostride, double *T, double *g, double *ld,
                     const double *net, int64_t net_stride) {
  if (nq <= 0 || tab.count <= 0) return;
  dim3 gr((unsigned)((nq + kBlock - 1) / kBlock), (unsigned)tab.count);
  hipLaunchKernelGGL(k_finalize, gr, dim3(kBlock), 0, st, tab, by_slot ? 1 : 0, nq, n_chunks, part_stride, part,
                     px, py, pz, nx, ny, nz, wdS, role, kcond, ostride, T, g, ld, net, net_stride);
}

// 32 lanes per row (coalesced along the row), a fixed butterfly sum
constexpr int kRowLanes = 32;
__global__ void k_gather(int64_t nrow, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                         const double *__restrict__ val, const double *__restrict__ in,
                         double *__restrict__ out) {
  const int sub = threadIdx.x & (kRowLanes - 1);
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kRowLanes) + threadIdx.x / kRowLanes;
  if (r >= nrow) return;   // whole 32-lane groups leave together
  double s = 0.0;
  for (int64_t e = rowptr[r] + sub; e < rowptr[r + 1]; e += kRowLanes) s = fma(val[e], in[col[e]], s);
#pragma unroll
  for (int off = kRowLanes / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kRowLanes);
  if (sub == 0) out[r] = s;
}

void launch_gather(hipStream_t st, int64_t nrow, const int64_t *rowptr, const int32_t *col,
                   const double *val, const double *in, double *out) {
  if (nrow <= 0) return;
  const int64_t rows_per_group = kBlock / kRowLanes;
  dim3 g((unsigned)((nrow + rows_per_group - 1) / rows_per_group));
  hipLaunchKernelGGL(k_gather, g, dim3(kBlock), 0, st, nrow, rowptr, col, val, in, out);
}

void launch_csr_eval(hipStream_t st, int64_t nrow, const int64_t *rowptr, const int32_t *col,
                     const double *val, const double *u, double *out) {
  launch_gather(st, nrow, rowptr, col, val, u, out);
}

// ---------------------------------------------------------------------------
// stencil operator helpers
// ---------------------------------------------------------------------------
// y_row = sum_o S[o][row] x[row + offset(o)]; neighbour indices are clamped to
// the array (their coefficients are zero), so no load leaves the vector.
__device__ __forceinline__ double stencil_row(const StencilOp &S, const double *__restrict__ val,
                                              const double *__restrict__ x, int64_t row) {
  const int n0 = S.n[0], n1 = S.n[1];
  const int64_t n01 = (int64_t)n0 * n1;
  const int64_t nm1 = S.nrow - 1;
  double s = 0.0;
  int o = 0;
  for (int d2 = -S.hw[2]; d2 <= S.hw[2]; ++d2)
    for (int d1 = -S.hw[1]; d1 <= S.hw[1]; ++d1) {
      const int64_t b = row + (int64_t)d1 * n0 + (int64_t)d2 * n01;
      for (int d0 = -S.hw[0]; d0 <= S.hw[0]; ++d0, ++o) {
        int64_t nb = b + d0;
        nb = nb < 0 ? 0 : (nb > nm1 ? nm1 : nb);
        s = fma(val[(int64_t)o * S.nrow + row], x[nb], s);
      }
    }
  return s;
}

__global__ void k_theta_init(StencilOp A, const double *__restrict__ Bval, const double *__restrict__ v,
                             const double *__restrict__ F1, const double *__restrict__ F0, double theta,
                             const double *__restrict__ x, double *__restrict__ r, double *__restrict__ part) {
  double acc = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < A.nrow;
       row += (int64_t)gridDim.x * blockDim.x) {
    double rv = 0.0;
    if (!A.free_mask || A.free_mask[row]) {
      const double rhs = stencil_row(A, Bval, v, row) + theta * F1[row] + (1.0 - theta) * F0[row];
      acc += rhs * rhs;
      rv = rhs - stencil_row(A, A.A, x, row);
    }
    r[row] = rv;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_theta_init(hipStream_t st, const StencilOp &A, const double *Bval, const double *v,
                       const double *F1, const double *F0, double theta, double *x, double *r,
                       double *part) {
  dim3 g((unsigned)parts_for(A.nrow));
  hipLaunchKernelGGL(k_theta_init, g, dim3(kBlock), 0, st, A, Bval, v, F1, F0, theta, x, r, part);
}

__global__ void k_scatter(int64_t nD, const int64_t *__restrict__ dofs, const double *__restrict__ vals,
                          double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nD) x[dofs[i]] = vals[i];
}

void launch_scatter_dirichlet(hipStream_t st, int64_t nD, const int64_t *dofs, const double *vals,
                              double *x) {
  if (nD <= 0) return;
  dim3 g((unsigned)((nD + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_scatter, g, dim3(kBlock), 0, st, nD, dofs, vals, x);
}

// r = b - A x (32 lanes per row) and partials of |b|^2
__global__ void k_csr_residual(CsrOp A, const double *__restrict__ b, const double *__restrict__ x,
                               double *__restrict__ r) {
  const int sub = threadIdx.x & (kRowLanes - 1);
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kRowLanes) + threadIdx.x / kRowLanes;
  if (row >= A.nrow) return;
  double s = 0.0;
  for (int64_t e = A.rowptr[row] + sub; e < A.rowptr[row + 1]; e += kRowLanes) s = fma(A.val[e], x[A.col[e]], s);
#pragma unroll
  for (int off = kRowLanes / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kRowLanes);
  if (sub == 0) r[row] = b[row] - s;
}

__global__ void k_sq_parts(int64_t n, const double *__restrict__ b, double *__restrict__ part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += b[i] * b[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_csr_init(hipStream_t st, const CsrOp &A, const double *b, const double *x, double *r,
                     double *part) {
  const int64_t rows_per_group = kBlock / kRowLanes;
  if (A.nrow > 0)
    hipLaunchKernelGGL(k_csr_residual, dim3((unsigned)((A.nrow + rows_per_group - 1) / rows_per_group)), dim3(kBlock),
                       0, st, A, b, x, r);
  hipLaunchKernelGGL(k_sq_parts, dim3((unsigned)parts_for(A.nrow)), dim3(kBlock), 0, st, A.nrow, b, part);
}

// ---------------------------------------------------------------------------
// preconditioners (write z and partials of r.z)
// ---------------------------------------------------------------------------
__global__ void k_jacobi(int64_t n, const double *__restrict__ inv_diag, const double *__restrict__ r,
                         double *__restrict__ z, double *__restrict__ part, const PcgScalars *sc) {
  if (sc && sc->done) return;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double zi = inv_diag[i] * r[i];
    z[i] = zi;
    acc = fma(r[i], zi, acc);
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_jacobi(hipStream_t st, int64_t n, const double *inv_diag, const double *r, double *z,
                   double *part, PcgScalars *sc) {
  dim3 g((unsigned)parts_for(n));
  hipLaunchKernelGGL(k_jacobi, g, dim3(kBlock), 0, st, n, inv_diag, r, z, part, sc);
}

// One mode product of the fast-diagonalisation solve.  The box of free
// indices has sizes m[0..2]; "full" vectors use the n-grid with offset lo,
// "compact" ones the m-box.  out[j along dim] = sum_k W[k, j] in[k along dim]
// with W = U (transposed use: TR) ; optional scaling by inv_diag.
template <bool IN_FULL, bool OUT_FULL, bool TR>
__device__ __forceinline__ double fd_mode_body(const FdOp &F, int dim, const double *__restrict__ in,
                                               double *__restrict__ out, const double *__restrict__ U, bool scale,
                                               const double *__restrict__ rdot, int64_t t0, int64_t tstep) {
  const int m0 = F.m[0], m1 = F.m[1], m2 = F.m[2];
  const int64_t nbox = (int64_t)m0 * m1 * m2;
  const int md = F.m[dim];
  double acc = 0.0;
  for (int64_t t = t0; t < nbox; t += tstep) {
    int j[3] = {(int)(t % m0), (int)((t / m0) % m1), (int)(t / ((int64_t)m0 * m1))};
    const int jd = j[dim];
    double s = 0.0;
    for (int k = 0; k < md; ++k) {
      j[dim] = k;
      int64_t src;
      if (IN_FULL)
        src = (int64_t)(j[0] + F.lo[0]) + (int64_t)F.n[0] * ((j[1] + F.lo[1]) + (int64_t)F.n[1] * (j[2] + F.lo[2]));
      else
        src = (int64_t)j[0] + (int64_t)m0 * (j[1] + (int64_t)m1 * j[2]);
      const double w = TR ? U[(int64_t)k * md + jd] : U[(int64_t)jd * md + k];
      s = fma(w, in[src], s);
    }
    j[dim] = jd;
    if (scale) s *= F.inv_diag[t];
    int64_t dst;
    if (OUT_FULL)
      dst = (int64_t)(j[0] + F.lo[0]) + (int64_t)F.n[0] * ((j[1] + F.lo[1]) + (int64_t)F.n[1] * (j[2] + F.lo[2]));
    else
      dst = t;
    out[dst] = s;
    if (rdot) acc = fma(rdot[dst], s, acc);
  }
  return acc;
}

template <bool IN_FULL, bool OUT_FULL, bool TR>
__global__ void k_fd_mode(FdOp F, int dim, const double *__restrict__ in, double *__restrict__ out,
                          const double *__restrict__ U, bool scale, const double *__restrict__ rdot,
                          double *__restrict__ part, const PcgScalars *sc) {
  if (sc && sc->done) return;
  const double acc = fd_mode_body<IN_FULL, OUT_FULL, TR>(F, dim, in, out, U, scale, rdot,
                                                         (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                                                         (int64_t)gridDim.x * blockDim.x);
  if (part) {
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

// the same mode product for every solve of a batch (blockIdx.y): stage 0
// reads the full vector r + off[b] into t1, stages 1..4 run between t1 and
// t2, stage 5 writes the full vector z + off[b]
template <bool IN_FULL, bool OUT_FULL, bool TR>
__global__ void k_fd_mode_batch(FdBatch B, int dim, int stage, const double *__restrict__ r, double *__restrict__ z,
                                bool scale, const PcgScalars *sc) {
  if (sc && sc->done) return;
  const FdOp &F = B.f[blockIdx.y];
  const double *in = stage == 0 ? r + B.off[blockIdx.y] : ((stage & 1) ? F.t1 : F.t2);
  double *out = stage == 5 ? z + B.off[blockIdx.y] : ((stage & 1) ? F.t2 : F.t1);
  (void)fd_mode_body<IN_FULL, OUT_FULL, TR>(F, dim, in, out, F.U[dim], scale, nullptr,
                                            (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                                            (int64_t)gridDim.x * blockDim.x);
}

__global__ void k_fill(int64_t n, double *__restrict__ z, double v, const PcgScalars *sc) {
  if (sc && sc->done) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = v;
}

// The same mode products with the fibres along `dim` staged in LDS: a
// workgroup takes 256 / m_d consecutive fibres (the other two indices in
// order, the lower one fastest) and the m_d x m_d factor, reads each input
// once (along the fibre for dim 0, across fibres otherwise, so that the
// reads are coalesced), and each thread forms one output with the sum in the
// order of fd_mode_body (the results are bitwise those of k_fd_mode_batch).
// For factors up to kFdLdsMax (m_d <= 64).
constexpr int kFdLdsMax = 64;
template <bool IN_FULL, bool OUT_FULL, bool TR>
__global__ __launch_bounds__(256) void k_fd_mode_lds(FdBatch B, int dim, int stage, const double *__restrict__ r,
                                                     double *__restrict__ z, bool scale, const PcgScalars *sc) {
  if (sc && sc->done) return;
  __shared__ double lu[kFdLdsMax * kFdLdsMax];
  __shared__ double lin[256];
  const FdOp &F = B.f[blockIdx.y];
  const double *in = stage == 0 ? (B.gidx ? r : r + B.off[blockIdx.y]) : ((stage & 1) ? F.t1 : F.t2);
  double *out = stage == 5 ? z + B.off[blockIdx.y] : ((stage & 1) ? F.t2 : F.t1);
  const int md = F.m[dim];
  const int da = dim == 0 ? 1 : 0, dc = dim == 2 ? 1 : 2;   // the other two directions, da < dc
  const int ma = F.m[da];
  const int64_t nfib = (int64_t)ma * F.m[dc];
  const int fb = 256 / md;                                  // fibres per workgroup
  const int64_t f0 = (int64_t)blockIdx.x * fb;
  if (f0 >= nfib) return;                                   // the whole workgroup
  const double *U = F.U[dim];
  for (int i = threadIdx.x; i < md * md; i += blockDim.x) lu[i] = U[i];
  // element of thread t: fibre f and index k along dim
  const int t = threadIdx.x;
  const bool act = t < fb * md;
  const int f = dim == 0 ? t / md : t % fb, k = dim == 0 ? t % md : t / fb;
  const int64_t fib = f0 + f;
  const bool ok = act && fib < nfib;
  int j[3];
  j[dim] = k;
  j[da] = (int)(fib % ma);
  j[dc] = (int)(fib / ma);
  if (act) {
    double v = 0.0;
    if (ok) {
      const int64_t src = IN_FULL ? (int64_t)(j[0] + F.lo[0]) +
                                        (int64_t)F.n[0] * ((j[1] + F.lo[1]) + (int64_t)F.n[1] * (j[2] + F.lo[2]))
                                  : (int64_t)j[0] + (int64_t)F.m[0] * (j[1] + (int64_t)F.m[1] * j[2]);
      if (stage == 0 && B.gidx) {
        const int64_t g = B.gidx[B.off[blockIdx.y] + src];
        v = g >= 0 ? r[g] : 0.0;
      } else {
        v = in[src];
      }
    }
    lin[f * md + k] = v;
  }
  __syncthreads();
  if (!ok) return;
  // output k of fibre f
  double s = 0.0;
  for (int q = 0; q < md; ++q) {
    const double w = TR ? lu[q * md + k] : lu[k * md + q];
    s = fma(w, lin[f * md + q], s);
  }
  const int64_t tb = (int64_t)j[0] + (int64_t)F.m[0] * (j[1] + (int64_t)F.m[1] * j[2]);
  if (scale) s *= F.inv_diag[tb];
  const int64_t dst = OUT_FULL ? (int64_t)(j[0] + F.lo[0]) +
                                     (int64_t)F.n[0] * ((j[1] + F.lo[1]) + (int64_t)F.n[1] * (j[2] + F.lo[2]))
                               : tb;
  out[dst] = s;
}

bool fd_batch_in_lds(const FdBatch &B) {
  for (int q = 0; q < B.count; ++q)
    for (int d = 0; d < 3; ++d)
      if (B.f[q].m[d] > kFdLdsMax) return false;
  return true;
}

void launch_fd_batch(hipStream_t st, const FdBatch &B, const double *r, double *z, const PcgScalars *sc) {
  if (B.count <= 0) return;
  int64_t nbox = 1;
  for (int b = 0; b < B.count; ++b) nbox = std::max<int64_t>(nbox, (int64_t)B.f[b].m[0] * B.f[b].m[1] * B.f[b].m[2]);
  dim3 b(kBlock), g((unsigned)parts_for(nbox), (unsigned)B.count);
  // forward: t1 = U0^T r, t2 = U1^T t1, t1 = D^{-1} U2^T t2; backward: t2 = U2 t1, t1 = U1 t2, z = U0 t1
  if (fd_batch_in_lds(B)) {
    // workgroups per mode product: the most any solve needs
    unsigned gx[3] = {1, 1, 1};
    for (int d = 0; d < 3; ++d)
      for (int q = 0; q < B.count; ++q) {
        const FdOp &F = B.f[q];
        const int64_t nfib = (int64_t)F.m[0] * F.m[1] * F.m[2] / F.m[d];
        const int fb = 256 / F.m[d];
        gx[d] = std::max(gx[d], (unsigned)((nfib + fb - 1) / fb));
      }
    auto gd = [&](int d) { return dim3(gx[d], (unsigned)B.count); };
    hipLaunchKernelGGL((k_fd_mode_lds<true, false, true>), gd(0), b, 0, st, B, 0, 0, r, z, false, sc);
    hipLaunchKernelGGL((k_fd_mode_lds<false, false, true>), gd(1), b, 0, st, B, 1, 1, r, z, false, sc);
    hipLaunchKernelGGL((k_fd_mode_lds<false, false, true>), gd(2), b, 0, st, B, 2, 2, r, z, true, sc);
    hipLaunchKernelGGL((k_fd_mode_lds<false, false, false>), gd(2), b, 0, st, B, 2, 3, r, z, false, sc);
    hipLaunchKernelGGL((k_fd_mode_lds<false, false, false>), gd(1), b, 0, st, B, 1, 4, r, z, false, sc);
    hipLaunchKernelGGL((k_fd_mode_lds<false, true, false>), gd(0), b, 0, st, B, 0, 5, r, z, false, sc);
    return;
  }
  hipLaunchKernelGGL((k_fd_mode_batch<true, false, true>), g, b, 0, st, B, 0, 0, r, z, false, sc);
  hipLaunchKernelGGL((k_fd_mode_batch<false, false, true>), g, b, 0, st, B, 1, 1, r, z, false, sc);
  hipLaunchKernelGGL((k_fd_mode_batch<false, false, true>), g, b, 0, st, B, 2, 2, r, z, true, sc);
  hipLaunchKernelGGL((k_fd_mode_batch<false, false, false>), g, b, 0, st, B, 2, 3, r, z, false, sc);
  hipLaunchKernelGGL((k_fd_mode_batch<false, false, false>), g, b, 0, st, B, 1, 4, r, z, false, sc);
  hipLaunchKernelGGL((k_fd_mode_batch<false, true, false>), g, b, 0, st, B, 0, 5, r, z, false, sc);
}

void launch_fd(hipStream_t st, const FdOp &F, int64_t n, const double *r, double *z, double *part,
               PcgScalars *sc) {
  const int64_t nbox = (int64_t)F.m[0] * F.m[1] * F.m[2];
  const bool full_box = nbox == n;
  dim3 b(kBlock);
  dim3 gb((unsigned)parts_for(nbox));
  // z outside the box stays zero (fixed rows)
  if (!full_box) hipLaunchKernelGGL(k_fill, dim3(parts_for(n)), b, 0, st, n, z, 0.0, sc);
  // forward: t1 = U0^T r, t2 = U1^T t1, t1 = D^{-1} U2^T t2
  hipLaunchKernelGGL((k_fd_mode<true, false, true>), gb, b, 0, st, F, 0, r, F.t1, F.U[0], false,
                     (const double *)nullptr, (double *)nullptr, sc);
  hipLaunchKernelGGL((k_fd_mode<false, false, true>), gb, b, 0, st, F, 1, F.t1, F.t2, F.U[1], false,
                     (const double *)nullptr, (double *)nullptr, sc);
  hipLaunchKernelGGL((k_fd_mode<false, false, true>), gb, b, 0, st, F, 2, F.t2, F.t1, F.U[2], true,
                     (const double *)nullptr, (double *)nullptr, sc);
  // backward: t2 = U2 t1, t1 = U1 t2, z = U0 t1 (+ partials of r.z)
  hipLaunchKernelGGL((k_fd_mode<false, false, false>), gb, b, 0, st, F, 2, F.t1, F.t2, F.U[2], false,
                     (const double *)nullptr, (double *)nullptr, sc);
  hipLaunchKernelGGL((k_fd_mode<false, false, false>), gb, b, 0, st, F, 1, F.t2, F.t1, F.U[1], false,
                     (const double *)nullptr, (double *)nullptr, sc);
  hipLaunchKernelGGL((k_fd_mode<false, true, false>), gb, b, 0, st, F, 0, F.t1, z, F.U[0], false, r, part,
                     sc);
  // partial slots beyond the box-kernel grid are unused by construction
  (void)n;
}

// ---------------------------------------------------------------------------
// PCG steps
// ---------------------------------------------------------------------------
__global__ void k_pcg_start(int64_t n, int n_part_b, const double *__restrict__ part_b, int n_part_rz,
                            const double *__restrict__ part_rz, const double *__restrict__ z,
                            double *__restrict__ p, PcgScalars *sc, double rtol) {
  const double b2 = reduce_parts(part_b, n_part_b);
  const double rz = reduce_parts(part_rz, n_part_rz);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->bnorm2 = b2;
    sc->rz = rz;
    sc->rr = -1.0;
    sc->alpha = sc->beta = 0.0;
    sc->iter = 0;
    sc->rtol2 = rtol * rtol;
    // zero right-hand side (or exact start): nothing to do
    sc->done = (rz == 0.0) ? 1 : 0;
  }
}

void launch_pcg_start(hipStream_t st, int64_t n, int n_part_b, const double *part_b, int n_part_rz,
                      const double *part_rz, const double *z, double *p, PcgScalars *sc, double rtol) {
  dim3 g((unsigned)parts_for(n));
  hipLaunchKernelGGL(k_pcg_start, g, dim3(kBlock), 0, st, n, n_part_b, part_b, n_part_rz, part_rz, z, p, sc,
                     rtol);
}

__global__ void k_stencil_apply_dot(StencilOp A, const double *__restrict__ p, double *__restrict__ q,
                                    double *__restrict__ part, const PcgScalars *sc) {
  if (sc->done) return;
  double acc = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < A.nrow;
       row += (int64_t)gridDim.x * blockDim.x) {
    double y = 0.0;
    if (!A.free_mask || A.free_mask[row]) y = stencil_row(A, A.A, p, row);
    q[row] = y;
    acc = fma(p[row], y, acc);
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_stencil_apply_dot(hipStream_t st, const StencilOp &A, const double *p, double *q, double *part,
                              PcgScalars *sc) {
  dim3 g((unsigned)parts_for(A.nrow));
  hipLaunchKernelGGL(k_stencil_apply_dot, g, dim3(kBlock), 0, st, A, p, q, part, sc);
}

// q = A p: 32 lanes per row, each lane every 32nd entry of the row
// (coalesced reads along it), the lanes' sums added by a fixed butterfly;
// one workgroup per 8 rows, so that every compute unit takes part
constexpr int kCsrLanes = kRowLanes;
__global__ void k_csr_apply(CsrOp A, const double *__restrict__ p, double *__restrict__ q, const PcgScalars *sc) {
  if (sc->done) return;
  const int sub = threadIdx.x & (kCsrLanes - 1);
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kCsrLanes) + threadIdx.x / kCsrLanes;
  if (row >= A.nrow) return;   // whole 32-lane groups leave together
  double s = 0.0;
  for (int64_t e = A.rowptr[row] + sub; e < A.rowptr[row + 1]; e += kCsrLanes) s = fma(A.val[e], p[A.col[e]], s);
#pragma unroll
  for (int off = kCsrLanes / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kCsrLanes);
  if (sub == 0) q[row] = s;
}

// partials of a . b over n entries, parts_for(n) of them
__global__ void k_dot_parts(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                            double *__restrict__ part, const PcgScalars *sc) {
  if (sc->done) return;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc = fma(a[i], b[i], acc);
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

void launch_csr_apply_dot(hipStream_t st, const CsrOp &A, const double *p, double *q, double *part,
                          PcgScalars *sc) {
  const int64_t rows_per_group = kBlock / kCsrLanes;
  if (A.nrow > 0)
    hipLaunchKernelGGL(k_csr_apply, dim3((unsigned)((A.nrow + rows_per_group - 1) / rows_per_group)), dim3(kBlock),
                       0, st, A, p, q, sc);
  hipLaunchKernelGGL(k_dot_parts, dim3((unsigned)parts_for(A.nrow)), dim3(kBlock), 0, st, A.nrow, p, q, part, sc);
}

// r . z of the iteration is summed here from the preconditioner's partials
// (the same fixed-order sum as in k_pcg_start) and stored for
// k_pcg_direction, a later launch: no block of a launch reads what another
// block of it writes
__global__ void k_pcg_update(int64_t n, int n_part, const double *__restrict__ part_pq, int n_part_rz,
                             const double *__restrict__ part_rz, const double *__restrict__ p,
                             const double *__restrict__ q, double *__restrict__ x, double *__restrict__ r,
                             double *__restrict__ part_rr, PcgScalars *sc) {
  if (sc->done) return;
  const double pq = reduce_parts(part_pq, n_part);
  if (!(pq > 0.0)) {  // breakdown: the operator is not positive on p
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->done = 2;
    return;
  }
  const double rz = reduce_parts(part_rz, n_part_rz);
  const double alpha = rz / pq;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    acc = fma(ri, ri, acc);
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->alpha = alpha;
    sc->rz = rz;
  }
}

void launch_pcg_update(hipStream_t st, int64_t n, int n_part, const double *part_pq, int n_part_rz,
                       const double *part_rz, const double *p, const double *q, double *x, double *r,
                       double *part_rr, PcgScalars *sc) {
  dim3 g((unsigned)parts_for(n));
  hipLaunchKernelGGL(k_pcg_update, g, dim3(kBlock), 0, st, n, n_part, part_pq, n_part_rz, part_rz, p, q, x, r,
                     part_rr, sc);
}

__global__ void k_pcg_direction(int64_t n, int n_part_rr, int n_part_rz, const double *__restrict__ part_rr,
                                const double *__restrict__ part_rz, const double *__restrict__ z,
                                double *__restrict__ p, PcgScalars *sc) {
  if (sc->done) return;
  const double rr = reduce_parts(part_rr, n_part_rr);
  const double rz_new = reduce_parts(part_rz, n_part_rz);
  const bool conv = rr <= sc->rtol2 * sc->bnorm2;
  // sc->rz (the previous r . z) was stored by k_pcg_update and is not
  // written here; the next k_pcg_update sums rz_new again from part_rz
  const double beta = rz_new / sc->rz;
  if (!conv) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      p[i] = fma(beta, p[i], z[i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rr = rr;
    sc->beta = beta;
    sc->iter = sc->iter + 1;
    if (conv) sc->done = 1;
  }
}

void launch_pcg_direction(hipStream_t st, int64_t n, int n_part_rr, int n_part_rz, const double *part_rr,
                          const double *part_rz, const double *z, double *p, PcgScalars *sc) {
  dim3 g((unsigned)parts_for(n));
  hipLaunchKernelGGL(k_pcg_direction, g, dim3(kBlock), 0, st, n, n_part_rr, n_part_rz, part_rr, part_rz, z, p,
                     sc);
}

}  // namespace sa
