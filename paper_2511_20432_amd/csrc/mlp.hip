// Far-history network kernels for gfx950: bfloat16 matrix-core GEMM with a
// fused bias/GELU epilogue for the hidden layers, FP32 vector-ALU first and
// output layers, the backward pieces, Adam, and the far-energy summary.
#include "mlp.h"

#include <algorithm>
#include <vector>

namespace sa {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kT = 256;

// FP32 -> bfloat16, round to nearest even (v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU in the tanh form of Hendrycks & Gimpel, "Gaussian Error Linear Units"
// (2016): gelu(z) ~ z (1 + tanh(c (z + k z^3))) / 2 with c = sqrt(2 / pi),
// k = 0.044715.  Since (1 + tanh v) / 2 = 1 / (1 + exp(-2 v)), it takes one
// exp2 and one reciprocal: z / (1 + 2^(z (a + b z^2))) with a = -2 c log2(e),
// b = k a.  Its largest distance from the erf form is 4.7e-4 (near z = 2.7,
// where the bfloat16 step of the stored activation is 1.6e-2); for z -> -inf
// the exp2 overflows to +inf and the result is -0.
constexpr float kGeluA = -2.302208198144325f;
constexpr float kGeluB = -0.1029432395800235f;
constexpr float kGeluC2 = 1.5957691216057308f;    // 2 c
constexpr float kGeluC2K3 = 0.21406444881780076f; // 6 c k

__device__ __forceinline__ float gelu_sig(float z) {
  const float z2 = z * z;
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * fmaf(kGeluB, z2, kGeluA)));
}

__device__ __forceinline__ float gelu(float z) { return z * gelu_sig(z); }

// derivative of the same function: s + z s (1 - s) 2 c (1 + 3 k z^2), s = 1 / (1 + exp(-2 v))
__device__ __forceinline__ float gelu_grad(float z) {
  const float s = gelu_sig(z);
  return fmaf(z * s * (1.0f - s), fmaf(kGeluC2K3, z * z, kGeluC2), s);
}

// ---------------------------------------------------------------------------
// GEMM on the matrix cores: v_mfma_f32_32x32x16_bf16.  Operand layout of one
// 32 x 32 x 16 product per wave: lane l supplies row (A) / column (B) l % 32
// and the 8 consecutive k values 8 (l / 32) .. 8 (l / 32) + 7; the 16 FP32
// results of lane l are column l % 32, rows 8 (r / 4) + 4 (l / 32) + r % 4.
// A workgroup of 4 waves computes a 64 x 64 tile (wave w the 32 x 32 block
// (w & 1, w >> 1)); per 64-wide k-slab both operand tiles are staged in LDS
// as [row][k] with coalesced global reads whatever the operand's layout (a
// row-contiguous operand is read along k, a column-contiguous one along its
// rows and transposed on the way in), the next slab's loads in flight during
// the current slab's products.  Split-K: workgroup z of gridDim.z sums the
// k range [z kc, (z + 1) kc) into FP32 partials, added in z order by
// k_gemm_reduce, which applies the epilogue.
// ---------------------------------------------------------------------------
constexpr int kGT = 64;                 // tile rows / columns / k per slab
constexpr int kGLd = kGT + 8;           // bfloat16 per LDS row (16 B padding)

// 8 consecutive bfloat16 of one operand tile row along k (kcontig) or 8
// consecutive rows at one k (!kcontig), zero outside [0, R) x [0, K); vec:
// the 8 values are one aligned 16-byte word (unit stride along them)
struct Chunk {
  u16x8_t v;
};

__device__ __forceinline__ Chunk fetch_chunk(const bf16_t *__restrict__ p, int64_t sr, int64_t sk, int64_t R,
                                             int64_t K, int64_t r0, int64_t k0, int c, bool kcontig, bool vec) {
  Chunk ch;
  ch.v = u16x8_t{0, 0, 0, 0, 0, 0, 0, 0};
  if (kcontig) {
    const int64_t r = r0 + (c >> 3), k = k0 + 8 * (c & 7);
    if (r >= R) return ch;
    if (vec && k + 8 <= K) {
      ch.v = *reinterpret_cast<const u16x8_t *>(p + r * sr + k);
      return ch;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (k + e < K) ch.v[e] = p[r * sr + (k + e) * sk];
  } else {
    const int64_t k = k0 + (c >> 3), r = r0 + 8 * (c & 7);
    if (k >= K) return ch;
    if (vec && r + 8 <= R) {
      ch.v = *reinterpret_cast<const u16x8_t *>(p + r + k * sk);
      return ch;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (r + e < R) ch.v[e] = p[(r + e) * sr + k * sk];
  }
  return ch;
}

__device__ __forceinline__ void put_chunk(bf16_t *l, const Chunk &ch, int c, bool kcontig) {
  if (kcontig) {
    *reinterpret_cast<u16x8_t *>(l + (c >> 3) * kGLd + 8 * (c & 7)) = ch.v;
  } else {
    const int k = c >> 3, r = 8 * (c & 7);
#pragma unroll
    for (int e = 0; e < 8; ++e) l[(r + e) * kGLd + k] = ch.v[e];
  }
}

__device__ __forceinline__ void gemm_store(const GemmArgs &g, int64_t row, int64_t col, float v) {
  if (row >= g.M || col >= g.N) return;
  if (g.bias) v += g.bias[col];
  if (g.z) g.z[row * g.ldz + col] = v;
  if (g.act == 1) v = gelu(v);
  if (g.out) g.out[row * g.ldo + col] = f2bf(v);
  if (g.outf) g.outf[row * g.ldf + col] = v;
}

// ak / bk: A row-contiguous along k (a_sk == 1), B column-contiguous along k
// (b_sk == 1); kc: k range per split (a multiple of 64)
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g, int ak, int bk, int va, int vb, int64_t kc) {
  __shared__ __align__(16) bf16_t lA[kGT * kGLd];
  __shared__ __align__(16) bf16_t lB[kGT * kGLd];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 31, hh = lane >> 5;
  const int64_t m0 = (int64_t)blockIdx.y * kGT, n0 = (int64_t)blockIdx.x * kGT;
  const int64_t kb = (int64_t)blockIdx.z * kc;
  const int64_t ke = kb + kc < g.K ? kb + kc : g.K;
  // chunks of 8 values: 512 per operand tile, two per thread
  Chunk a[2], b[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    a[u] = fetch_chunk(g.A, g.a_sm, g.a_sk, g.M, ke, m0, kb, tid + 256 * u, ak, va);
    b[u] = fetch_chunk(g.B, g.b_sn, g.b_sk, g.N, ke, n0, kb, tid + 256 * u, bk, vb);
  }
  f32x16_t acc = {};
  const bf16_t *ra = lA + (32 * (w & 1) + li) * kGLd + 8 * hh;
  const bf16_t *rb = lB + (32 * (w >> 1) + li) * kGLd + 8 * hh;
  for (int64_t k0 = kb; k0 < ke; k0 += kGT) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      put_chunk(lA, a[u], tid + 256 * u, ak);
      put_chunk(lB, b[u], tid + 256 * u, bk);
    }
    __syncthreads();
    if (k0 + kGT < ke) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        a[u] = fetch_chunk(g.A, g.a_sm, g.a_sk, g.M, ke, m0, k0 + kGT, tid + 256 * u, ak, va);
        b[u] = fetch_chunk(g.B, g.b_sn, g.b_sk, g.N, ke, n0, k0 + kGT, tid + 256 * u, bk, vb);
      }
    }
#pragma unroll
    for (int s = 0; s < kGT / 16; ++s) {
      const u16x8_t av = *reinterpret_cast<const u16x8_t *>(ra + 16 * s);
      const u16x8_t bv = *reinterpret_cast<const u16x8_t *>(rb + 16 * s);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                    __builtin_bit_cast(bf16x8_t, bv), acc, 0, 0, 0);
    }
  }
  const int64_t col = n0 + 32 * (w >> 1) + li;
  float *part = gridDim.z > 1 ? g.ws + (int64_t)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = m0 + 32 * (w & 1) + 8 * (r >> 2) + 4 * hh + (r & 3);
    if (part) {
      if (row < g.M && col < g.N) part[row * g.N + col] = acc[r];
    } else {
      gemm_store(g, row, col, acc[r]);
    }
  }
}

// sum of the split-K partials in split order, then the epilogue
__global__ void k_gemm_reduce(GemmArgs g, int splits) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.M * g.N) return;
  float v = 0.f;
  for (int z = 0; z < splits; ++z) v += g.ws[(int64_t)z * g.M * g.N + i];
  gemm_store(g, i / g.N, i % g.N, v);
}

// ---------------------------------------------------------------------------
// sums over the batch rows (bias and FP32-layer weight gradients):
// out[i][j] = sum_b P[b][i] Q[b][j] (Q NULL: 1), the rows split into at most
// kRedChunks chunks of R rows, each summed in row order into a partial, the
// partials added in chunk order (k_part_sum): a fixed order for a given B
// ---------------------------------------------------------------------------
constexpr int kRedChunks = 64;

__device__ __forceinline__ float ldf(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldf(const bf16_t *p, int64_t i) { return bf2f(p[i]); }

template <typename TP, typename TQ>
__global__ void k_atb_part(int64_t B, int64_t R, int I, int64_t ldp, const TP *__restrict__ P, int J, int64_t ldq,
                           const TQ *__restrict__ Q, float *__restrict__ part) {
  const int64_t ij = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ij >= (int64_t)I * J) return;
  const int i = (int)(ij / J), j = (int)(ij % J);
  const int64_t b0 = (int64_t)blockIdx.y * R, b1 = b0 + R < B ? b0 + R : B;
  float s = 0.f;
  if (Q) {
    for (int64_t b = b0; b < b1; ++b) s = fmaf(ldf(P, b * ldp + i), ldf(Q, b * ldq + j), s);
  } else {
    for (int64_t b = b0; b < b1; ++b) s += ldf(P, b * ldp + i);
  }
  part[(int64_t)blockIdx.y * I * J + ij] = s;
}

__global__ void k_part_sum(int chunks, int64_t n, const float *__restrict__ part, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + i];
  out[i] = s;
}

__global__ void k_to_bf16(int64_t n, const float *__restrict__ x, bf16_t *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

__global__ void k_to_bf16_t(int64_t R, int64_t C, const float *__restrict__ x, bf16_t *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * C) return;
  const int64_t r = i / C, c = i % C;
  y[c * R + r] = f2bf(x[i]);
}

// first layer, thread per (row, 8 hidden units)
__global__ void k_layer1_full(int64_t rows, const float *__restrict__ X, const float *__restrict__ W1,
                              const float *__restrict__ b1, float *__restrict__ z1, bf16_t *__restrict__ h1) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = t >> 5;
  const int f0 = (int)(t & 31) * 8;
  if (r >= rows) return;
  const float *x = X + r * kMlpIn;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int f = f0 + e;
    const float *w = W1 + (int64_t)f * kMlpIn;
    float s = b1[f];
    for (int j = 0; j < kMlpIn; ++j) s = fmaf(w[j], x[j], s);
    z1[r * kMlpHid + f] = s;
    h1[r * kMlpHid + f] = f2bf(gelu(s));
  }
}

__global__ void k_layer1_const(const float *__restrict__ bins, const float *__restrict__ W1,
                               const float *__restrict__ b1, float *__restrict__ c) {
  const int s = blockIdx.x, f = threadIdx.x;
  const float *w = W1 + (int64_t)f * kMlpIn + kMlpPoint;
  const float *b = bins + (int64_t)s * kMlpBins;
  float v = b1[f];
  for (int j = 0; j < kMlpBins; ++j) v = fmaf(w[j], b[j], v);
  c[(int64_t)s * kMlpHid + f] = v;
}

__global__ void k_layer1_points(int64_t r0, int64_t rows, int64_t nq, const float *__restrict__ pf,
                                const float *__restrict__ c, const float *__restrict__ W1,
                                bf16_t *__restrict__ h1) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t lr = t >> 5;
  if (lr >= rows) return;
  const int64_t r = r0 + lr, s = r / nq, q = r % nq;
  const int f0 = (int)(t & 31) * 8;
  float x[kMlpPoint];
#pragma unroll
  for (int j = 0; j < kMlpPoint; ++j) x[j] = pf[q * kMlpPoint + j];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int f = f0 + e;
    const float *w = W1 + (int64_t)f * kMlpIn;
    float v = c[s * kMlpHid + f];
#pragma unroll
    for (int j = 0; j < kMlpPoint; ++j) v = fmaf(w[j], x[j], v);
    h1[lr * kMlpHid + f] = f2bf(gelu(v));
  }
}

// output layer: 16 lanes per row, 16 hidden units each, fixed-order reduction
__device__ __forceinline__ void out_row(const bf16_t *h, const float *W5, const float *b5, int sub, float y[4]) {
  float a[4] = {0.f, 0.f, 0.f, 0.f};
  const int k0 = sub * 16;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const float hv = bf2f(h[k0 + e]);
#pragma unroll
    for (int o = 0; o < 4; ++o) a[o] = fmaf(W5[o * kMlpHid + k0 + e], hv, a[o]);
  }
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    float v = a[o];
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
    y[o] = v + b5[o];
  }
}

__global__ void k_layer_out(int64_t rows, const bf16_t *__restrict__ h4, const float *__restrict__ W5,
                            const float *__restrict__ b5, float *__restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = t >> 4;
  const int sub = (int)(t & 15);
  if (r >= rows) return;   // whole 16-lane groups leave together
  float v[4];
  out_row(h4 + r * kMlpHid, W5, b5, sub, v);
  if (sub == 0)
    for (int o = 0; o < 4; ++o) y[r * kMlpOut + o] = v[o];
}

__global__ void k_layer_out_field(int64_t r0, int64_t rows, int64_t nq, const bf16_t *__restrict__ h4,
                                  const float *__restrict__ W5, const float *__restrict__ b5, double ts, double gs,
                                  int64_t ostride, double *__restrict__ net) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t lr = t >> 4;
  const int sub = (int)(t & 15);
  if (lr >= rows) return;
  float v[4];
  out_row(h4 + lr * kMlpHid, W5, b5, sub, v);
  if (sub == 0) {
    const int64_t r = r0 + lr, s = r / nq, q = r % nq;
    double *o = net + s * 4 * ostride + q;
    o[0] = ts * (double)v[0];
    o[ostride] = gs * (double)v[1];
    o[2 * ostride] = gs * (double)v[2];
    o[3 * ostride] = gs * (double)v[3];
  }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
__global__ void k_out_dy(int64_t B, const float *__restrict__ y, const float *__restrict__ t, float *__restrict__ dy,
                         double *__restrict__ loss_part) {
  __shared__ double sh[kT];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (r < B) {
    const float sc = 2.0f / (float)(B * kMlpOut);
    for (int o = 0; o < kMlpOut; ++o) {
      const float d = y[r * kMlpOut + o] - t[r * kMlpOut + o];
      dy[r * kMlpOut + o] = sc * d;
      e2 += (double)d * d;
    }
  }
  sh[threadIdx.x] = e2;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = sh[0];
}

__global__ void k_out_dz4(int64_t B, const float *__restrict__ dy, const float *__restrict__ z4,
                          const float *__restrict__ W5, bf16_t *__restrict__ dz4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * kMlpHid) return;
  const int64_t r = i / kMlpHid;
  const int k = (int)(i % kMlpHid);
  float dh = 0.f;
  for (int o = 0; o < kMlpOut; ++o) dh = fmaf(dy[r * kMlpOut + o], W5[o * kMlpHid + k], dh);
  dz4[i] = f2bf(dh * gelu_grad(z4[i]));
}

__global__ void k_gelu_backward(int64_t n, const float *__restrict__ dh, const float *__restrict__ z,
                                bf16_t *__restrict__ dz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dz[i] = f2bf(dh[i] * gelu_grad(z[i]));
}

__global__ void k_layer1_dz(int64_t n, const float *__restrict__ dh, const float *__restrict__ z,
                            float *__restrict__ dz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dz[i] = dh[i] * gelu_grad(z[i]);
}

__global__ void k_adam(int64_t n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// far-energy summary: per-thread bin partials in LDS, then a fixed-order sum
constexpr int kFB = 128;
__global__ __launch_bounds__(kFB) void k_far_bins(PathTab tab, const int8_t *__restrict__ sbin,
                                                  const double *__restrict__ E, double inv_scale,
                                                  float *__restrict__ bins) {
  __shared__ double part[kFB * kMlpBins];   // 64 KiB
  const int s = blockIdx.x, t = threadIdx.x;
  double *mine = part + t * kMlpBins;
  for (int b = 0; b < kMlpBins; ++b) mine[b] = 0.0;
  const int64_t n = tab.n_far[s], base = tab.src0[s];
  const int64_t per = (n + kFB - 1) / kFB;
  const int64_t lo = t * per, hi = lo + per < n ? lo + per : n;
  for (int64_t i = lo; i < hi; ++i) {
    const int b = sbin[base + i];
    mine[b] += E[base + i];
  }
  __syncthreads();
  if (t < kMlpBins) {
    double acc = 0.0;
    for (int u = 0; u < kFB; ++u) acc += part[u * kMlpBins + t];
    bins[(int64_t)s * kMlpBins + t] = (float)(acc * inv_scale);
  }
}

__global__ void k_net_inputs(int64_t nq, const float *__restrict__ pf, const float *__restrict__ bins,
                             float *__restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq * kMlpIn) return;
  const int64_t q = i / kMlpIn;
  const int j = (int)(i % kMlpIn);
  X[i] = j < kMlpPoint ? pf[q * kMlpPoint + j] : bins[j - kMlpPoint];
}

// ---------------------------------------------------------------------------
// fused network: registers hold the activations, LDS holds one weight matrix
// ---------------------------------------------------------------------------
constexpr int kNW = 8;                  // waves per workgroup (two per SIMD, at most 256 registers each)
constexpr int kNRows = kNW * 32;        // rows per workgroup: 32 points per wave
constexpr int kLdsLd = kMlpHid + 8;     // bfloat16 per LDS row of W (16 B padding)

__device__ __forceinline__ int swap23(int k) { return (k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1); }

__global__ void k_net_permute(const bf16_t *__restrict__ W, bf16_t *__restrict__ Wp) {
  const int i = blockIdx.x, k = threadIdx.x;   // row, column
  Wp[i * kMlpHid + k] = W[i * kMlpHid + (k & ~15) + swap23(k & 15)];
}

// stage W [256][256] into LDS rows of kLdsLd
__device__ __forceinline__ void stage_w(const bf16_t *__restrict__ W, bf16_t *lw) {
  __syncthreads();
  for (int id = threadIdx.x; id < kMlpHid * (kMlpHid / 8); id += blockDim.x) {
    const int row = id >> 5, c8 = id & 31;
    *reinterpret_cast<u16x8_t *>(lw + row * kLdsLd + c8 * 8) =
        *reinterpret_cast<const u16x8_t *>(W + row * kMlpHid + c8 * 8);
  }
  __syncthreads();
}

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack2(float lo, float hi) { return (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16); }

// materialise a packed activation word where it is made: keeps the compiler
// from carrying its two FP32 factors to the next layer's first product
__device__ __forceinline__ uint32_t pinned(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// The 256 outputs of a layer are 8 tiles of 32 rows, taken in pairs: the
// 32 products of pair t (W rows 32 t .. 32 t + 63 times the 32 points'
// activations B, 16 k-slices of 8 bfloat16 as 4 packed words, two
// independent accumulator chains), then the pair's epilogue (bias, GELU,
// bfloat16).  Two waves share each SIMD, so one wave's products run beside
// the other's epilogue.
__device__ __forceinline__ void pair_products(const bf16_t *lw, const u32x4_t (&B)[16], int t, int s, int li, int hh,
                                              f32x16_t &c0, f32x16_t &c1) {
  const u16x8_t a0 = *reinterpret_cast<const u16x8_t *>(lw + (32 * t + li) * kLdsLd + 16 * s + 8 * hh);
  const u16x8_t a1 = *reinterpret_cast<const u16x8_t *>(lw + (32 * t + 32 + li) * kLdsLd + 16 * s + 8 * hh);
  const bf16x8_t b = __builtin_bit_cast(bf16x8_t, B[s]);
  c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a0), b, c0, 0, 0, 0);
  c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a1), b, c1, 0, 0, 0);
}

// one k-slice's schedule: its two A-operand reads from LDS, then its two
// products (the reads are issued just before their use, which bounds the
// registers in flight)
__device__ __forceinline__ void slice_schedule() {
  __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // LDS reads
  __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // MFMA
}

// elements r, r + 1 (r even) of tile t: bias + GELU + bfloat16 into the next
// layer's B operand.  Element 4 ((r/4) & 1) + r % 4 of slice 2 t + r / 8
// holds feature 32 t + 8 (r/4) + 4 hh + r % 4 (the order the permuted W3, W4
// columns expect)
__device__ __forceinline__ void epi2(const f32x16_t &acc, const float *__restrict__ bias, int t, int r, int hh,
                                     u32x4_t (&Bn)[16]) {
  const int f = 32 * t + 8 * (r >> 2) + 4 * hh + (r & 3);
  Bn[2 * t + (r >> 3)][(4 * ((r >> 2) & 1) + (r & 3)) >> 1] =
      pinned(pack2(gelu(acc[r] + bias[f]), gelu(acc[r + 1] + bias[f + 1])));
}

// a hidden layer: per pair of output tiles the 32 products, then the
// epilogue of both tiles (the other wave of the SIMD runs meanwhile)
__device__ __forceinline__ void net_hidden(const bf16_t *lw, const u32x4_t (&B)[16], const float *bias, int li,
                                           int hh, u32x4_t (&Bn)[16]) {
#pragma unroll
  for (int t = 0; t < 8; t += 2) {
    f32x16_t c0 = {}, c1 = {};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      pair_products(lw, B, t, s, li, hh, c0, c1);
      slice_schedule();
    }
#pragma unroll
    for (int r = 0; r < 16; r += 2) epi2(c0, bias, t, r, hh, Bn);
#pragma unroll
    for (int r = 0; r < 16; r += 2) epi2(c1, bias, t + 1, r, hh, Bn);
    __builtin_amdgcn_sched_barrier(0);   // one tile pair's values in flight at a time
  }
}

// last hidden layer, elements r, r + 1 of tile t: h4 = bf16(gelu(z4)) into
// the FP32 output layer (w5t [256][4] in LDS: W5 transposed)
__device__ __forceinline__ void out2(const f32x16_t &acc, const float *__restrict__ b4, const float *w5t, int t,
                                     int r, int hh, float (&y)[4]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int rr = r + k;
    const int f = 32 * t + 8 * (rr >> 2) + 4 * hh + (rr & 3);
    const float h = bf2f(f2bf(gelu(acc[rr] + b4[f])));
    const float4 w = *reinterpret_cast<const float4 *>(w5t + 4 * f);
    y[0] = fmaf(w.x, h, y[0]);
    y[1] = fmaf(w.y, h, y[1]);
    y[2] = fmaf(w.z, h, y[2]);
    y[3] = fmaf(w.w, h, y[3]);
  }
}

__device__ __forceinline__ void net_last(const bf16_t *lw, const u32x4_t (&B)[16], const float *b4,
                                         const float *w5t, int li, int hh, float (&y)[4]) {
#pragma unroll 1
  for (int t = 0; t < 8; t += 2) {
    f32x16_t c0 = {}, c1 = {};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      pair_products(lw, B, t, s, li, hh, c0, c1);
      slice_schedule();
    }
#pragma unroll
    for (int r = 0; r < 16; r += 2) out2(c0, b4, w5t, t, r, hh, y);
#pragma unroll
    for (int r = 0; r < 16; r += 2) out2(c1, b4, w5t, t + 1, r, hh, y);
    __builtin_amdgcn_sched_barrier(0);
  }
}

constexpr size_t kNetLdsW = (size_t)kMlpHid * kLdsLd * sizeof(bf16_t);
constexpr size_t kNetLdsW1 = (size_t)kMlpHid * kMlpPoint * sizeof(float);
constexpr size_t kNetLdsW5 = (size_t)kMlpHid * kMlpOut * sizeof(float);
constexpr size_t kNetLdsBias = (size_t)3 * kMlpHid * sizeof(float);

__global__ __launch_bounds__(kNW * 64, 1) void k_net_fused(NetArgs a) {
  extern __shared__ __align__(16) unsigned char net_lds[];
  bf16_t *lw = reinterpret_cast<bf16_t *>(net_lds);
  float *w1 = reinterpret_cast<float *>(net_lds + kNetLdsW);               // [256][6]
  float *w5t = reinterpret_cast<float *>(net_lds + kNetLdsW + kNetLdsW1);  // [256][4]
  float *lb = reinterpret_cast<float *>(net_lds + kNetLdsW + kNetLdsW1 + kNetLdsW5);  // b2, b3, b4
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31, hh = lane >> 5;
  for (int i = threadIdx.x; i < kMlpHid * kMlpPoint; i += blockDim.x)
    w1[i] = a.W1[(i / kMlpPoint) * kMlpIn + i % kMlpPoint];
  for (int i = threadIdx.x; i < kMlpHid * kMlpOut; i += blockDim.x)
    w5t[i] = a.W5[(i % kMlpOut) * kMlpHid + i / kMlpOut];
  for (int i = threadIdx.x; i < kMlpHid; i += blockDim.x) {
    lb[i] = a.b2[i];
    lb[kMlpHid + i] = a.b3[i];
    lb[2 * kMlpHid + i] = a.b4[i];
  }
  __syncthreads();

  // first layer (FP32): lane holds features 16 s + 8 hh + e of its point
  const int64_t lr = (int64_t)blockIdx.x * kNRows + 32 * w + li;
  const bool valid = lr < a.rows;
  const int64_t r = a.r0 + (valid ? lr : 0);
  const int64_t slot = r / a.nq, q = r % a.nq;
  float x[kMlpPoint];
#pragma unroll
  for (int d = 0; d < kMlpPoint; ++d) x[d] = valid ? a.pf[q * kMlpPoint + d] : 0.0f;
  const float *cs = a.c + slot * kMlpHid;
  u32x4_t B[16], Bn[16];
#pragma unroll
  for (int sl = 0; sl < 16; ++sl)
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      float v[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int f = 16 * sl + 8 * hh + e + k;
        v[k] = cs[f];
#pragma unroll
        for (int d = 0; d < kMlpPoint; ++d) v[k] = fmaf(w1[f * kMlpPoint + d], x[d], v[k]);
      }
      B[sl][e >> 1] = pinned(pack2(gelu(v[0]), gelu(v[1])));
      if (e & 2) __builtin_amdgcn_sched_barrier(0);   // bound the registers in flight
    }

  stage_w(a.W2, lw);
  net_hidden(lw, B, lb, li, hh, Bn);
  stage_w(a.W3p, lw);
  net_hidden(lw, Bn, lb + kMlpHid, li, hh, B);
  stage_w(a.W4p, lw);
  float y[4] = {0.f, 0.f, 0.f, 0.f};
  net_last(lw, B, lb + 2 * kMlpHid, w5t, li, hh, y);
#pragma unroll
  for (int o = 0; o < 4; ++o) y[o] += __shfl_xor(y[o], 32, 64);   // the two lane halves hold one point
  if (hh == 0 && valid) {
    double *out = a.net + slot * 4 * a.ostride + q;
    out[0] = a.ts * (double)(y[0] + a.b5[0]);
    out[a.ostride] = a.gs * (double)(y[1] + a.b5[1]);
    out[2 * a.ostride] = a.gs * (double)(y[2] + a.b5[2]);
    out[3 * a.ostride] = a.gs * (double)(y[3] + a.b5[3]);
  }
}

inline unsigned nblk(int64_t n, int b = kT) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_gemm_bf16(hipStream_t st, const GemmArgs &g) {
  if (g.M <= 0 || g.N <= 0) return;
  const bool ak = g.a_sk == 1, bk = g.b_sk == 1;
  const bool va = ((uintptr_t)g.A % 16) == 0 && (ak ? g.a_sm % 8 == 0 : (g.a_sm == 1 && g.a_sk % 8 == 0));
  const bool vb = ((uintptr_t)g.B % 16) == 0 && (bk ? g.b_sn % 8 == 0 : (g.b_sn == 1 && g.b_sk % 8 == 0));
  const int64_t tm = (g.M + kGT - 1) / kGT, tn = (g.N + kGT - 1) / kGT;
  // split the k range when the tiles alone cannot fill the chip
  int64_t splits = 1;
  if (g.ws && g.K > 4 * kGT && tm * tn < 256) {
    splits = std::min<int64_t>((g.K + 4 * kGT - 1) / (4 * kGT), std::max<int64_t>(1, 256 / (tm * tn)));
    splits = std::min<int64_t>(splits, g.ws_floats / (g.M * g.N));
    splits = std::max<int64_t>(splits, 1);
  }
  int64_t kc = (g.K + splits - 1) / splits;
  kc = std::max<int64_t>(kGT, (kc + kGT - 1) / kGT * kGT);
  splits = std::max<int64_t>(1, (g.K + kc - 1) / kc);
  hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)tn, (unsigned)tm, (unsigned)splits), dim3(256), 0, st, g, ak ? 1 : 0,
                     bk ? 1 : 0, va ? 1 : 0, vb ? 1 : 0, kc);
  if (splits > 1) hipLaunchKernelGGL(k_gemm_reduce, dim3(nblk(g.M * g.N)), dim3(kT), 0, st, g, (int)splits);
}

int64_t trainer_ws_floats() {
  return std::max<int64_t>((int64_t)kRedChunks * kMlpHid * kMlpIn, (int64_t)16 * kMlpHid * kMlpHid);
}

void launch_to_bf16(hipStream_t st, int64_t n, const float *x, bf16_t *y) {
  if (n > 0) hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(kT), 0, st, n, x, y);
}

void launch_to_bf16_t(hipStream_t st, int64_t R, int64_t C, const float *x, bf16_t *y) {
  if (R * C > 0) hipLaunchKernelGGL(k_to_bf16_t, dim3(nblk(R * C)), dim3(kT), 0, st, R, C, x, y);
}

void launch_layer1_full(hipStream_t st, int64_t rows, const float *X, const float *W1, const float *b1, float *z1,
                        bf16_t *h1) {
  if (rows > 0) hipLaunchKernelGGL(k_layer1_full, dim3(nblk(rows * 32)), dim3(kT), 0, st, rows, X, W1, b1, z1, h1);
}

void launch_layer1_const(hipStream_t st, int count, const float *bins, const float *W1, const float *b1, float *c) {
  if (count > 0) hipLaunchKernelGGL(k_layer1_const, dim3(count), dim3(kMlpHid), 0, st, bins, W1, b1, c);
}

void launch_layer1_points(hipStream_t st, int64_t r0, int64_t rows, int64_t nq, const float *pf, const float *c,
                          const float *W1, bf16_t *h1) {
  if (rows > 0)
    hipLaunchKernelGGL(k_layer1_points, dim3(nblk(rows * 32)), dim3(kT), 0, st, r0, rows, nq, pf, c, W1, h1);
}

void launch_layer_out(hipStream_t st, int64_t rows, const bf16_t *h4, const float *W5, const float *b5, float *y) {
  if (rows > 0) hipLaunchKernelGGL(k_layer_out, dim3(nblk(rows * 16)), dim3(kT), 0, st, rows, h4, W5, b5, y);
}

void launch_layer_out_field(hipStream_t st, int64_t r0, int64_t rows, int64_t nq, const bf16_t *h4,
                            const float *W5, const float *b5, double t_scale, double g_scale, int64_t ostride,
                            double *net) {
  if (rows > 0)
    hipLaunchKernelGGL(k_layer_out_field, dim3(nblk(rows * 16)), dim3(kT), 0, st, r0, rows, nq, h4, W5, b5,
                       t_scale, g_scale, ostride, net);
}

int loss_parts(int64_t B) { return (int)((B + kT - 1) / kT); }

namespace {

// out[i][j] = sum_b P[b][i] Q[b][j] (Q NULL: 1) through the chunk partials in ws
template <typename TP, typename TQ>
void atb(hipStream_t st, int64_t B, int I, int64_t ldp, const TP *P, int J, int64_t ldq, const TQ *Q, float *ws,
         float *out) {
  const int64_t R = std::max<int64_t>(1, (B + kRedChunks - 1) / kRedChunks);
  const int chunks = B > 0 ? (int)((B + R - 1) / R) : 0;
  const int64_t n = (int64_t)I * J;
  if (chunks > 0)
    hipLaunchKernelGGL((k_atb_part<TP, TQ>), dim3(nblk(n), (unsigned)chunks), dim3(kT), 0, st, B, R, I, ldp, P, J,
                       ldq, Q, ws);
  hipLaunchKernelGGL(k_part_sum, dim3(nblk(n)), dim3(kT), 0, st, chunks, n, ws, out);
}

}  // namespace

void launch_out_backward(hipStream_t st, int64_t B, const float *y, const float *t, const bf16_t *h4,
                         const float *z4, const float *W5, float *dy, double *loss_part, bf16_t *dz4, float *dW5,
                         float *db5, float *ws) {
  if (B <= 0) return;
  hipLaunchKernelGGL(k_out_dy, dim3(nblk(B)), dim3(kT), 0, st, B, y, t, dy, loss_part);
  hipLaunchKernelGGL(k_out_dz4, dim3(nblk(B * kMlpHid)), dim3(kT), 0, st, B, dy, z4, W5, dz4);
  atb(st, B, kMlpOut, kMlpOut, dy, kMlpHid, kMlpHid, h4, ws, dW5);
  atb(st, B, kMlpOut, kMlpOut, dy, 1, 0, (const float *)nullptr, ws, db5);
}

void launch_gelu_backward(hipStream_t st, int64_t n, const float *dh, const float *z, bf16_t *dz) {
  if (n > 0) hipLaunchKernelGGL(k_gelu_backward, dim3(nblk(n)), dim3(kT), 0, st, n, dh, z, dz);
}

void launch_colsum_bf16(hipStream_t st, int64_t B, int64_t N, const bf16_t *dz, float *db, float *ws) {
  if (N > 0) atb(st, B, (int)N, N, dz, 1, 0, (const float *)nullptr, ws, db);
}

void launch_layer1_backward(hipStream_t st, int64_t B, const float *dh1, const float *z1, const float *X,
                            float *dz1, float *dW1, float *db1, float *ws) {
  if (B <= 0) return;
  hipLaunchKernelGGL(k_layer1_dz, dim3(nblk(B * kMlpHid)), dim3(kT), 0, st, B * kMlpHid, dh1, z1, dz1);
  atb(st, B, kMlpHid, kMlpHid, dz1, kMlpIn, kMlpIn, X, ws, dW1);
  atb(st, B, kMlpHid, kMlpHid, dz1, 1, 0, (const float *)nullptr, ws, db1);
}

double reduce_loss_host(hipStream_t st, const double *loss_part, int n) {
  std::vector<double> h(n);
  if (hipMemcpyAsync(h.data(), loss_part, n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return NAN;
  if (hipStreamSynchronize(st) != hipSuccess) return NAN;
  double s = 0.0;
  for (double v : h) s += v;
  return s;
}

void launch_adam(hipStream_t st, int64_t n, float *w, const float *g, float *m, float *v, float lr, float b1,
                 float b2, float eps, int t) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  if (n > 0) hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(kT), 0, st, n, w, g, m, v, lr, b1, b2, eps, c1, c2);
}

size_t net_fused_lds() { return kNetLdsW + kNetLdsW1 + kNetLdsW5 + kNetLdsBias; }

bool net_fused_prepare() {
  return hipFuncSetAttribute((const void *)k_net_fused, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)net_fused_lds()) == hipSuccess;
}

void launch_net_fused(hipStream_t st, const NetArgs &a) {
  if (a.rows <= 0) return;
  hipLaunchKernelGGL(k_net_fused, dim3(nblk(a.rows, kNRows)), dim3(kNW * 64), net_fused_lds(), st, a);
}

void launch_net_permute(hipStream_t st, const bf16_t *W, bf16_t *Wp) {
  hipLaunchKernelGGL(k_net_permute, dim3(kMlpHid), dim3(kMlpHid), 0, st, W, Wp);
}

void launch_net_inputs(hipStream_t st, int64_t nq, const float *pf, const float *bins, float *X) {
  if (nq > 0) hipLaunchKernelGGL(k_net_inputs, dim3(nblk(nq * kMlpIn)), dim3(kT), 0, st, nq, pf, bins, X);
}

void launch_far_bins(hipStream_t st, const PathTab &tab, const int8_t *sbin, const double *E, double e_scale,
                     float *bins) {
  if (tab.count <= 0) return;
  hipLaunchKernelGGL(k_far_bins, dim3(tab.count), dim3(kFB), 0, st, tab, sbin, E, 1.0 / e_scale, bins);
}

}  // namespace sa
