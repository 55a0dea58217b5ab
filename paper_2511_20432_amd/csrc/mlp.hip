// Far-history network kernels for gfx950: bfloat16 matrix-core GEMM with a
// fused bias/GELU epilogue for the hidden layers, FP32 vector-ALU first and
// output layers, the backward pieces, Adam, and the far-energy summary.
#include "mlp.h"

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

// erf by Abramowitz & Stegun, Handbook of Mathematical Functions, 7.1.26:
// erf(x) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-x^2), t = 1 / (1 + p x),
// |error| <= 1.5e-7 for x >= 0; odd extension for x < 0
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  const float poly =
      fmaf(fmaf(fmaf(fmaf(1.061405429f, t, -1.453152027f), t, 1.421413741f), t, -0.284496736f), t, 0.254829592f) * t;
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * ax * ax);
  return copysignf(fmaf(-poly, e, 1.0f), x);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.72134752044448170f * z * z);
}

// ---------------------------------------------------------------------------
// GEMM on the matrix cores: v_mfma_f32_32x32x16_bf16.  Operand layout of one
// 32 x 32 x 16 product per wave: lane l supplies row (A) / column (B) l % 32
// and the 8 consecutive k values 8 (l / 32) .. 8 (l / 32) + 7; the 16 FP32
// results of lane l are column l % 32, rows 8 (r / 4) + 4 (l / 32) + r % 4.
// A workgroup of 4 waves computes a 128 x 64 tile: wave w rows 32 w .. 32 w + 31,
// two 32-column tiles; operands come straight from global memory (the B
// operand, the weights, is shared by every workgroup and stays in cache).
// ---------------------------------------------------------------------------
__device__ __forceinline__ u16x8_t load8(const bf16_t *p, bool valid, int64_t base, int64_t kk, int64_t sk,
                                         int64_t K, bool vec) {
  u16x8_t r = {0, 0, 0, 0, 0, 0, 0, 0};
  if (!valid) return r;
  if (vec && kk + 8 <= K) return *reinterpret_cast<const u16x8_t *>(p + base + kk);
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (kk + e < K) r[e] = p[base + (kk + e) * sk];
  return r;
}

__device__ __forceinline__ void gemm_store(const GemmArgs &g, int64_t row, int64_t col, float v) {
  if (row >= g.M || col >= g.N) return;
  if (g.bias) v += g.bias[col];
  if (g.z) g.z[row * g.ldz + col] = v;
  if (g.act == 1) v = gelu(v);
  if (g.out) g.out[row * g.ldo + col] = f2bf(v);
  if (g.outf) g.outf[row * g.ldf + col] = v;
}

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g, int vec_a, int vec_b) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31, hh = lane >> 5;
  const int64_t m0 = (int64_t)blockIdx.y * 128 + 32 * w;
  const int64_t n0 = (int64_t)blockIdx.x * 64;
  if (m0 >= g.M) return;
  const int64_t am = m0 + li, bn0 = n0 + li, bn1 = n0 + 32 + li;
  const bool va = am < g.M, vb0 = bn0 < g.N, vb1 = bn1 < g.N;
  const int64_t abase = am * g.a_sm, b0base = bn0 * g.b_sn, b1base = bn1 * g.b_sn;
  f32x16_t acc0 = {}, acc1 = {};
  for (int64_t k0 = 0; k0 < g.K; k0 += 16) {
    const int64_t kk = k0 + 8 * hh;
    const u16x8_t a = load8(g.A, va, abase, kk, g.a_sk, g.K, vec_a);
    const u16x8_t b0 = load8(g.B, vb0, b0base, kk, g.b_sk, g.K, vec_b);
    const u16x8_t b1 = load8(g.B, vb1, b1base, kk, g.b_sk, g.K, vec_b);
    const bf16x8_t av = __builtin_bit_cast(bf16x8_t, a);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8_t, b0), acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8_t, b1), acc1, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t row = m0 + 8 * (r >> 2) + 4 * hh + (r & 3);
    gemm_store(g, row, bn0, acc0[r]);
    gemm_store(g, row, bn1, acc1[r]);
  }
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

__global__ void k_out_dW5(int64_t B, const float *__restrict__ dy, const bf16_t *__restrict__ h4,
                          float *__restrict__ dW5, float *__restrict__ db5) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpOut * kMlpHid) {
    const int o = i / kMlpHid, k = i % kMlpHid;
    float s = 0.f;
    for (int64_t b = 0; b < B; ++b) s = fmaf(dy[b * kMlpOut + o], bf2f(h4[b * kMlpHid + k]), s);
    dW5[i] = s;
  } else if (i < kMlpOut * kMlpHid + kMlpOut) {
    const int o = i - kMlpOut * kMlpHid;
    float s = 0.f;
    for (int64_t b = 0; b < B; ++b) s += dy[b * kMlpOut + o];
    db5[o] = s;
  }
}

__global__ void k_gelu_backward(int64_t n, const float *__restrict__ dh, const float *__restrict__ z,
                                bf16_t *__restrict__ dz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dz[i] = f2bf(dh[i] * gelu_grad(z[i]));
}

__global__ void k_colsum_bf16(int64_t B, int64_t N, const bf16_t *__restrict__ dz, float *__restrict__ db) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int64_t b = 0; b < B; ++b) s += bf2f(dz[b * N + n]);
  db[n] = s;
}

__global__ void k_layer1_dz(int64_t n, const float *__restrict__ dh, const float *__restrict__ z,
                            float *__restrict__ dz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dz[i] = dh[i] * gelu_grad(z[i]);
}

__global__ void k_layer1_dW(int64_t B, const float *__restrict__ dz1, const float *__restrict__ X,
                            float *__restrict__ dW1, float *__restrict__ db1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpHid * kMlpIn) {
    const int f = i / kMlpIn, j = i % kMlpIn;
    float s = 0.f;
    for (int64_t b = 0; b < B; ++b) s = fmaf(dz1[b * kMlpHid + f], X[b * kMlpIn + j], s);
    dW1[i] = s;
  } else if (i < kMlpHid * kMlpIn + kMlpHid) {
    const int f = i - kMlpHid * kMlpIn;
    float s = 0.f;
    for (int64_t b = 0; b < B; ++b) s += dz1[b * kMlpHid + f];
    db1[f] = s;
  }
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
constexpr int kNW = 4;                  // waves per workgroup (one per SIMD: 444 registers per wave)
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

// two 32-row output tiles t, t + 1 of a hidden layer: W rows 32 t .. 32 t + 63
// times the 32 points' activations B (16 k-slices of 8 bfloat16 as 4 packed
// words); two independent accumulator chains keep the matrix pipe busy
__device__ __forceinline__ void net_tiles(const bf16_t *lw, const u32x4_t (&B)[16], int t, int li, int hh,
                                          f32x16_t &acc0, f32x16_t &acc1) {
  acc0 = f32x16_t{};
  acc1 = f32x16_t{};
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const u16x8_t a0 = *reinterpret_cast<const u16x8_t *>(lw + (32 * t + li) * kLdsLd + 16 * s + 8 * hh);
    const u16x8_t a1 = *reinterpret_cast<const u16x8_t *>(lw + (32 * t + 32 + li) * kLdsLd + 16 * s + 8 * hh);
    const bf16x8_t b = __builtin_bit_cast(bf16x8_t, B[s]);
    acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a0), b, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a1), b, acc1, 0, 0, 0);
  }
}

// bias + GELU + bfloat16 of tile t into the next layer's B operand: element
// 4 ((r/4) & 1) + r % 4 of slice 2 t + r / 8 holds feature 32 t + 8 (r/4) + 4 hh + r % 4
// (the order the permuted W3, W4 columns expect)
__device__ __forceinline__ void net_store(const f32x16_t &acc, const float *__restrict__ bias, int t, int hh,
                                          u32x4_t (&Bn)[16]) {
#pragma unroll
  for (int r = 0; r < 16; r += 2) {
    const int f = 32 * t + 8 * (r >> 2) + 4 * hh + (r & 3);
    Bn[2 * t + (r >> 3)][(4 * ((r >> 2) & 1) + (r & 3)) >> 1] =
        pack2(gelu(acc[r] + bias[f]), gelu(acc[r + 1] + bias[f + 1]));
  }
}

__device__ __forceinline__ void net_hidden(const bf16_t *lw, const u32x4_t (&B)[16], const float *__restrict__ bias,
                                           int li, int hh, u32x4_t (&Bn)[16]) {
#pragma unroll
  for (int t = 0; t < 8; t += 2) {
    f32x16_t acc0, acc1;
    net_tiles(lw, B, t, li, hh, acc0, acc1);
    net_store(acc0, bias, t, hh, Bn);
    net_store(acc1, bias, t + 1, hh, Bn);
  }
}

// last hidden layer: h4 = bf16(gelu(z4)) of tile t into the FP32 output layer
__device__ __forceinline__ void net_out_acc(const f32x16_t &acc, const float *__restrict__ b4,
                                            const float *__restrict__ W5, int t, int hh, float (&y)[4]) {
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const int f = 32 * t + 8 * (rr >> 2) + 4 * hh + (rr & 3);
    const float h = bf2f(f2bf(gelu(acc[rr] + b4[f])));
#pragma unroll
    for (int o = 0; o < 4; ++o) y[o] = fmaf(W5[o * kMlpHid + f], h, y[o]);
  }
}

__global__ __launch_bounds__(kNW * 64, 1) void k_net_fused(NetArgs a) {
  extern __shared__ __align__(16) unsigned char net_lds[];
  bf16_t *lw = reinterpret_cast<bf16_t *>(net_lds);
  float *w1 = reinterpret_cast<float *>(net_lds + (size_t)kMlpHid * kLdsLd * sizeof(bf16_t));   // [256][6]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31, hh = lane >> 5;
  for (int i = threadIdx.x; i < kMlpHid * kMlpPoint; i += blockDim.x)
    w1[i] = a.W1[(i / kMlpPoint) * kMlpIn + i % kMlpPoint];
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
      B[sl][e >> 1] = pack2(gelu(v[0]), gelu(v[1]));
    }

  stage_w(a.W2, lw);
  net_hidden(lw, B, a.b2, li, hh, Bn);
  stage_w(a.W3p, lw);
  net_hidden(lw, Bn, a.b3, li, hh, B);
  stage_w(a.W4p, lw);
  // last hidden layer: h4 = bf16(gelu(z4)) straight into the FP32 output layer
  float y[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int t = 0; t < 8; t += 2) {
    f32x16_t acc0, acc1;
    net_tiles(lw, B, t, li, hh, acc0, acc1);
    net_out_acc(acc0, a.b4, a.W5, t, hh, y);
    net_out_acc(acc1, a.b4, a.W5, t + 1, hh, y);
  }
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
  const bool va = g.a_sk == 1 && g.a_sm % 8 == 0 && ((uintptr_t)g.A % 16) == 0;
  const bool vb = g.b_sk == 1 && g.b_sn % 8 == 0 && ((uintptr_t)g.B % 16) == 0;
  dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 127) / 128));
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, g, va ? 1 : 0, vb ? 1 : 0);
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

void launch_out_backward(hipStream_t st, int64_t B, const float *y, const float *t, const bf16_t *h4,
                         const float *z4, const float *W5, float *dy, double *loss_part, bf16_t *dz4, float *dW5,
                         float *db5) {
  if (B <= 0) return;
  hipLaunchKernelGGL(k_out_dy, dim3(nblk(B)), dim3(kT), 0, st, B, y, t, dy, loss_part);
  hipLaunchKernelGGL(k_out_dz4, dim3(nblk(B * kMlpHid)), dim3(kT), 0, st, B, dy, z4, W5, dz4);
  hipLaunchKernelGGL(k_out_dW5, dim3(nblk(kMlpOut * kMlpHid + kMlpOut)), dim3(kT), 0, st, B, dy, h4, dW5, db5);
}

void launch_gelu_backward(hipStream_t st, int64_t n, const float *dh, const float *z, bf16_t *dz) {
  if (n > 0) hipLaunchKernelGGL(k_gelu_backward, dim3(nblk(n)), dim3(kT), 0, st, n, dh, z, dz);
}

void launch_colsum_bf16(hipStream_t st, int64_t B, int64_t N, const bf16_t *dz, float *db) {
  if (N > 0) hipLaunchKernelGGL(k_colsum_bf16, dim3(nblk(N)), dim3(kT), 0, st, B, N, dz, db);
}

void launch_layer1_backward(hipStream_t st, int64_t B, const float *dh1, const float *z1, const float *X,
                            float *dz1, float *dW1, float *db1) {
  if (B <= 0) return;
  hipLaunchKernelGGL(k_layer1_dz, dim3(nblk(B * kMlpHid)), dim3(kT), 0, st, B * kMlpHid, dh1, z1, dz1);
  hipLaunchKernelGGL(k_layer1_dW, dim3(nblk(kMlpHid * kMlpIn + kMlpHid)), dim3(kT), 0, st, B, dz1, X, dW1, db1);
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

size_t net_fused_lds() {
  return (size_t)kMlpHid * kLdsLd * sizeof(bf16_t) + (size_t)kMlpHid * kMlpPoint * sizeof(float);
}

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
