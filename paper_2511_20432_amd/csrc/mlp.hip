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

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;   // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
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

void launch_net_inputs(hipStream_t st, int64_t nq, const float *pf, const float *bins, float *X) {
  if (nq > 0) hipLaunchKernelGGL(k_net_inputs, dim3(nblk(nq * kMlpIn)), dim3(kT), 0, st, nq, pf, bins, X);
}

void launch_far_bins(hipStream_t st, const PathTab &tab, const int8_t *sbin, const double *E, double e_scale,
                     float *bins) {
  if (tab.count <= 0) return;
  hipLaunchKernelGGL(k_far_bins, dim3(tab.count), dim3(kFB), 0, st, tab, sbin, E, 1.0 / e_scale, bins);
}

}  // namespace sa
