// Far-history network kernels (device code in mlp.hip).
//
// Network (70 -> 256 -> 256 -> 256 -> 256 -> 4, GELU after each hidden
// layer): the first and the output layer run in FP32 on the vector ALUs; the
// three 256 x 256 layers run on the matrix cores with bfloat16 operands and
// FP32 accumulation, their activations stored in bfloat16.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace sa {

typedef uint16_t bf16_t;   // bfloat16 bit pattern

constexpr int kMlpIn = 70;
constexpr int kMlpPoint = 6;    // per-point inputs (normalised position, normal)
constexpr int kMlpBins = 64;    // far-energy summary
constexpr int kMlpHid = 256;
constexpr int kMlpOut = 4;

// offsets (floats) of the FP32 parameter vector: W1 [256][70], b1, W2 [256][256],
// b2, W3, b3, W4, b4, W5 [4][256], b5
struct MlpLayout {
  static constexpr int64_t W1 = 0;
  static constexpr int64_t b1 = W1 + (int64_t)kMlpHid * kMlpIn;
  static constexpr int64_t W2 = b1 + kMlpHid;
  static constexpr int64_t b2 = W2 + (int64_t)kMlpHid * kMlpHid;
  static constexpr int64_t W3 = b2 + kMlpHid;
  static constexpr int64_t b3 = W3 + (int64_t)kMlpHid * kMlpHid;
  static constexpr int64_t W4 = b3 + kMlpHid;
  static constexpr int64_t b4 = W4 + (int64_t)kMlpHid * kMlpHid;
  static constexpr int64_t W5 = b4 + kMlpHid;
  static constexpr int64_t b5 = W5 + (int64_t)kMlpOut * kMlpHid;
  static constexpr int64_t total = b5 + kMlpOut;
};

// C(m, n) = act(sum_k A(m, k) B(k, n) + bias[n]) with A(m, k) = A[m a_sm + k a_sk],
// B(k, n) = B[k b_sk + n b_sn] in bfloat16, FP32 accumulation.  Outputs (each
// optional): z = the pre-activation (FP32), out = act(.) in bfloat16, outf =
// act(.) in FP32.  ws (may be NULL) of ws_floats floats: a workspace that lets
// a product with few output tiles and a long k range split that range over
// workgroups (FP32 partials added in a fixed order).
struct GemmArgs {
  int64_t M, N, K;
  const bf16_t *A;
  int64_t a_sm, a_sk;
  const bf16_t *B;
  int64_t b_sk, b_sn;
  const float *bias;
  int act;              // 0 identity, 1 GELU
  float *z;  int64_t ldz;
  bf16_t *out;  int64_t ldo;
  float *outf;  int64_t ldf;
  float *ws;  int64_t ws_floats;
};
// workspace the trainer's products and batch sums need (floats)
int64_t trainer_ws_floats();
void launch_gemm_bf16(hipStream_t st, const GemmArgs &g);

// FP32 <-> bfloat16 (round to nearest, ties to even)
void launch_to_bf16(hipStream_t st, int64_t n, const float *x, bf16_t *y);
// y[c][r] = bf16(x[r][c]) for an R x C FP32 matrix
void launch_to_bf16_t(hipStream_t st, int64_t R, int64_t C, const float *x, bf16_t *y);

// first layer on rows with full 70-wide FP32 inputs X [rows][70]:
// z1 = W1 x + b1 (FP32), h1 = bf16(gelu(z1))
void launch_layer1_full(hipStream_t st, int64_t rows, const float *X, const float *W1, const float *b1, float *z1,
                        bf16_t *h1);
// first layer on boundary rows: row r = s * nq + q (slot s, point q);
// z1 = c[s] + W1[:, 0:6] pf[q]; c[s] = b1 + W1[:, 6:70] bins[s] (launch_layer1_const)
void launch_layer1_const(hipStream_t st, int count, const float *bins, const float *W1, const float *b1, float *c);
void launch_layer1_points(hipStream_t st, int64_t r0, int64_t rows, int64_t nq, const float *pf, const float *c,
                          const float *W1, bf16_t *h1);
// output layer: y[r][o] = b5[o] + sum_k W5[o][k] h4[r][k]
void launch_layer_out(hipStream_t st, int64_t rows, const bf16_t *h4, const float *W5, const float *b5, float *y);
// boundary rows r0 .. r0+rows of the output layer, scaled into the network
// field of each slot: net[(s*4 + o) * ostride + q] = scale_o * y_o
void launch_layer_out_field(hipStream_t st, int64_t r0, int64_t rows, int64_t nq, const bf16_t *h4,
                            const float *W5, const float *b5, double t_scale, double g_scale, int64_t ostride,
                            double *net);

// backward pieces (training)
// dy = 2 (y - t) / (B * 4); sum of (y - t)^2 per 256 rows in loss_part
// [(B + 255) / 256]; dh4 = W5^T dy; dz4 = bf16(dh4 gelu'(z4));
// dW5 = dy^T h4, db5 = sum dy (FP32; the rows in at most 64 chunks, each
// summed in row order, the chunks in order).  ws: trainer_ws_floats() floats
int loss_parts(int64_t B);
void launch_out_backward(hipStream_t st, int64_t B, const float *y, const float *t, const bf16_t *h4,
                         const float *z4, const float *W5, float *dy, double *loss_part, bf16_t *dz4, float *dW5,
                         float *db5, float *ws);
// dz = bf16(dh gelu'(z)) over B x 256
void launch_gelu_backward(hipStream_t st, int64_t n, const float *dh, const float *z, bf16_t *dz);
// db[n] = sum_b dz[b][n] (bfloat16 rows, FP32 sums in the fixed order above)
void launch_colsum_bf16(hipStream_t st, int64_t B, int64_t N, const bf16_t *dz, float *db, float *ws);
// first layer: dz1 = dh1 gelu'(z1) (FP32); dW1 = dz1^T X, db1 = sum dz1
void launch_layer1_backward(hipStream_t st, int64_t B, const float *dh1, const float *z1, const float *X,
                            float *dz1, float *dW1, float *db1, float *ws);
double reduce_loss_host(hipStream_t st, const double *loss_part, int n);

// Adam on the FP32 master vector (bias-corrected, step t >= 1)
void launch_adam(hipStream_t st, int64_t n, float *w, const float *g, float *m, float *v, float lr, float b1,
                 float b2, float eps, int t);

// Whole network on boundary rows r0 .. r0+rows of the slot-major row space
// (row r: slot r / nq, point r % nq), activations kept in registers: each
// wave computes D = W H^T for 32 points (one MFMA column tile), the 8 waves
// of a workgroup sharing the weight matrix staged in LDS, and the 32 x 32
// accumulator layout of one layer is the next layer's B
// operand once the columns of W3 and W4 are permuted within 16-blocks
// (launch_net_permute).  Writes the scaled far field like
// launch_layer_out_field.
struct NetArgs {
  int64_t r0, rows, nq;
  const float *pf;              // [nq][6]
  const float *c;               // [slot][256] first-layer constants
  const float *W1;              // [256][70] FP32
  const bf16_t *W2, *W3p, *W4p; // [256][256] bfloat16 (W3, W4 column-permuted)
  const float *b2, *b3, *b4, *W5, *b5;
  double ts, gs;
  int64_t ostride;
  double *net;
};
size_t net_fused_lds();
bool net_fused_prepare();
void launch_net_fused(hipStream_t st, const NetArgs &a);
// Wp[i][16 s + k] = W[i][16 s + swap23(k)] (bfloat16), swap23 exchanging bits 2 and 3
void launch_net_permute(hipStream_t st, const bf16_t *W, bf16_t *Wp);

// network inputs of one slot at nq points: X[q] = [pf[q] (6), bins (64)]
void launch_net_inputs(hipStream_t st, int64_t nq, const float *pf, const float *bins, float *X);

// far-energy summary of each slot: bins[s][64] = sum over the sources
// [0, n_far[s]) of path tab.path[s] of E_i / e_scale into bin sbin[i] (the
// 4 x 4 x 4 bin of each source, fixed at set-up); FP64 sums in a fixed order
void launch_far_bins(hipStream_t st, const PathTab &tab, const int8_t *sbin, const double *E, double e_scale,
                     float *bins);

}  // namespace sa
