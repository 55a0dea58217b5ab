// C ABI of the far-history network trainer: FP32 master weights, bfloat16
// copies for the matrix cores, forward, backward and Adam on the GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "mlp.h"
#include "sa_internal.h"

using sa::bf16_t;
using sa::MlpLayout;

static_assert(MlpLayout::total == sa::kNetParams, "network parameter count");

struct sa_mlp {
  hipStream_t own = nullptr, stream = nullptr;
  std::vector<void *> owned;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // [n_params]
  bf16_t *Wb[3] = {}, *WTb[3] = {};                               // layers 2..4
  int t = 0;                                                      // Adam steps taken
  int64_t cap = 0;                                                // rows of the work buffers
  float *z[5] = {};
  bf16_t *hb[5] = {};
  float *y = nullptr, *dy = nullptr, *dh = nullptr, *dz1 = nullptr;
  bf16_t *dz = nullptr;
  double *loss_part = nullptr;
  float *ws = nullptr;                                            // workspace of the products and batch sums
  ~sa_mlp() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void *p : owned) (void)hipFree(p);
    if (own) (void)hipStreamDestroy(own);
  }
};

namespace {

struct Fail {
  int code;
  std::string msg;
};

void hck(hipError_t e, const char *what) {
  if (e != hipSuccess) throw Fail{SA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

template <class T>
T *alloc(sa_mlp *h, size_t n) {
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw Fail{SA_ENOMEM, "hipMalloc failed"};
  h->owned.push_back(p);
  return (T *)p;
}

template <class F>
int guard(F &&f) {
  try {
    return f();
  } catch (const Fail &e) {
    sa::set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    sa::set_last_error("host allocation failed");
    return SA_ENOMEM;
  } catch (...) {
    sa::set_last_error("unexpected failure");
    return SA_EINVAL;
  }
}

const int64_t kOff[3] = {MlpLayout::W2, MlpLayout::W3, MlpLayout::W4};
const int64_t kBias[3] = {MlpLayout::b2, MlpLayout::b3, MlpLayout::b4};

void refresh_bf16(sa_mlp *h) {
  for (int l = 0; l < 3; ++l) {
    sa::launch_to_bf16(h->stream, (int64_t)sa::kMlpHid * sa::kMlpHid, h->w + kOff[l], h->Wb[l]);
    sa::launch_to_bf16_t(h->stream, sa::kMlpHid, sa::kMlpHid, h->w + kOff[l], h->WTb[l]);
  }
}

void ensure_cap(sa_mlp *h, int64_t B) {
  if (B <= h->cap) return;
  hck(hipStreamSynchronize(h->stream), "sync");
  // the old work buffers stay owned until destruction; training uses one size
  const int64_t c = std::max<int64_t>(B, 1024);
  const int64_t H = sa::kMlpHid;
  for (int l = 1; l <= 4; ++l) {
    h->z[l] = alloc<float>(h, c * H);
    h->hb[l] = alloc<bf16_t>(h, c * H);
  }
  h->y = alloc<float>(h, c * sa::kMlpOut);
  h->dy = alloc<float>(h, c * sa::kMlpOut);
  h->dh = alloc<float>(h, c * H);
  h->dz1 = alloc<float>(h, c * H);
  h->dz = alloc<bf16_t>(h, c * H);
  h->loss_part = alloc<double>(h, sa::loss_parts(c));
  if (!h->ws) h->ws = alloc<float>(h, sa::trainer_ws_floats());
  h->cap = c;
}

// forward over B rows of X [B][70] (device); leaves z, h, y in the work buffers
void forward(sa_mlp *h, int64_t B, const float *X) {
  const int64_t H = sa::kMlpHid;
  sa::launch_layer1_full(h->stream, B, X, h->w + MlpLayout::W1, h->w + MlpLayout::b1, h->z[1], h->hb[1]);
  for (int l = 2; l <= 4; ++l) {
    sa::GemmArgs g{};
    g.M = B;
    g.N = H;
    g.K = H;
    g.A = h->hb[l - 1];
    g.a_sm = H;
    g.a_sk = 1;
    g.B = h->Wb[l - 2];      // B(k, n) = W_l[n][k]
    g.b_sk = 1;
    g.b_sn = H;
    g.bias = h->w + kBias[l - 2];
    g.act = 1;
    g.z = h->z[l];
    g.ldz = H;
    g.out = h->hb[l];
    g.ldo = H;
    sa::launch_gemm_bf16(h->stream, g);
  }
  sa::launch_layer_out(h->stream, B, h->hb[4], h->w + MlpLayout::W5, h->w + MlpLayout::b5, h->y);
}

// gradients of the mean squared error into h->g; returns the loss
double backward(sa_mlp *h, int64_t B, const float *X, const float *T) {
  const int64_t H = sa::kMlpHid;
  sa::launch_out_backward(h->stream, B, h->y, T, h->hb[4], h->z[4], h->w + MlpLayout::W5, h->dy, h->loss_part,
                          h->dz, h->g + MlpLayout::W5, h->g + MlpLayout::b5, h->ws);
  for (int l = 4; l >= 2; --l) {
    // dW_l[n][k] = sum_b dz[b][n] h_{l-1}[b][k]
    sa::GemmArgs gw{};
    gw.M = H;
    gw.N = H;
    gw.K = B;
    gw.A = h->dz;
    gw.a_sm = 1;
    gw.a_sk = H;
    gw.B = h->hb[l - 1];
    gw.b_sk = H;
    gw.b_sn = 1;
    gw.outf = h->g + kOff[l - 2];
    gw.ldf = H;
    gw.ws = h->ws;
    gw.ws_floats = sa::trainer_ws_floats();
    sa::launch_gemm_bf16(h->stream, gw);
    sa::launch_colsum_bf16(h->stream, B, H, h->dz, h->g + kBias[l - 2], h->ws);
    // dh_{l-1}[b][k] = sum_n dz[b][n] W_l[n][k]
    sa::GemmArgs gd{};
    gd.M = B;
    gd.N = H;
    gd.K = H;
    gd.A = h->dz;
    gd.a_sm = H;
    gd.a_sk = 1;
    gd.B = h->WTb[l - 2];    // B(k = n, col = k_in) = W_l^T[k_in][n]
    gd.b_sk = 1;
    gd.b_sn = H;
    gd.outf = h->dh;
    gd.ldf = H;
    sa::launch_gemm_bf16(h->stream, gd);
    if (l > 2) sa::launch_gelu_backward(h->stream, B * H, h->dh, h->z[l - 1], h->dz);
  }
  sa::launch_layer1_backward(h->stream, B, h->dh, h->z[1], X, h->dz1, h->g + MlpLayout::W1, h->g + MlpLayout::b1,
                             h->ws);
  hck(hipGetLastError(), "kernel launch");
  return sa::reduce_loss_host(h->stream, h->loss_part, sa::loss_parts(B)) / (double)(B * sa::kMlpOut);
}

}  // namespace

extern "C" {

int64_t sa_mlp_n_params(void) { return MlpLayout::total; }

int sa_mlp_create(const float *params, int64_t n, sa_mlp **out) {
  if (out) *out = nullptr;
  return guard([&]() -> int {
    if (!out || !params) throw Fail{SA_EINVAL, "NULL argument"};
    if (n != MlpLayout::total) throw Fail{SA_EINVAL, "parameter count does not match the network"};
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(params[i])) throw Fail{SA_EINVAL, "non-finite parameter"};
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) throw Fail{SA_EDEVICE, "no HIP device"};
    std::unique_ptr<sa_mlp> h(new sa_mlp());
    hck(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking), "stream");
    h->stream = h->own;
    h->w = alloc<float>(h.get(), n);
    h->g = alloc<float>(h.get(), n);
    h->m = alloc<float>(h.get(), n);
    h->v = alloc<float>(h.get(), n);
    hck(hipMemcpyAsync(h->w, params, n * sizeof(float), hipMemcpyHostToDevice, h->stream), "upload");
    hck(hipMemsetAsync(h->g, 0, n * sizeof(float), h->stream), "memset");
    hck(hipMemsetAsync(h->m, 0, n * sizeof(float), h->stream), "memset");
    hck(hipMemsetAsync(h->v, 0, n * sizeof(float), h->stream), "memset");
    for (int l = 0; l < 3; ++l) {
      h->Wb[l] = alloc<bf16_t>(h.get(), (size_t)sa::kMlpHid * sa::kMlpHid);
      h->WTb[l] = alloc<bf16_t>(h.get(), (size_t)sa::kMlpHid * sa::kMlpHid);
    }
    refresh_bf16(h.get());
    hck(hipStreamSynchronize(h->stream), "sync");
    hck(hipGetLastError(), "kernel launch");
    *out = h.release();
    return SA_OK;
  });
}

int sa_mlp_get_params(sa_mlp *h, float *params, int64_t n) {
  return guard([&]() -> int {
    if (!h || !params) throw Fail{SA_EINVAL, "NULL argument"};
    if (n != MlpLayout::total) throw Fail{SA_EINVAL, "parameter count does not match the network"};
    hck(hipMemcpyAsync(params, h->w, n * sizeof(float), hipMemcpyDeviceToHost, h->stream), "download");
    hck(hipStreamSynchronize(h->stream), "sync");
    return SA_OK;
  });
}

int sa_mlp_forward(sa_mlp *h, int64_t B, const float *X, float *Y) {
  return guard([&]() -> int {
    if (!h || (B > 0 && (!X || !Y))) throw Fail{SA_EINVAL, "NULL argument"};
    if (B < 0) throw Fail{SA_EINVAL, "negative batch"};
    if (B == 0) return SA_OK;
    ensure_cap(h, B);
    forward(h, B, X);
    hck(hipMemcpyAsync(Y, h->y, B * sa::kMlpOut * sizeof(float), hipMemcpyDeviceToDevice, h->stream), "copy");
    hck(hipStreamSynchronize(h->stream), "sync");
    hck(hipGetLastError(), "kernel launch");
    return SA_OK;
  });
}

int sa_mlp_gradients(sa_mlp *h, int64_t B, const float *X, const float *T, float *grad, double *loss) {
  return guard([&]() -> int {
    if (!h || !X || !T) throw Fail{SA_EINVAL, "NULL argument"};
    if (B < 1) throw Fail{SA_EINVAL, "batch must hold at least one row"};
    ensure_cap(h, B);
    forward(h, B, X);
    const double L = backward(h, B, X, T);
    if (grad) {
      hck(hipMemcpyAsync(grad, h->g, MlpLayout::total * sizeof(float), hipMemcpyDeviceToHost, h->stream),
          "download");
      hck(hipStreamSynchronize(h->stream), "sync");
    }
    if (loss) *loss = L;
    return SA_OK;
  });
}

int sa_mlp_train_step(sa_mlp *h, int64_t B, const float *X, const float *T, float lr, double *loss) {
  return guard([&]() -> int {
    if (!h || !X || !T) throw Fail{SA_EINVAL, "NULL argument"};
    if (B < 1) throw Fail{SA_EINVAL, "batch must hold at least one row"};
    if (!(lr > 0.0f)) throw Fail{SA_EINVAL, "learning rate must be positive"};
    ensure_cap(h, B);
    forward(h, B, X);
    const double L = backward(h, B, X, T);
    if (!std::isfinite(L)) throw Fail{SA_ENOCONV, "training loss is not finite"};
    h->t += 1;
    sa::launch_adam(h->stream, MlpLayout::total, h->w, h->g, h->m, h->v, lr, 0.9f, 0.999f, 1e-8f, h->t);
    refresh_bf16(h);
    hck(hipGetLastError(), "kernel launch");
    if (loss) *loss = L;
    return SA_OK;
  });
}

int sa_mlp_set_stream(sa_mlp *h, void *hip_stream) {
  return guard([&]() -> int {
    if (!h) throw Fail{SA_EINVAL, "NULL object"};
    hck(hipStreamSynchronize(h->stream), "sync");
    h->stream = hip_stream ? (hipStream_t)hip_stream : h->own;
    return SA_OK;
  });
}

void sa_mlp_destroy(sa_mlp *h) { delete h; }

}  // extern "C"
