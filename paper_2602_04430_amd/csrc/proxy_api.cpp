// Host side of the learned proxy: parameters (FP32 masters, BF16 copy of W1, Adam state),
// the feature standardiser, training steps and batched inference.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/kvop.h"
#include "host_util.h"
#include "kernels.h"

using namespace kvop;

struct kvop_proxy {
  int d = 0, H = 0;
  int64_t P = 0;                 // packed parameter count: W1 [H d] | b1 [H] | W2 [2 H] | b2 [2]
  float* params = nullptr;       // FP32 masters
  float* m = nullptr;
  float* v = nullptr;
  float* grads = nullptr;
  uint16_t* w1b = nullptr;       // BF16 copy of W1 for the forward projection
  float* mean = nullptr;
  float* istd = nullptr;
  int step = 0;
  float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  DevBuf ws;
  ~kvop_proxy() {
    for (void* p : {(void*)params, (void*)m, (void*)v, (void*)grads, (void*)w1b, (void*)mean, (void*)istd})
      if (p) (void)hipFree(p);
  }
  int64_t o_b1() const { return (int64_t)H * d; }
  int64_t o_w2() const { return o_b1() + H; }
  int64_t o_b2() const { return o_w2() + 2 * H; }
};

namespace {

// per-batch workspace: x [B d] bf16 | xT [d B] bf16 | h1 [B H] | a [B H] | dz [2B] | dh1 [B H] |
// dh1T [H B] bf16 | loss_row [B] | loss [1]
struct ProxyWs {
  uint16_t *x, *xT, *dh1T;
  float *h1, *a, *dz, *dh1, *loss_row, *loss;
};

kvop_status carve_ws(kvop_proxy* p, int B, hipStream_t st, ProxyWs* w) {
  const int64_t d = p->d, H = p->H;
  size_t o_x = 0, o_xT = o_x + align_up(B * d * 2, 256), o_h1 = o_xT + align_up(B * d * 2, 256),
         o_a = o_h1 + align_up(B * H * 4, 256), o_dz = o_a + align_up(B * H * 4, 256),
         o_dh1 = o_dz + align_up(2 * B * 4, 256), o_dh1T = o_dh1 + align_up(B * H * 4, 256),
         o_lr = o_dh1T + align_up(H * B * 2, 256), o_l = o_lr + align_up(B * 4, 256), end = o_l + 256;
  if (p->ws.reserve(end, st) != hipSuccess) return fail(KVOP_ENOMEM, "proxy workspace");
  char* b = (char*)p->ws.p;
  w->x = (uint16_t*)(b + o_x);
  w->xT = (uint16_t*)(b + o_xT);
  w->h1 = (float*)(b + o_h1);
  w->a = (float*)(b + o_a);
  w->dz = (float*)(b + o_dz);
  w->dh1 = (float*)(b + o_dh1);
  w->dh1T = (uint16_t*)(b + o_dh1T);
  w->loss_row = (float*)(b + o_lr);
  w->loss = (float*)(b + o_l);
  return KVOP_OK;
}

// forward projection + head backward + reductions: gradients of the mean CE loss in p->grads
kvop_status proxy_backward(kvop_proxy* p, const float* feats, const int32_t* labels, const int32_t* rows, int B,
                           hipStream_t st, ProxyWs* w) {
  kvop_status s = carve_ws(p, B, st, w);
  if (s != KVOP_OK) return s;
  const int d = p->d, H = p->H;
  HIPTRY(proxy_gather(feats, d, rows, B, p->mean, p->istd, w->x, w->xT, st));
  {
    GemmShape g{B, H, d, d, d, H};
    HIPTRY(gemm(DT_BF16, DT_F32, EPI_STORE, gemm_pick_tile(DT_BF16, EPI_STORE, g), w->x, p->w1b, w->h1, g, st));
  }
  HIPTRY(proxy_head_train(w->h1, B, H, p->params + p->o_b1(), p->params + p->o_w2(), p->params + p->o_b2(), labels,
                          rows, w->a, w->dz, w->dh1, w->dh1T, w->loss_row, st));
  {
    // dW1 [H, d] = dh1^T [H, B] . x [B, d]: contraction over the batch (x^T is [d, B])
    GemmShape g{H, d, B, B, B, d};
    HIPTRY(gemm(DT_BF16, DT_F32, EPI_STORE, gemm_pick_tile(DT_BF16, EPI_STORE, g), w->dh1T, w->xT, p->grads, g, st));
  }
  HIPTRY(proxy_reduce(w->a, w->dz, w->dh1, w->loss_row, B, H, p->grads + p->o_b1(), p->grads + p->o_w2(),
                      p->grads + p->o_b2(), w->loss, st));
  return KVOP_OK;
}

// Scratch of the allocation-free inference: for one call's rows the standardised BF16
// features [n, d_in], then (256-byte aligned) the FP32 hidden pre-activations [n, d_hidden].
// One copy per GPU, held until the process ends.  Host code never uses this name as an
// address: the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[KVOP_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on the first call per device).
kvop_status scratch_address(void** out) {
  int dev = -1;
  HIPTRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(KVOP_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(KVOP_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return KVOP_OK;
}

}  // namespace

extern "C" {

kvop_status kvop_proxy_create(int32_t d_in, int32_t d_hidden, const float* params_dev, kvop_proxy** out) {
  if (!out || !params_dev) return fail(KVOP_EINVAL, "null argument");
  if (d_in < 64 || d_in % 64 || d_hidden < 64 || d_hidden % 64 || d_hidden > 512)
    return fail(KVOP_EINVAL, "proxy sizes: d_in multiple of 64, d_hidden multiple of 64 and <= 512");
  kvop_proxy* p = new (std::nothrow) kvop_proxy();
  if (!p) return fail(KVOP_ENOMEM, "host allocation");
  p->d = d_in;
  p->H = d_hidden;
  p->P = (int64_t)d_hidden * d_in + 3LL * d_hidden + 2;
  size_t pb = p->P * 4;
  if (hipMalloc((void**)&p->params, pb) != hipSuccess || hipMalloc((void**)&p->m, pb) != hipSuccess ||
      hipMalloc((void**)&p->v, pb) != hipSuccess || hipMalloc((void**)&p->grads, pb) != hipSuccess ||
      hipMalloc((void**)&p->w1b, (size_t)d_hidden * d_in * 2) != hipSuccess ||
      hipMalloc((void**)&p->mean, d_in * 4) != hipSuccess || hipMalloc((void**)&p->istd, d_in * 4) != hipSuccess) {
    delete p;
    return fail(KVOP_ENOMEM, "proxy allocation");
  }
  std::vector<float> zeros(d_in, 0.f), ones(d_in, 1.f);
  if (hipMemcpy(p->params, params_dev, pb, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemset(p->m, 0, pb) != hipSuccess || hipMemset(p->v, 0, pb) != hipSuccess ||
      hipMemset(p->grads, 0, pb) != hipSuccess ||
      hipMemcpy(p->mean, zeros.data(), d_in * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->istd, ones.data(), d_in * 4, hipMemcpyHostToDevice) != hipSuccess ||
      f32_to_bf16(p->params, p->w1b, (int64_t)d_hidden * d_in, nullptr) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    delete p;
    return fail(KVOP_EDEVICE, "proxy upload");
  }
  *out = p;
  return KVOP_OK;
}

kvop_status kvop_proxy_destroy(kvop_proxy* p) {
  if (!p) return fail(KVOP_EINVAL, "null proxy");
  (void)hipDeviceSynchronize();
  delete p;
  return KVOP_OK;
}

kvop_status kvop_proxy_fit_standardizer(kvop_proxy* p, const float* feats, int64_t n, void* stream) {
  if (!p || !feats || n < 1) return fail(KVOP_EINVAL, "bad arguments");
  HIPTRY(proxy_stats(feats, n, p->d, p->mean, p->istd, (hipStream_t)stream));
  return KVOP_OK;
}

kvop_status kvop_proxy_set_standardizer(kvop_proxy* p, const float* mean_dev, const float* inv_std_dev, void* stream) {
  if (!p || !mean_dev || !inv_std_dev) return fail(KVOP_EINVAL, "bad arguments");
  HIPTRY(hipMemcpyAsync(p->mean, mean_dev, p->d * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  HIPTRY(hipMemcpyAsync(p->istd, inv_std_dev, p->d * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return KVOP_OK;
}

kvop_status kvop_proxy_grads(kvop_proxy* p, const float* feats, const int32_t* labels, const int32_t* rows,
                             int32_t batch, void* stream, float* grads_out, float* loss_out) {
  if (!p || !feats || !labels || batch < 8 || batch % 8) return fail(KVOP_EINVAL, "batch must be a multiple of 8");
  hipStream_t st = (hipStream_t)stream;
  ProxyWs w;
  kvop_status s = proxy_backward(p, feats, labels, rows, batch, st, &w);
  if (s != KVOP_OK) return s;
  if (grads_out) HIPTRY(hipMemcpyAsync(grads_out, p->grads, p->P * 4, hipMemcpyDeviceToDevice, st));
  if (loss_out) HIPTRY(hipMemcpyAsync(loss_out, w.loss, 4, hipMemcpyDeviceToDevice, st));
  return KVOP_OK;
}

kvop_status kvop_proxy_train_step(kvop_proxy* p, const float* feats, const int32_t* labels, const int32_t* rows,
                                  int32_t batch, float lr, void* stream, float* loss_out) {
  if (!p || !feats || !labels || batch < 8 || batch % 8) return fail(KVOP_EINVAL, "batch must be a multiple of 8");
  if (!(lr > 0.f)) return fail(KVOP_EINVAL, "learning rate must be positive");
  hipStream_t st = (hipStream_t)stream;
  ProxyWs w;
  kvop_status s = proxy_backward(p, feats, labels, rows, batch, st, &w);
  if (s != KVOP_OK) return s;
  p->step++;
  HIPTRY(proxy_adam(p->params, p->grads, p->m, p->v, p->P, (int64_t)p->H * p->d, p->w1b, lr, p->beta1, p->beta2,
                    p->eps, p->step, st));
  if (loss_out) HIPTRY(hipMemcpyAsync(loss_out, w.loss, 4, hipMemcpyDeviceToDevice, st));
  return KVOP_OK;
}

kvop_status kvop_proxy_infer(kvop_proxy* p, const float* feats, int64_t n, float tau, void* stream, int8_t* cls,
                             float* conf, int8_t* answered) {
  if (!p || (n > 0 && (!feats || !cls || !conf || !answered)) || n < 0) return fail(KVOP_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const int chunk = 65536;
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int B = (int)std::min<int64_t>(chunk, n - r0);
    ProxyWs w;
    kvop_status s = carve_ws(p, B, st, &w);
    if (s != KVOP_OK) return s;
    HIPTRY(proxy_gather(feats + r0 * p->d, p->d, nullptr, B, p->mean, p->istd, w.x, nullptr, st));
    GemmShape g{B, p->H, p->d, p->d, p->d, p->H};
    HIPTRY(gemm(DT_BF16, DT_F32, EPI_STORE, gemm_pick_tile(DT_BF16, EPI_STORE, g), w.x, p->w1b, w.h1, g, st));
    HIPTRY(proxy_head_infer(w.h1, B, p->H, p->params + p->o_b1(), p->params + p->o_w2(), p->params + p->o_b2(), tau,
                            cls + r0, conf + r0, answered + r0, st));
  }
  return KVOP_OK;
}

kvop_status kvop_proxy_infer_noalloc(kvop_proxy* p, const float* feats, int64_t n, float tau, void* stream,
                                     int8_t* cls, float* conf, int8_t* answered) {
  if (!p || (n > 0 && (!feats || !cls || !conf || !answered)) || n < 0) return fail(KVOP_EINVAL, "bad arguments");
  const int64_t d = p->d, H = p->H;
  const int64_t max_rows = ((int64_t)KVOP_NOALLOC_SCRATCH_BYTES - 256) / (2 * d + 4 * H);
  if (n > max_rows)
    return fail(KVOP_EINVAL, "kvop_proxy_infer_noalloc takes at most " + std::to_string(max_rows) + " rows for d_in " +
                                 std::to_string(d) + ", d_hidden " + std::to_string(H) + " (" + std::to_string(n) +
                                 " given): split the call");
  if (n == 0) return KVOP_OK;
  void* base = nullptr;
  kvop_status s = scratch_address(&base);
  if (s != KVOP_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  uint16_t* x = (uint16_t*)base;
  float* h1 = (float*)((char*)base + align_up(n * d * 2, 256));
  const int B = (int)n;
  HIPTRY(proxy_gather(feats, p->d, nullptr, B, p->mean, p->istd, x, nullptr, st));
  GemmShape g{B, p->H, p->d, p->d, p->d, p->H};
  HIPTRY(gemm(DT_BF16, DT_F32, EPI_STORE, gemm_pick_tile(DT_BF16, EPI_STORE, g), x, p->w1b, h1, g, st));
  HIPTRY(proxy_head_infer(h1, B, p->H, p->params + p->o_b1(), p->params + p->o_w2(), p->params + p->o_b2(), tau, cls,
                          conf, answered, st));
  return KVOP_OK;
}

kvop_status kvop_proxy_params(kvop_proxy* p, float* out_dev, void* stream) {
  if (!p || !out_dev) return fail(KVOP_EINVAL, "bad arguments");
  HIPTRY(hipMemcpyAsync(out_dev, p->params, p->P * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return KVOP_OK;
}

}  // extern "C"
