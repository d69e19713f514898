// Learned proxy: z = W2 gelu(W1 x + b1) + b2 on standardised pooled document features,
// p = softmax(z), answered iff max p > tau (the confident items of a two-stage cascade).
//
// Training step (BF16 compute, FP32 master weights, deterministic):
//   gather    : x = bf16((F[row] - mean) * inv_std) for the minibatch rows, also transposed
//   layer 1   : h1 = x W1^T on the BF16 MFMA projection kernel (FP32 out)
//   head      : one wavefront per row: a = gelu(h1 + b1), z = a W2^T + b2, softmax, CE loss,
//               dz = (p - y)/B, da = dz W2, dh1 = da * gelu'(h1 + b1) (FP32; dh1^T also in BF16)
//   dW1       : dh1^T x on the projection kernel (contraction over the batch)
//   reduce    : dW2 = dz^T a, db2 = sum dz, db1 = sum dh1, loss = mean CE (fixed order)
//   adam      : bias-corrected Adam on the FP32 masters; refresh the BF16 copy of W1
#include "common.h"
#include "kernels.h"

namespace kvop {

// ---------------------------------------------------------------- standardiser
// one thread per feature: mean and 1/std over n rows (two passes, FP32; std floor 1e-6)
__global__ void proxy_stats_kernel(const float* __restrict__ F, int64_t n, int d, float* __restrict__ mean,
                                   float* __restrict__ istd) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d) return;
  float s = 0.f;
  for (int64_t r = 0; r < n; r++) s += F[r * d + c];
  float mu = s / (float)n;
  float q = 0.f;
  for (int64_t r = 0; r < n; r++) {
    float t = F[r * d + c] - mu;
    q += t * t;
  }
  float sd = sqrtf(q / (float)n);
  mean[c] = mu;
  istd[c] = 1.0f / fmaxf(sd, 1e-6f);
}

hipError_t proxy_stats(const float* F, int64_t n, int d, float* mean, float* istd, hipStream_t st) {
  hipLaunchKernelGGL(proxy_stats_kernel, dim3((d + 255) / 256), dim3(256), 0, st, F, n, d, mean, istd);
  return hipGetLastError();
}

// ---------------------------------------------------------------- gather (+ transpose)
// tile of 32 rows x 64 features per workgroup; xT (optional) receives the transpose
__global__ __launch_bounds__(256) void proxy_gather_kernel(const float* __restrict__ F, int d,
                                                           const int32_t* __restrict__ rows, int B,
                                                           const float* __restrict__ mean,
                                                           const float* __restrict__ istd, bf16_t* __restrict__ x,
                                                           bf16_t* __restrict__ xT) {
  __shared__ bf16_t tile[32][64 + 2];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 32 * 64; e += 256) {
    int rr = e / 64, cc = e % 64;
    int b = r0 + rr, c = c0 + cc;
    bf16_t v = 0;
    if (b < B && c < d) {
      int64_t src = rows ? rows[b] : b;
      v = f2bf((F[src * d + c] - mean[c]) * istd[c]);
      x[(int64_t)b * d + c] = v;
    }
    tile[rr][cc] = v;
  }
  if (!xT) return;
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 64; e += 256) {
    int cc = e / 32, rr = e % 32;
    int b = r0 + rr, c = c0 + cc;
    if (b < B && c < d) xT[(int64_t)c * B + b] = tile[rr][cc];
  }
}

hipError_t proxy_gather(const float* F, int d, const int32_t* rows, int B, const float* mean, const float* istd,
                        bf16_t* x, bf16_t* xT, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  dim3 grid((d + 63) / 64, (B + 31) / 32);
  hipLaunchKernelGGL(proxy_gather_kernel, grid, dim3(256), 0, st, F, d, rows, B, mean, istd, x, xT);
  return hipGetLastError();
}

// ---------------------------------------------------------------- per-row head
__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// one wavefront per row; H <= 512 (H/64 hidden units per lane)
template <bool TRAIN>
__global__ __launch_bounds__(256) void proxy_head_kernel(const float* __restrict__ h1, int B, int H,
                                                         const float* __restrict__ b1, const float* __restrict__ W2,
                                                         const float* __restrict__ b2, const int32_t* __restrict__ labels,
                                                         const int32_t* __restrict__ rows, float tau,
                                                         int8_t* __restrict__ cls, float* __restrict__ conf,
                                                         int8_t* __restrict__ answered, float* __restrict__ a_out,
                                                         float* __restrict__ dz_out, float* __restrict__ dh1,
                                                         bf16_t* __restrict__ dh1T, float* __restrict__ loss_row) {
  int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= B) return;
  constexpr int MAXU = 8;
  float pre[MAXU], act[MAXU];
  float z0 = 0.f, z1 = 0.f;
  const int U = H / 64;
#pragma unroll
  for (int u = 0; u < MAXU; u++) {
    if (u >= U) break;
    int j = lane + 64 * u;
    pre[u] = h1[(int64_t)b * H + j] + b1[j];
    act[u] = gelu_f(pre[u]);
    z0 += act[u] * W2[j];
    z1 += act[u] * W2[H + j];
  }
  z0 = wave_sum(z0) + b2[0];
  z1 = wave_sum(z1) + b2[1];
  float m = fmaxf(z0, z1);
  float e0 = expf(z0 - m), e1 = expf(z1 - m);
  float p0 = e0 / (e0 + e1), p1 = e1 / (e0 + e1);
  if constexpr (!TRAIN) {
    if (lane == 0) {
      int c = p1 > p0 ? 1 : 0;
      float cf = c ? p1 : p0;
      cls[b] = (int8_t)c;
      conf[b] = cf;
      answered[b] = cf > tau ? 1 : 0;
    }
  } else {
    int y = labels[rows ? rows[b] : b];
    float lse = m + logf(e0 + e1);
    float d0 = (p0 - (y == 0 ? 1.f : 0.f)) / (float)B;
    float d1 = (p1 - (y == 1 ? 1.f : 0.f)) / (float)B;
    if (lane == 0) {
      loss_row[b] = lse - (y == 1 ? z1 : z0);
      dz_out[2 * b] = d0;
      dz_out[2 * b + 1] = d1;
    }
#pragma unroll
    for (int u = 0; u < MAXU; u++) {
      if (u >= U) break;
      int j = lane + 64 * u;
      float da = d0 * W2[j] + d1 * W2[H + j];
      float g = da * gelu_grad_f(pre[u]);
      a_out[(int64_t)b * H + j] = act[u];
      dh1[(int64_t)b * H + j] = g;
      dh1T[(int64_t)j * B + b] = f2bf(g);
    }
  }
}

hipError_t proxy_head_infer(const float* h1, int n, int H, const float* b1, const float* W2, const float* b2,
                            float tau, int8_t* cls, float* conf, int8_t* answered, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (H % 64 || H > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(proxy_head_kernel<false>, dim3((n + 3) / 4), dim3(256), 0, st, h1, n, H, b1, W2, b2, nullptr,
                     nullptr, tau, cls, conf, answered, nullptr, nullptr, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t proxy_head_train(const float* h1, int B, int H, const float* b1, const float* W2, const float* b2,
                            const int32_t* labels, const int32_t* rows, float* a, float* dz, float* dh1, bf16_t* dh1T,
                            float* loss_row, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (H % 64 || H > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(proxy_head_kernel<true>, dim3((B + 3) / 4), dim3(256), 0, st, h1, B, H, b1, W2, b2, labels, rows,
                     0.f, nullptr, nullptr, nullptr, a, dz, dh1, dh1T, loss_row);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reductions over the batch
// thread j: db1[j], dW2[0][j], dW2[1][j]; thread 0 also db2 and the mean loss (fixed order)
__global__ void proxy_reduce_kernel(const float* __restrict__ a, const float* __restrict__ dz,
                                    const float* __restrict__ dh1, const float* __restrict__ loss_row, int B, int H,
                                    float* __restrict__ g_b1, float* __restrict__ g_w2, float* __restrict__ g_b2,
                                    float* __restrict__ loss) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < H) {
    float sb = 0.f, s0 = 0.f, s1 = 0.f;
    for (int b = 0; b < B; b++) {
      float av = a[(int64_t)b * H + j];
      sb += dh1[(int64_t)b * H + j];
      s0 += dz[2 * b] * av;
      s1 += dz[2 * b + 1] * av;
    }
    g_b1[j] = sb;
    g_w2[j] = s0;
    g_w2[H + j] = s1;
  }
  if (j == 0) {
    float d0 = 0.f, d1 = 0.f, l = 0.f;
    for (int b = 0; b < B; b++) {
      d0 += dz[2 * b];
      d1 += dz[2 * b + 1];
      l += loss_row[b];
    }
    g_b2[0] = d0;
    g_b2[1] = d1;
    if (loss) *loss = l / (float)B;
  }
}

hipError_t proxy_reduce(const float* a, const float* dz, const float* dh1, const float* loss_row, int B, int H,
                        float* g_b1, float* g_w2, float* g_b2, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(proxy_reduce_kernel, dim3((H + 255) / 256), dim3(256), 0, st, a, dz, dh1, loss_row, B, H, g_b1, g_w2,
                     g_b2, loss);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Adam
// p -= lr * mhat / (sqrt(vhat) + eps), mhat = m / (1 - b1^t), vhat = v / (1 - b2^t); the first
// n_w1 parameters (W1) are also written as BF16 for the next forward pass
__global__ void proxy_adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                  float* __restrict__ v, int64_t n, int64_t n_w1, bf16_t* __restrict__ w1b, float lr,
                                  float beta1, float beta2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = beta1 * m[i] + (1.f - beta1) * gi;
  float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (i < n_w1) w1b[i] = f2bf(pi);
}

hipError_t proxy_adam(float* p, const float* g, float* m, float* v, int64_t n, int64_t n_w1, bf16_t* w1b, float lr,
                      float beta1, float beta2, float eps, int step, hipStream_t st) {
  float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(proxy_adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, n_w1, w1b,
                     lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ s, bf16_t* __restrict__ d, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = f2bf(s[i]);
}
hipError_t f32_to_bf16(const float* s, bf16_t* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, d, n);
  return hipGetLastError();
}

}  // namespace kvop
