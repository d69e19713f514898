// Query-agnostic cache compression by expected attention: the offline choice of the rows a
// compressed cache profile keeps (Section 2.3; Section 5, "Offline").  Runs inside kv_build,
// per layer, on the pre-rotation queries, keys and values the QKV projection just produced.
//
// Per (document, query head): the document's queries define a Gaussian (mean mu, population
// covariance S); the rotation averaged over the n positions after the document (L .. L+n-1)
// maps it to mu_r = R mu, S_r = R S R^T; every rotated key k of the head's kv head gets the
// expected log-weight  mu_r.k / sqrt(D) + k^T S_r k / (2 D)  (the Gaussian's moment generating
// function at k / sqrt(D)).  Per (document, kv head): softmax of those over the document's keys,
// times the value norm, averaged over the group's query heads, normalised to total 1 and added
// to the row's running score (one accumulator per (row, kv head): no atomics, the result does
// not depend on scheduling).  Selection: per document, the k highest scores (equal scores:
// lower row first) listed in ascending row order, by a radix select over the score bits.
//
// Work layout of the log-weight kernel (256 threads = 4 wavefronts): the D x D covariance is
// split so that wavefront w owns rows [w D/4, (w+1) D/4) and lane l an (D/32) x (D/8) block
// (rows by l / 8, columns by l % 8): D = 128 gives 64 accumulators per lane.  Each document
// row (query, then key) is staged in LDS as floats; a lane reads D/32 + D/8 of its values per
// row and does (D/32)(D/8) FMAs.  The covariance then goes through LDS once to apply the
// averaged rotation (each output element combines at most four inputs: the rotation mixes
// dimension j only with j +- D/2).
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace kvop {

namespace {

constexpr int kEaThreads = 256;
constexpr int kEaChunk = 64;  // document rows staged in LDS at a time

template <typename T>
__device__ inline float ld_f(const T* p);
template <>
__device__ inline float ld_f<float>(const float* p) { return *p; }
template <>
__device__ inline float ld_f<bf16_t>(const bf16_t* p) { return bf2f(*p); }

__device__ inline float block_sum(float v, float* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}
__device__ inline float block_max(float v, float* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// ---------------------------------------------------------------- expected log-weights
template <typename T, int D>
__global__ __launch_bounds__(kEaThreads) void ea_logw_kernel(const T* __restrict__ qkv, int64_t ld, int H, int Hkv,
                                                             const int64_t* __restrict__ row_off, int n_future,
                                                             const float* __restrict__ cos_tab,
                                                             const float* __restrict__ sin_tab,
                                                             float* __restrict__ e_out) {
  constexpr int BR = D / 32, BC = D / 8, H2 = D / 2;
  __shared__ float region[D * D > kEaChunk * D ? D * D : kEaChunk * D];  // covariance, or staged rows
  __shared__ float mu[D], mur[D], cb[H2], sb[H2];
  __shared__ float red[4][kEaChunk];
  const int doc = blockIdx.x / H, h = blockIdx.x % H, g = (h * Hkv) / H;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t r0 = row_off[doc];
  const int L = (int)(row_off[doc + 1] - r0);
  const T* Q = qkv + r0 * ld + (int64_t)h * D;
  const T* Kp = qkv + r0 * ld + (int64_t)(H + g) * D;
  const int a0 = w * (D / 4) + (lane >> 3) * BR, b0 = (lane & 7) * BC;

  // mean of the pre-rotation queries (each dimension's rows split over 256 / D threads)
  {
    constexpr int SPLIT = kEaThreads / D;
    const int j = tid % D, part = tid / D;
    float s = 0.f;
#pragma unroll 4
    for (int i = part; i < L; i += SPLIT) s += ld_f(Q + (int64_t)i * ld + j);
    region[tid] = s;
    __syncthreads();
    if (tid < D) {
      float t = 0.f;
      for (int q = 0; q < SPLIT; q++) t += region[q * D + tid];
      mu[tid] = t / (float)L;
    }
    __syncthreads();
  }
  // covariance (centred products), accumulated in the lane's block
  float acc[BR][BC];
#pragma unroll
  for (int a = 0; a < BR; a++)
#pragma unroll
    for (int b = 0; b < BC; b++) acc[a][b] = 0.f;
  for (int c0 = 0; c0 < L; c0 += kEaChunk) {
    for (int e = tid; e < kEaChunk * D; e += kEaThreads) {
      const int i = e / D, j = e % D;
      region[e] = (c0 + i < L) ? ld_f(Q + (int64_t)(c0 + i) * ld + j) - mu[j] : 0.f;
    }
    __syncthreads();
    const int n = min(kEaChunk, L - c0);
#pragma unroll 1
    for (int i = 0; i < n; i++) {
      const float* x = region + i * D;
      float xa[BR], xb[BC];
#pragma unroll
      for (int a = 0; a < BR; a++) xa[a] = x[a0 + a];
#pragma unroll
      for (int b = 0; b < BC; b++) xb[b] = x[b0 + b];
#pragma unroll
      for (int a = 0; a < BR; a++)
#pragma unroll
        for (int b = 0; b < BC; b++) acc[a][b] = fmaf(xa[a], xb[b], acc[a][b]);
    }
    __syncthreads();
  }
  // averaged rotation over the future positions, and the rotated mean
  if (tid < H2) {
    float c = 0.f, s = 0.f;
    for (int p = L; p < L + n_future; p++) {
      c += cos_tab[(int64_t)p * H2 + tid];
      s += sin_tab[(int64_t)p * H2 + tid];
    }
    cb[tid] = c / (float)n_future;
    sb[tid] = s / (float)n_future;
  }
  const float invL = 1.0f / (float)L;
#pragma unroll
  for (int a = 0; a < BR; a++)
#pragma unroll
    for (int b = 0; b < BC; b++) region[(a0 + a) * D + b0 + b] = acc[a][b] * invL;
  __syncthreads();
  if (tid < D) {
    const int j = tid % H2;
    mur[tid] = tid < H2 ? cb[j] * mu[tid] - sb[j] * mu[tid + H2] : sb[j] * mu[j] + cb[j] * mu[tid];
  }
  // S_r = R S R^T in place, one 2x2 quad (a, a + D/2) x (b, b + D/2) at a time: the rotation
  // mixes dimension j only with j + D/2, so a quad's four outputs depend only on its inputs
  for (int qd = tid; qd < H2 * H2; qd += kEaThreads) {
    const int qa = qd / H2, qb = qd % H2;
    float* r0p = region + qa * D;
    float* r1p = region + (qa + H2) * D;
    const float s00 = r0p[qb], s01 = r0p[qb + H2], s10 = r1p[qb], s11 = r1p[qb + H2];
    const float ca = cb[qa], sa = sb[qa], cc = cb[qb], sc = sb[qb];
    const float t00 = ca * s00 - sa * s10, t01 = ca * s01 - sa * s11;  // rows: R S
    const float t10 = sa * s00 + ca * s10, t11 = sa * s01 + ca * s11;
    r0p[qb] = cc * t00 - sc * t01;                                     // columns: (R S) R^T
    r0p[qb + H2] = sc * t00 + cc * t01;
    r1p[qb] = cc * t10 - sc * t11;
    r1p[qb + H2] = sc * t10 + cc * t11;
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < BR; a++)
#pragma unroll
    for (int b = 0; b < BC; b++) acc[a][b] = region[(a0 + a) * D + b0 + b];
  __syncthreads();  // covariance reads done before the region holds keys
  // expected log-weight of every rotated key
  const float inv_sqrt_d = rsqrtf((float)D), inv_2d = 0.5f / (float)D;
  for (int c0 = 0; c0 < L; c0 += kEaChunk) {
    for (int e = tid; e < kEaChunk * H2; e += kEaThreads) {
      const int i = e / H2, j = e % H2, p = c0 + i;
      float k1 = 0.f, k2 = 0.f;
      if (p < L) {
        const float x1 = ld_f(Kp + (int64_t)p * ld + j), x2 = ld_f(Kp + (int64_t)p * ld + j + H2);
        const float cs = cos_tab[(int64_t)p * H2 + j], sn = sin_tab[(int64_t)p * H2 + j];
        k1 = x1 * cs - x2 * sn;
        k2 = x2 * cs + x1 * sn;
      }
      region[i * D + j] = k1;
      region[i * D + j + H2] = k2;
    }
    __syncthreads();
    const int n = min(kEaChunk, L - c0);
#pragma unroll 1
    for (int i = 0; i < n; i++) {
      const float* k = region + i * D;
      float kb[BC];
#pragma unroll
      for (int b = 0; b < BC; b++) kb[b] = k[b0 + b];
      float part = 0.f;
#pragma unroll
      for (int a = 0; a < BR; a++) {
        float y = 0.f;
#pragma unroll
        for (int b = 0; b < BC; b++) y = fmaf(acc[a][b], kb[b], y);
        const float ka = k[a0 + a];
        part = fmaf(ka, y * inv_2d, part);
        if ((lane & 7) == 0) part = fmaf(ka, mur[a0 + a] * inv_sqrt_d, part);
      }
      part = wave_sum(part);
      if (lane == 0) red[w][i] = part;
    }
    __syncthreads();
    if (tid < n) e_out[(r0 + c0 + tid) * H + h] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- contributions
template <typename T, int D>
__global__ __launch_bounds__(kEaThreads) void ea_contrib_kernel(const T* __restrict__ qkv, int64_t ld, int H, int Hkv,
                                                                const int64_t* __restrict__ row_off,
                                                                const float* __restrict__ e_in,
                                                                float* __restrict__ acc) {
  __shared__ float red[4];
  __shared__ float mx[64], zs[64];
  const int doc = blockIdx.x / Hkv, g = blockIdx.x % Hkv, G = H / Hkv;
  const int tid = threadIdx.x;
  const int64_t r0 = row_off[doc];
  const int L = (int)(row_off[doc + 1] - r0);
  const T* V = qkv + r0 * ld + (int64_t)(H + Hkv + g) * D;
  for (int q = 0; q < G; q++) {
    const int h = g * G + q;
    float m = -INFINITY;
    for (int i = tid; i < L; i += kEaThreads) m = fmaxf(m, e_in[(r0 + i) * H + h]);
    m = block_max(m, red);
    float z = 0.f;
    for (int i = tid; i < L; i += kEaThreads) z += __expf(e_in[(r0 + i) * H + h] - m);
    z = block_sum(z, red);
    if (tid == 0) { mx[q] = m; zs[q] = z; }
  }
  __syncthreads();
  auto contrib = [&](int i) {
    float vn = 0.f;
    for (int j = 0; j < D; j++) {
      const float x = ld_f(V + (int64_t)i * ld + j);
      vn = fmaf(x, x, vn);
    }
    float wsum = 0.f;
    for (int q = 0; q < G; q++) wsum += __expf(e_in[(r0 + i) * H + g * G + q] - mx[q]) / zs[q];
    return wsum / (float)G * sqrtf(vn);
  };
  float tot = 0.f;
  for (int i = tid; i < L; i += kEaThreads) tot += contrib(i);
  tot = block_sum(tot, red);
  for (int i = tid; i < L; i += kEaThreads)
    acc[(r0 + i) * Hkv + g] += tot > 0.f ? contrib(i) / tot : 1.0f / (float)L;
}

__global__ void ea_finish_kernel(const float* __restrict__ acc, int Hkv, int rows, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  float s = 0.f;
  for (int g = 0; g < Hkv; g++) s += acc[(int64_t)i * Hkv + g];
  out[i] = s;
}

__global__ void ea_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------- selection
// float -> unsigned key with the same order (all finite values and infinities)
__device__ inline uint32_t order_key(float f) {
  const uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// exclusive prefix sum over the block (256 threads); returns the block total in *total
__device__ inline int block_scan(int v, int* total, int* wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0;
  for (int k = 0; k < w; k++) before += wsum[k];
  *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  return before + x - v;
}

__global__ __launch_bounds__(kEaThreads) void ea_select_kernel(const float* __restrict__ scores,
                                                               const int64_t* __restrict__ doc_off,
                                                               const int32_t* __restrict__ kcount,
                                                               const int64_t* __restrict__ out_off,
                                                               int32_t* __restrict__ idx) {
  __shared__ int wsum[4];
  __shared__ float red[4];
  const int d = blockIdx.x, tid = threadIdx.x;
  const int64_t s0 = doc_off[d];
  const int L = (int)(doc_off[d + 1] - s0), k = kcount[d];
  int32_t* out = idx + out_off[d];
  if (k >= L) {
    for (int i = tid; i < L; i += kEaThreads) out[i] = i;
    return;
  }
  // largest t with #(key >= t) >= k, bit by bit from the top
  uint32_t t = 0;
  for (int bit = 31; bit >= 0; bit--) {
    const uint32_t cand = t | (1u << bit);
    int c = 0;
    for (int i = tid; i < L; i += kEaThreads) c += order_key(scores[s0 + i]) >= cand ? 1 : 0;
    if ((int)block_sum((float)c, red) >= k) t = cand;  // counts stay below 2^24: exact in float
  }
  int gt = 0;
  for (int i = tid; i < L; i += kEaThreads) gt += order_key(scores[s0 + i]) > t ? 1 : 0;
  const int need = k - (int)block_sum((float)gt, red);  // rows equal to t still to take, >= 1
  int eq_before = 0, out_before = 0;
  for (int c0 = 0; c0 < L; c0 += kEaThreads) {
    const int i = c0 + tid;
    const uint32_t key = i < L ? order_key(scores[s0 + i]) : 0u;
    const int eq = (i < L && key == t) ? 1 : 0;
    int eq_tot;
    const int eq_rank = eq_before + block_scan(eq, &eq_tot, wsum);
    const int take = (i < L && (key > t || (eq && eq_rank < need))) ? 1 : 0;
    int take_tot;
    const int pos = out_before + block_scan(take, &take_tot, wsum);
    if (take) out[pos] = i;
    eq_before += eq_tot;
    out_before += take_tot;
    __syncthreads();
  }
}

template <typename T, int D>
hipError_t ea_layer_t(const void* qkv, int64_t ld, int H, int Hkv, const int64_t* row_off, int nd, int n_future,
                      const float* cos_tab, const float* sin_tab, float* e_ws, float* acc, hipStream_t st) {
  hipLaunchKernelGGL((ea_logw_kernel<T, D>), dim3(nd * H), dim3(kEaThreads), 0, st, (const T*)qkv, ld, H, Hkv,
                     row_off, n_future, cos_tab, sin_tab, e_ws);
  hipLaunchKernelGGL((ea_contrib_kernel<T, D>), dim3(nd * Hkv), dim3(kEaThreads), 0, st, (const T*)qkv, ld, H, Hkv,
                     row_off, (const float*)e_ws, acc);
  return hipGetLastError();
}

}  // namespace

hipError_t ea_layer(int dt, int D, const void* qkv, int64_t ld, int H, int Hkv, const int64_t* row_off, int nd,
                    int n_future, const float* cos_tab, const float* sin_tab, float* e_ws, float* acc,
                    hipStream_t st) {
  if (nd <= 0) return hipSuccess;
  if (H % Hkv || H / Hkv > 64) return hipErrorInvalidValue;
  if (dt == DT_F32) {
    if (D == 128) return ea_layer_t<float, 128>(qkv, ld, H, Hkv, row_off, nd, n_future, cos_tab, sin_tab, e_ws, acc, st);
    if (D == 64) return ea_layer_t<float, 64>(qkv, ld, H, Hkv, row_off, nd, n_future, cos_tab, sin_tab, e_ws, acc, st);
    if (D == 32) return ea_layer_t<float, 32>(qkv, ld, H, Hkv, row_off, nd, n_future, cos_tab, sin_tab, e_ws, acc, st);
  } else {
    if (D == 128) return ea_layer_t<bf16_t, 128>(qkv, ld, H, Hkv, row_off, nd, n_future, cos_tab, sin_tab, e_ws, acc, st);
    if (D == 64) return ea_layer_t<bf16_t, 64>(qkv, ld, H, Hkv, row_off, nd, n_future, cos_tab, sin_tab, e_ws, acc, st);
    if (D == 32) return ea_layer_t<bf16_t, 32>(qkv, ld, H, Hkv, row_off, nd, n_future, cos_tab, sin_tab, e_ws, acc, st);
  }
  return hipErrorInvalidValue;
}

hipError_t ea_zero(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ea_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t ea_finish(const float* acc, int Hkv, int rows, float* out, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(ea_finish_kernel, dim3((rows + 255) / 256), dim3(256), 0, st, acc, Hkv, rows, out);
  return hipGetLastError();
}

hipError_t ea_select(const float* scores, const int64_t* doc_off, const int32_t* kcount, const int64_t* out_off,
                     int n_docs, int32_t* idx, hipStream_t st) {
  if (n_docs <= 0) return hipSuccess;
  hipLaunchKernelGGL(ea_select_kernel, dim3(n_docs), dim3(kEaThreads), 0, st, scores, doc_off, kcount, out_off, idx);
  return hipGetLastError();
}

}  // namespace kvop
