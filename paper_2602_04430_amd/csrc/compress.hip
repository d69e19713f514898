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
// eight consecutive elements as floats (16-byte aligned for BF16, 32-byte for FP32)
__device__ inline void ld8(const float* p, float (&x)[8]) {
  const f32x4 a = *reinterpret_cast<const f32x4*>(p), b = *reinterpret_cast<const f32x4*>(p + 4);
#pragma unroll
  for (int i = 0; i < 4; i++) { x[i] = a[i]; x[i + 4] = b[i]; }
}
__device__ inline void ld8(const bf16_t* p, float (&x)[8]) {
  const u32x4 v = *reinterpret_cast<const u32x4*>(p);
#pragma unroll
  for (int i = 0; i < 4; i++) {
    x[2 * i] = __builtin_bit_cast(float, v[i] << 16);
    x[2 * i + 1] = __builtin_bit_cast(float, v[i] & 0xffff0000u);
  }
}

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
                                                             const int64_t* __restrict__ row_off,
                                                             const int32_t* __restrict__ items, int n_future,
                                                             const float* __restrict__ cos_tab,
                                                             const float* __restrict__ sin_tab,
                                                             float* __restrict__ e_out) {
  constexpr int BR = D / 32, BC = D / 8, H2 = D / 2;
  __shared__ __attribute__((aligned(16))) float region[D * D > kEaChunk * D ? D * D : kEaChunk * D];  // S, or rows
  __shared__ float mu[D], mur[D], cb[H2], sb[H2];
  // work item: (document, first key, key count); the statistics always cover all the
  // document's rows, the keys are this item's segment
  const int32_t* it = items + 3 * (blockIdx.x / H);
  const int doc = it[0], k_lo = it[1], k_hi = it[1] + it[2], h = blockIdx.x % H, g = (h * Hkv) / H;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t r0 = row_off[doc];
  const int L = (int)(row_off[doc + 1] - r0);
  const T* Q = qkv + r0 * ld + (int64_t)h * D;
  const T* Kp = qkv + r0 * ld + (int64_t)(H + g) * D;
  const int a0 = w * (D / 4) + (lane >> 3) * BR, b0 = (lane & 7) * BC;

  // mean of the pre-rotation queries (FP32 path: a pass of its own, each dimension's rows
  // split over 256 / D threads; the BF16 path sums the rows it stages for the covariance)
  if constexpr (sizeof(T) == 4) {
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
  // covariance into region (float [D][D])
  const float invL = 1.0f / (float)L;
  if constexpr (sizeof(T) == 2) {
    // BF16 queries: S = sum over rows of q q^T on MFMA (exact products, FP32 sums) from a
    // transposed LDS tile (tile[d][r] = q[c0 + r][d], pitch 40 so that the 16 rows one
    // fragment read touches fall on distinct banks), then S / L - mu mu^T
    constexpr int NB = D / 16, PK = 40, NBW = NB * NB / 4, DG = D / 8;
    static_assert(NBW * 4 == NB * NB, "output blocks per wavefront");
    bf16_t* tile = reinterpret_cast<bf16_t*>(region);
    f32x4 cacc[NBW];
#pragma unroll
    for (int j = 0; j < NBW; j++) cacc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int sr = tid >> 3, sd = (tid & 7) * DG;   // staging: row, first dimension
    float colsum[DG];
#pragma unroll
    for (int u = 0; u < DG; u++) colsum[u] = 0.f;
    for (int c0 = 0; c0 < L; c0 += 32) {
      bf16_t v[DG];
      if (c0 + sr < L) {
        const bf16_t* src = Q + (int64_t)(c0 + sr) * ld + sd;
#pragma unroll
        for (int u = 0; u < DG; u += 4) {
          const u32x2 x = *reinterpret_cast<const u32x2*>(src + u);
          v[u] = (bf16_t)(x[0] & 0xffff);
          v[u + 1] = (bf16_t)(x[0] >> 16);
          v[u + 2] = (bf16_t)(x[1] & 0xffff);
          v[u + 3] = (bf16_t)(x[1] >> 16);
        }
      } else {
#pragma unroll
        for (int u = 0; u < DG; u++) v[u] = 0;
      }
#pragma unroll
      for (int u = 0; u < DG; u++) {
        tile[(sd + u) * PK + sr] = v[u];
        colsum[u] += bf2f(v[u]);
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NBW; j++) {
        const int bi = w * NBW + j, br = bi / NB, bc = bi % NB;
        const u32x4 fa = *reinterpret_cast<const u32x4*>(tile + (br * 16 + (lane & 15)) * PK + 8 * (lane >> 4));
        const u32x4 fb = *reinterpret_cast<const u32x4*>(tile + (bc * 16 + (lane & 15)) * PK + 8 * (lane >> 4));
        cacc[j] = mfma_bf16(__builtin_bit_cast(u16x8, fa), __builtin_bit_cast(u16x8, fb), cacc[j]);
      }
      __syncthreads();
    }
    // mean: the 32 staging threads of each dimension group add their column sums
    float* part = region + D * PK / 2;   // past the tile (floats)
#pragma unroll
    for (int u = 0; u < DG; u++) part[sr * D + sd + u] = colsum[u];
    __syncthreads();
    if (tid < D) {
      float t = 0.f;
      for (int q = 0; q < 32; q++) t += part[q * D + tid];
      mu[tid] = t * invL;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NBW; j++) {
      const int bi = w * NBW + j, br = bi / NB, bc = bi % NB;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int ra = br * 16 + 4 * (lane >> 4) + r, rb = bc * 16 + (lane & 15);
        region[ra * D + rb] = cacc[j][r] * invL - mu[ra] * mu[rb];
      }
    }
  } else {
    // FP32 queries: centred products on the vector ALU, accumulated in the lane's block
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
#pragma unroll
    for (int a = 0; a < BR; a++)
#pragma unroll
      for (int b = 0; b < BC; b++) region[(a0 + a) * D + b0 + b] = acc[a][b] * invL;
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
  __syncthreads();  // covariance reads done before the region holds keys
  // expected log-weight of every rotated key: one key per lane (256 per pass), its rotated
  // values in registers; S_r rows are read from LDS by all lanes at once (broadcast), so no
  // cross-lane reduction is needed
  const float inv_sqrt_d = rsqrtf((float)D), inv_2d = 0.5f / (float)D;
  for (int c0 = k_lo; c0 < k_hi; c0 += kEaThreads) {
    const int p = c0 + tid;
    float k[D];
    if (p < k_hi) {
      const T* kr = Kp + (int64_t)p * ld;
      const float* ct = cos_tab + (int64_t)p * H2;
      const float* st = sin_tab + (int64_t)p * H2;
#pragma unroll
      for (int j = 0; j < H2; j += 8) {
        float x1[8], x2[8];
        ld8(kr + j, x1);
        ld8(kr + j + H2, x2);
#pragma unroll
        for (int u = 0; u < 8; u += 4) {
          const f32x4 cs = *reinterpret_cast<const f32x4*>(ct + j + u);
          const f32x4 sn = *reinterpret_cast<const f32x4*>(st + j + u);
#pragma unroll
          for (int v = 0; v < 4; v++) {
            k[j + u + v] = x1[u + v] * cs[v] - x2[u + v] * sn[v];
            k[j + u + v + H2] = x2[u + v] * cs[v] + x1[u + v] * sn[v];
          }
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < D; j++) k[j] = 0.f;
    }
    float e = 0.f;
#pragma unroll 1
    for (int blk = 0; blk < D / 8; blk++) {
      float ka[8];
#pragma unroll
      for (int c = 0; c < D / 8; c++)   // blk is uniform: one branch taken, no indexed registers
        if (c == blk) {
#pragma unroll
          for (int u = 0; u < 8; u++) ka[u] = k[8 * c + u];
        }
      // the block's eight rows of S_r k as eight independent FMA chains (S_r rows: broadcast
      // LDS reads)
      const float* sr = region + 8 * blk * D;
      float y[8];
#pragma unroll
      for (int u = 0; u < 8; u++) y[u] = 0.f;
#pragma unroll
      for (int b = 0; b < D; b += 4) {
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const f32x4 s4 = *reinterpret_cast<const f32x4*>(sr + u * D + b);
          y[u] = fmaf(s4[0], k[b], y[u]);
          y[u] = fmaf(s4[1], k[b + 1], y[u]);
          y[u] = fmaf(s4[2], k[b + 2], y[u]);
          y[u] = fmaf(s4[3], k[b + 3], y[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 8; u++) e = fmaf(ka[u], fmaf(y[u], inv_2d, mur[8 * blk + u] * inv_sqrt_d), e);
    }
    if (p < k_hi) e_out[(r0 + p) * H + h] = e;
  }
}

// ---------------------------------------------------------------- contributions
template <typename T, int D>
__global__ __launch_bounds__(kEaThreads) void ea_contrib_kernel(const T* __restrict__ qkv, int64_t ld, int H, int Hkv,
                                                                const int64_t* __restrict__ row_off,
                                                                const int32_t* __restrict__ order,
                                                                const float* __restrict__ e_in,
                                                                float* __restrict__ acc) {
  __shared__ float red[4];
  __shared__ float mx[64], zs[64];
  const int doc = order[blockIdx.x / Hkv], g = blockIdx.x % Hkv, G = H / Hkv;
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
hipError_t ea_layer_t(const void* qkv, int64_t ld, int H, int Hkv, const int64_t* row_off, const int32_t* order,
                      int nd, const int32_t* items, int n_items, int n_future, const float* cos_tab,
                      const float* sin_tab, float* e_ws, float* acc, hipStream_t st) {
  hipLaunchKernelGGL((ea_logw_kernel<T, D>), dim3(n_items * H), dim3(kEaThreads), 0, st, (const T*)qkv, ld, H, Hkv,
                     row_off, items, n_future, cos_tab, sin_tab, e_ws);
  hipLaunchKernelGGL((ea_contrib_kernel<T, D>), dim3(nd * Hkv), dim3(kEaThreads), 0, st, (const T*)qkv, ld, H, Hkv,
                     row_off, order, (const float*)e_ws, acc);
  return hipGetLastError();
}

}  // namespace

hipError_t ea_layer(int dt, int D, const void* qkv, int64_t ld, int H, int Hkv, const int64_t* row_off,
                    const int32_t* order, int nd, const int32_t* items, int n_items, int n_future,
                    const float* cos_tab, const float* sin_tab, float* e_ws, float* acc, hipStream_t st) {
  if (nd <= 0) return hipSuccess;
  if (H % Hkv || H / Hkv > 64) return hipErrorInvalidValue;
  if (dt == DT_F32) {
    if (D == 128) return ea_layer_t<float, 128>(qkv, ld, H, Hkv, row_off, order, nd, items, n_items, n_future, cos_tab, sin_tab, e_ws, acc, st);
    if (D == 64) return ea_layer_t<float, 64>(qkv, ld, H, Hkv, row_off, order, nd, items, n_items, n_future, cos_tab, sin_tab, e_ws, acc, st);
    if (D == 32) return ea_layer_t<float, 32>(qkv, ld, H, Hkv, row_off, order, nd, items, n_items, n_future, cos_tab, sin_tab, e_ws, acc, st);
  } else {
    if (D == 128) return ea_layer_t<bf16_t, 128>(qkv, ld, H, Hkv, row_off, order, nd, items, n_items, n_future, cos_tab, sin_tab, e_ws, acc, st);
    if (D == 64) return ea_layer_t<bf16_t, 64>(qkv, ld, H, Hkv, row_off, order, nd, items, n_items, n_future, cos_tab, sin_tab, e_ws, acc, st);
    if (D == 32) return ea_layer_t<bf16_t, 32>(qkv, ld, H, Hkv, row_off, order, nd, items, n_items, n_future, cos_tab, sin_tab, e_ws, acc, st);
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
