// Bandwidth-bound kernels around the projections and the attention: embedding gather,
// RMSNorm (FP32 statistics), rotary embedding, the cache writer of the prefill (with
// per-16-row FP8 block quantisation), pooled document features, the restricted logit
// heads, index-list validation and weight conversion.  One wavefront per row where a
// row reduction is needed; 16-byte accesses where the layout allows.
#include "common.h"
#include "kernels.h"

namespace kvop {

// ---------------------------------------------------------------- embedding
template <typename T>
__global__ void embed_kernel(const T* __restrict__ E, const int32_t* __restrict__ tok, int S, int n_rows, int d,
                             int vocab, float* __restrict__ x) {
  int row = blockIdx.x;
  if (row >= n_rows) return;
  int t = S > 0 ? tok[row % S] : tok[row];
  t = min(max(t, 0), vocab - 1);  // ids are validated by the callers; the clamp only guards the gather
  const T* e = E + (int64_t)t * d;
  float* o = x + (int64_t)row * d;
  for (int c = threadIdx.x; c < d; c += blockDim.x) o[c] = to_f32(e[c]);
}

hipError_t embed_rows(int dt, const void* E, const int32_t* tok, int n_rows, int d, int vocab, float* x,
                      hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  if (dt == DT_F32)
    hipLaunchKernelGGL(embed_kernel<float>, dim3(n_rows), dim3(256), 0, st, (const float*)E, tok, 0, n_rows, d, vocab, x);
  else
    hipLaunchKernelGGL(embed_kernel<bf16_t>, dim3(n_rows), dim3(256), 0, st, (const bf16_t*)E, tok, 0, n_rows, d, vocab, x);
  return hipGetLastError();
}

hipError_t embed_suffix(int dt, const void* E, const int32_t* suffix, int S, int n_rows, int d, int vocab, float* x,
                        hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  if (dt == DT_F32)
    hipLaunchKernelGGL(embed_kernel<float>, dim3(n_rows), dim3(256), 0, st, (const float*)E, suffix, S, n_rows, d, vocab, x);
  else
    hipLaunchKernelGGL(embed_kernel<bf16_t>, dim3(n_rows), dim3(256), 0, st, (const bf16_t*)E, suffix, S, n_rows, d, vocab, x);
  return hipGetLastError();
}

// ---------------------------------------------------------------- RMSNorm
// One wavefront per row.  Rows of up to 8 x 256 values stay in registers between the sum of
// squares and the scaling (one read of x); the output is written 4 values per lane per store.
template <typename TO>
__global__ __launch_bounds__(256) void rmsnorm_kernel(const float* __restrict__ x, int64_t ldx,
                                                      const float* __restrict__ g, int n_rows, int d, float eps,
                                                      TO* __restrict__ y, int64_t ldy) {
  int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (row >= n_rows) return;
  const float* xr = x + (int64_t)row * ldx;
  TO* yr = y + (int64_t)row * ldy;
  constexpr int KEEP = 8;                     // 16-byte pieces per lane kept in registers
  f32x4 keep[KEEP];
  float ss = 0.f;
#pragma unroll
  for (int it = 0; it < KEEP; it++) {
    const int c = lane * 4 + 256 * it;
    if (c < d) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(xr + c);
      keep[it] = v;
      ss += v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
    }
  }
  for (int c = lane * 4 + 256 * KEEP; c < d; c += 256) {
    f32x4 v = *reinterpret_cast<const f32x4*>(xr + c);
    ss += v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
  }
  ss = wave_sum(ss);
  float inv = 1.0f / sqrtf(ss / (float)d + eps);
  auto put = [&](int c, const f32x4& v) {
    const f32x4 gg = *reinterpret_cast<const f32x4*>(g + c);
    if constexpr (sizeof(TO) == 2) {
      u32x2 pk;
      pk[0] = pack_bf16x2(v[0] * inv * gg[0], v[1] * inv * gg[1]);
      pk[1] = pack_bf16x2(v[2] * inv * gg[2], v[3] * inv * gg[3]);
      *reinterpret_cast<u32x2*>(yr + c) = pk;
    } else {
      *reinterpret_cast<f32x4*>(yr + c) =
          f32x4{v[0] * inv * gg[0], v[1] * inv * gg[1], v[2] * inv * gg[2], v[3] * inv * gg[3]};
    }
  };
#pragma unroll
  for (int it = 0; it < KEEP; it++) {
    const int c = lane * 4 + 256 * it;
    if (c < d) put(c, keep[it]);
  }
  for (int c = lane * 4 + 256 * KEEP; c < d; c += 256) put(c, *reinterpret_cast<const f32x4*>(xr + c));
}

hipError_t rmsnorm_rows(int dt, const float* x, int64_t ldx, const float* g, int n_rows, int d, float eps, void* y,
                        int64_t ldy, hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  if (d % 4 || ldx % 4 || ldy % 4) return hipErrorInvalidValue;   // 16- and 8-byte row accesses
  dim3 grid((n_rows + 3) / 4);
  if (dt == DT_F32)
    hipLaunchKernelGGL(rmsnorm_kernel<float>, grid, dim3(256), 0, st, x, ldx, g, n_rows, d, eps, (float*)y, ldy);
  else
    hipLaunchKernelGGL(rmsnorm_kernel<bf16_t>, grid, dim3(256), 0, st, x, ldx, g, n_rows, d, eps, (bf16_t*)y, ldy);
  return hipGetLastError();
}

// ---------------------------------------------------------------- rotary embedding
// thread per (row, head, 8 consecutive pairs i..i+7): (x_i, x_{i+D/2}) ->
// (x_i c - x_{i+D/2} s, x_{i+D/2} c + x_i s), 16- or 32-byte accesses (D/2 a multiple of 8)
template <typename T> struct Vec8;
template <> struct Vec8<bf16_t> {
  __device__ static void load(const bf16_t* p, float* x) {
    const u32x4 v = *reinterpret_cast<const u32x4*>(p);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      x[2 * q] = bf2f((bf16_t)(v[q] & 0xffffu));
      x[2 * q + 1] = bf2f((bf16_t)(v[q] >> 16));
    }
  }
  __device__ static void store(bf16_t* p, const float* x) {
    u32x4 v;
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = pack_bf16x2(x[2 * q], x[2 * q + 1]);
    *reinterpret_cast<u32x4*>(p) = v;
  }
};
template <> struct Vec8<float> {
  __device__ static void load(const float* p, float* x) {
    const f32x4 a = *reinterpret_cast<const f32x4*>(p), b = *reinterpret_cast<const f32x4*>(p + 4);
#pragma unroll
    for (int q = 0; q < 4; q++) { x[q] = a[q]; x[4 + q] = b[q]; }
  }
  __device__ static void store(float* p, const float* x) {
    *reinterpret_cast<f32x4*>(p) = f32x4{x[0], x[1], x[2], x[3]};
    *reinterpret_cast<f32x4*>(p + 4) = f32x4{x[4], x[5], x[6], x[7]};
  }
};

template <typename T>
__global__ __launch_bounds__(256) void rope_kernel(T* __restrict__ qkv, int64_t ld, int n_rows, int n_heads, int H,
                                                   int D, const int32_t* __restrict__ pos,
                                                   const float* __restrict__ cos_t, const float* __restrict__ sin_t,
                                                   T* __restrict__ q_alt, const int32_t* __restrict__ shift) {
  const int half = D / 2, groups = half / 8;
  const int per_row = n_heads * groups;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= per_row * n_rows) return;
  const int row = gid / per_row, rem = gid - row * per_row;
  const int head = rem / groups, i = (rem - head * groups) * 8;
  T* v = qkv + (int64_t)row * ld + head * D;
  float x1[8], x2[8], c[8], s[8], y1[8], y2[8];
  Vec8<T>::load(v + i, x1);
  Vec8<T>::load(v + i + half, x2);
  const int p = pos[row];
  Vec8<float>::load(cos_t + (int64_t)p * half + i, c);
  Vec8<float>::load(sin_t + (int64_t)p * half + i, s);
  if (q_alt && head < H && shift[row] >= 0) {
    const int p2 = p - shift[row];
    float c2[8], s2[8];
    Vec8<float>::load(cos_t + (int64_t)p2 * half + i, c2);
    Vec8<float>::load(sin_t + (int64_t)p2 * half + i, s2);
#pragma unroll
    for (int e = 0; e < 8; e++) rope_pair(x1[e], x2[e], c2[e], s2[e], y1[e], y2[e]);
    T* va = q_alt + (int64_t)row * ld + head * D;
    Vec8<T>::store(va + i, y1);
    Vec8<T>::store(va + i + half, y2);
  }
#pragma unroll
  for (int e = 0; e < 8; e++) rope_pair(x1[e], x2[e], c[e], s[e], y1[e], y2[e]);
  Vec8<T>::store(v + i, y1);
  Vec8<T>::store(v + i + half, y2);
}

hipError_t rope_qk(int dt, void* qkv, int64_t ld, int n_rows, int H, int Hkv, int D, const int32_t* pos,
                   const float* cos_tab, const float* sin_tab, void* q_alt, const int32_t* alt_shift,
                   hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  if ((D / 2) % 8 || ld % 8) return hipErrorInvalidValue;
  const int64_t total = (int64_t)n_rows * (H + Hkv) * (D / 16);
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)((total + 255) / 256));
  if (dt == DT_F32)
    hipLaunchKernelGGL(rope_kernel<float>, grid, dim3(256), 0, st, (float*)qkv, ld, n_rows, H + Hkv, H, D, pos, cos_tab,
                       sin_tab, (float*)q_alt, alt_shift);
  else
    hipLaunchKernelGGL(rope_kernel<bf16_t>, grid, dim3(256), 0, st, (bf16_t*)qkv, ld, n_rows, H + Hkv, H, D, pos,
                       cos_tab, sin_tab, (bf16_t*)q_alt, alt_shift);
  return hipGetLastError();
}

// Rows of a batch that repeat every src_rows rows before the rotation (every item's rows are
// the same suffix at layer 0): each row is copied from its source row r mod src_rows, the
// query and key heads (columns below rot_cols) rotated at the row's own position with the
// arithmetic of the projection's rotary epilogue, so the rows equal what that epilogue writes
// bit for bit; joins also get the queries rotated at position - shift into q_alt.
__global__ __launch_bounds__(256) void rope_broadcast_kernel(const bf16_t* __restrict__ src, int src_rows,
                                                             bf16_t* __restrict__ dst, int64_t ld, int n_rows,
                                                             int n_cols, int rot_cols, int q_cols, int D,
                                                             const int32_t* __restrict__ pos,
                                                             const float* __restrict__ cos_t,
                                                             const float* __restrict__ sin_t, bf16_t* __restrict__ q_alt,
                                                             const int32_t* __restrict__ shift) {
  const int half = D / 2, gph = half / 8;
  const int per_row = (n_cols / D) * gph;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)per_row * n_rows) return;
  const int row = (int)(gid / per_row), rem = (int)(gid - (int64_t)row * per_row);
  const int hh = rem / gph, i = (rem - hh * gph) * 8, col = hh * D + i;
  const bf16_t* sp = src + (int64_t)(row % src_rows) * ld + col;
  const u32x4 r1 = *reinterpret_cast<const u32x4*>(sp), r2 = *reinterpret_cast<const u32x4*>(sp + half);
  bf16_t* o = dst + (int64_t)row * ld + col;
  if (col >= rot_cols) {
    *reinterpret_cast<u32x4*>(o) = r1;
    *reinterpret_cast<u32x4*>(o + half) = r2;
    return;
  }
  float x1[8], x2[8];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    x1[2 * q] = bf2f((bf16_t)(r1[q] & 0xffffu));
    x1[2 * q + 1] = bf2f((bf16_t)(r1[q] >> 16));
    x2[2 * q] = bf2f((bf16_t)(r2[q] & 0xffffu));
    x2[2 * q + 1] = bf2f((bf16_t)(r2[q] >> 16));
  }
  auto rotate_store = [&](int p, bf16_t* d) {
    float c[8], s[8], y1[8], y2[8];
    Vec8<float>::load(cos_t + (int64_t)p * half + i, c);
    Vec8<float>::load(sin_t + (int64_t)p * half + i, s);
#pragma unroll
    for (int e = 0; e < 8; e++) rope_pair(x1[e], x2[e], c[e], s[e], y1[e], y2[e]);
    Vec8<bf16_t>::store(d, y1);
    Vec8<bf16_t>::store(d + half, y2);
  };
  const int p = pos[row];
  if (q_alt && col < q_cols && shift[row] >= 0) rotate_store(p - shift[row], q_alt + (int64_t)row * ld + col);
  rotate_store(p, o);
}

hipError_t rope_broadcast(const void* src, int src_rows, void* dst, int64_t ld, int n_rows, int n_cols, int rot_cols,
                          int q_cols, int D, const int32_t* pos, const float* cos_tab, const float* sin_tab, void* q_alt,
                          const int32_t* shift, hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  if (src_rows < 1 || D % 16 || n_cols % D || ld % 8 || (q_alt && !shift)) return hipErrorInvalidValue;
  const int64_t total = (int64_t)n_rows * (n_cols / D) * (D / 16);
  hipLaunchKernelGGL(rope_broadcast_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     (const bf16_t*)src, src_rows, (bf16_t*)dst, ld, n_rows, n_cols, rot_cols, q_cols, D, pos, cos_tab,
                     sin_tab, (bf16_t*)q_alt, shift);
  return hipGetLastError();
}

// ---------------------------------------------------------------- cache writer (prefill)
// One workgroup per (16-row block of a document, kv head): rotate k of the block's rows
// at their positions, then store k and v into the document's region.  FP8 caches get one
// scale per block and per K/V: amax / 448 (1 for an all-zero block), codes = E4M3(x/scale).
template <typename T, typename TKV>
__global__ __launch_bounds__(256) void write_kv_kernel(const T* __restrict__ qkv, int64_t ld,
                                                       const KvBlock* __restrict__ blocks, int H, int Hkv, int D,
                                                       int layer, int n_layers, const float* __restrict__ cos_t,
                                                       const float* __restrict__ sin_t, uint8_t* __restrict__ pool) {
  __shared__ float kv_s[2][16][128 + 1];
  __shared__ float red[2][4];
  const KvBlock b = blocks[blockIdx.x];
  const int h = blockIdx.y, half = D / 2;
  const int nrow = min(16, b.L - b.p0);
  const int kcol = H * D + h * D, vcol = (H + Hkv) * D + h * D;
  float amax_k = 0.f, amax_v = 0.f;
  for (int e = threadIdx.x; e < 16 * half; e += 256) {
    int r = e / half, i = e % half;
    float k1 = 0.f, k2 = 0.f, v1 = 0.f, v2 = 0.f;
    if (r < nrow) {
      const T* row = qkv + (int64_t)(b.row0 + r) * ld;
      float x1 = to_f32(row[kcol + i]), x2 = to_f32(row[kcol + i + half]);
      int p = b.p0 + r;
      float c = cos_t[(int64_t)p * half + i], s = sin_t[(int64_t)p * half + i];
      rope_pair(x1, x2, c, s, k1, k2);
      v1 = to_f32(row[vcol + i]);
      v2 = to_f32(row[vcol + i + half]);
    }
    kv_s[0][r][i] = k1; kv_s[0][r][i + half] = k2;
    kv_s[1][r][i] = v1; kv_s[1][r][i + half] = v2;
    amax_k = fmaxf(amax_k, fmaxf(fabsf(k1), fabsf(k2)));
    amax_v = fmaxf(amax_v, fmaxf(fabsf(v1), fabsf(v2)));
  }
  float sc_k = 1.f, sc_v = 1.f;
  if constexpr (sizeof(TKV) == 1) {
    amax_k = wave_max(amax_k);
    amax_v = wave_max(amax_v);
    if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = amax_k; red[1][threadIdx.x >> 6] = amax_v; }
  }
  __syncthreads();
  if constexpr (sizeof(TKV) == 1) {
    float ak = fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]));
    float av = fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]));
    sc_k = ak == 0.f ? 1.f : ak / 448.0f;
    sc_v = av == 0.f ? 1.f : av / 448.0f;
  }
  const int64_t kv_elems = (int64_t)b.L * D;
  uint8_t* base = pool + b.off;
  TKV* kdst = reinterpret_cast<TKV*>(base) + ((int64_t)(layer * Hkv + h) * 2) * kv_elems;
  TKV* vdst = kdst + kv_elems;
  for (int e = threadIdx.x; e < nrow * D; e += 256) {
    int r = e / D, c = e % D;
    float kx = kv_s[0][r][c], vx = kv_s[1][r][c];
    int64_t o = (int64_t)(b.p0 + r) * D + c;
    if constexpr (sizeof(TKV) == 1) {
      kdst[o] = (fp8_t)f32_to_e4m3(kx / sc_k);
      vdst[o] = (fp8_t)f32_to_e4m3(vx / sc_v);
    } else {
      kdst[o] = from_f32<TKV>(kx);
      vdst[o] = from_f32<TKV>(vx);
    }
  }
  if constexpr (sizeof(TKV) == 1) {
    if (threadIdx.x == 0) {
      int nblk = (b.L + 15) >> 4;
      float* sb = reinterpret_cast<float*>(base + (int64_t)2 * n_layers * Hkv * kv_elems);
      float* ks = sb + ((int64_t)(layer * Hkv + h) * 2) * nblk;
      ks[b.p0 >> 4] = sc_k;
      ks[nblk + (b.p0 >> 4)] = sc_v;
    }
  }
}

hipError_t rope_write_kv(int dt, int kvdt, void* qkv, int64_t ld, const KvBlock* blocks, int n_blocks, int H,
                         int Hkv, int D, int layer, int n_layers, const float* cos_tab, const float* sin_tab,
                         uint8_t* pool, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (D > 128) return hipErrorInvalidValue;
  dim3 grid(n_blocks, Hkv);
  if (dt == DT_F32) {
    if (kvdt != DT_F32) return hipErrorInvalidValue;
    hipLaunchKernelGGL((write_kv_kernel<float, float>), grid, dim3(256), 0, st, (const float*)qkv, ld, blocks, H, Hkv, D,
                       layer, n_layers, cos_tab, sin_tab, pool);
  } else if (kvdt == DT_BF16) {
    hipLaunchKernelGGL((write_kv_kernel<bf16_t, bf16_t>), grid, dim3(256), 0, st, (const bf16_t*)qkv, ld, blocks, H,
                       Hkv, D, layer, n_layers, cos_tab, sin_tab, pool);
  } else if (kvdt == DT_FP8) {
    hipLaunchKernelGGL((write_kv_kernel<bf16_t, fp8_t>), grid, dim3(256), 0, st, (const bf16_t*)qkv, ld, blocks, H, Hkv,
                       D, layer, n_layers, cos_tab, sin_tab, pool);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- row copy (decode bookkeeping)
template <typename T>
__global__ void copy_rows_kernel(const T* __restrict__ src, int64_t ld, int col0, int n_cols,
                                 const int32_t* __restrict__ srow, const int32_t* __restrict__ drow, int n,
                                 T* __restrict__ dst, int64_t ldd) {
  int i = blockIdx.x;
  if (i >= n) return;
  const T* s = src + (int64_t)srow[i] * ld + col0;
  T* d = dst + (int64_t)drow[i] * ldd;
  for (int c = threadIdx.x; c < n_cols; c += blockDim.x) d[c] = s[c];
}

hipError_t copy_kv_rows(int dt, const void* qkv, int64_t ld, int kcol, int n_cols, const int32_t* src_rows,
                        const int32_t* dst_rows, int n, void* dst, int64_t ldd, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (dt == DT_F32)
    hipLaunchKernelGGL(copy_rows_kernel<float>, dim3(n), dim3(256), 0, st, (const float*)qkv, ld, kcol, n_cols, src_rows,
                       dst_rows, n, (float*)dst, ldd);
  else
    hipLaunchKernelGGL(copy_rows_kernel<bf16_t>, dim3(n), dim3(256), 0, st, (const bf16_t*)qkv, ld, kcol, n_cols,
                       src_rows, dst_rows, n, (bf16_t*)dst, ldd);
  return hipGetLastError();
}

// ---------------------------------------------------------------- pooled features
// pass 1: inverse RMS of every row; pass 2: per (document, 256-column slab) mean of x * inv * g
__global__ __launch_bounds__(256) void inv_rms_kernel(const float* __restrict__ x, int d, int n_rows, float eps,
                                                      float* __restrict__ inv) {
  int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n_rows) return;
  const float* xr = x + (int64_t)row * d;
  float ss = 0.f;
  for (int c = lane; c < d; c += 64) ss += xr[c] * xr[c];
  ss = wave_sum(ss);
  if (lane == 0) inv[row] = 1.0f / sqrtf(ss / (float)d + eps);
}

__global__ __launch_bounds__(256) void pooled_kernel(const float* __restrict__ x, int d,
                                                     const int64_t* __restrict__ row_off, const float* __restrict__ inv,
                                                     const float* __restrict__ g, float* __restrict__ pooled) {
  int doc = blockIdx.x, c = blockIdx.y * 256 + threadIdx.x;
  if (c >= d) return;
  int64_t r0 = row_off[doc], r1 = row_off[doc + 1];
  float acc = 0.f;
  for (int64_t r = r0; r < r1; r++) acc += x[r * d + c] * inv[r];
  pooled[(int64_t)doc * d + c] = acc * g[c] / (float)(r1 - r0);
}

hipError_t pooled_mean(const float* x, int d, const int64_t* row_off, int n_docs, int n_rows, const float* g,
                       float eps, float* inv_scratch, float* pooled, hipStream_t st) {
  if (n_docs <= 0) return hipSuccess;
  hipLaunchKernelGGL(inv_rms_kernel, dim3((n_rows + 3) / 4), dim3(256), 0, st, x, d, n_rows, eps, inv_scratch);
  hipLaunchKernelGGL(pooled_kernel, dim3(n_docs, (d + 255) / 256), dim3(256), 0, st, x, d, row_off, inv_scratch, g,
                     pooled);
  return hipGetLastError();
}

// ---------------------------------------------------------------- logit heads
// one workgroup per item: y = rmsnorm(x_row) * g kept in LDS (FP32), then dot products with
// the requested head rows, reduced in FP32
template <typename T>
__global__ __launch_bounds__(256) void head_filter_kernel(const float* __restrict__ x, int64_t ldx, int d,
                                                          const float* __restrict__ g, float eps,
                                                          const T* __restrict__ W, int yes_id, int no_id, float thp,
                                                          float thn, const int32_t* __restrict__ in_rows,
                                                          const int32_t* __restrict__ out_rows,
                                                          float* __restrict__ logits, int8_t* __restrict__ decision) {
  __shared__ float red[3][4];
  int item = blockIdx.x;
  const float* xr = x + (int64_t)(in_rows ? in_rows[item] : item) * ldx;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float ss = 0.f;
  for (int c = threadIdx.x; c < d; c += 256) ss += xr[c] * xr[c];
  ss = wave_sum(ss);
  if (lane == 0) red[0][wv] = ss;
  __syncthreads();
  float tot = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  float inv = 1.0f / sqrtf(tot / (float)d + eps);
  const T* wy = W + (int64_t)yes_id * d;
  const T* wn = W + (int64_t)no_id * d;
  float ay = 0.f, an = 0.f;
  for (int c = threadIdx.x; c < d; c += 256) {
    float y = xr[c] * inv * g[c];
    ay += y * to_f32(wy[c]);
    an += y * to_f32(wn[c]);
  }
  ay = wave_sum(ay);
  an = wave_sum(an);
  if (lane == 0) { red[1][wv] = ay; red[2][wv] = an; }
  __syncthreads();
  if (threadIdx.x == 0) {
    float ly = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    float ln = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    const int64_t o = out_rows[item];
    logits[2 * o] = ly;
    logits[2 * o + 1] = ln;
    float lo = ly - ln;
    if (decision) decision[o] = lo > thp ? 1 : (lo < thn ? 0 : -1);
  }
}

hipError_t head_filter(int dt, const float* x, int64_t ldx, int n_items, int d, const float* g, float eps,
                       const void* head, int yes_id, int no_id, float th_pos, float th_neg, const int32_t* in_rows,
                       const int32_t* out_rows, float* logits, int8_t* decision, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (dt == DT_F32)
    hipLaunchKernelGGL(head_filter_kernel<float>, dim3(n_items), dim3(256), 0, st, x, ldx, d, g, eps,
                       (const float*)head, yes_id, no_id, th_pos, th_neg, in_rows, out_rows, logits, decision);
  else
    hipLaunchKernelGGL(head_filter_kernel<bf16_t>, dim3(n_items), dim3(256), 0, st, x, ldx, d, g, eps,
                       (const bf16_t*)head, yes_id, no_id, th_pos, th_neg, in_rows, out_rows, logits, decision);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void head_map_kernel(const float* __restrict__ x, int64_t ldx, int d,
                                                       const float* __restrict__ g, float eps,
                                                       const T* __restrict__ W, int lo, int n,
                                                       const int32_t* __restrict__ in_rows,
                                                       const int32_t* __restrict__ out_rows,
                                                       float* __restrict__ logits, int64_t ldl,
                                                       int32_t* __restrict__ tok_out, int64_t ldt,
                                                       int32_t* __restrict__ next_tok, bool next_by_out) {
  extern __shared__ __attribute__((aligned(16))) float ysm[];   // d floats, then n logits
  __shared__ float red[4];
  __shared__ int redi[4];
  int item = blockIdx.x;
  const float* xr = x + (int64_t)(in_rows ? in_rows[item] : item) * ldx;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float ss = 0.f;
  for (int c = threadIdx.x; c < d; c += 256) ss += xr[c] * xr[c];
  ss = wave_sum(ss);
  if (lane == 0) red[wv] = ss;
  __syncthreads();
  float inv = 1.0f / sqrtf((red[0] + red[1] + red[2] + red[3]) / (float)d + eps);
  for (int c = threadIdx.x; c < d; c += 256) ysm[c] = xr[c] * inv * g[c];
  __syncthreads();
  float* zl = ysm + d;
  // four head rows per wavefront at a time, eight consecutive values per lane and load, so
  // that a lane keeps four independent 16-byte (BF16) loads in flight per step
  for (int j0 = 4 * wv; j0 < n; j0 += 16) {
    float a[4] = {0.f, 0.f, 0.f, 0.f};
    for (int c = 8 * lane; c < d; c += 512) {
      float yv[8], wvv[4][8];
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (j0 + q < n) Vec8<T>::load(W + (int64_t)(lo + j0 + q) * d + c, wvv[q]);
      const f32x4 y0 = *reinterpret_cast<const f32x4*>(ysm + c), y1 = *reinterpret_cast<const f32x4*>(ysm + c + 4);
#pragma unroll
      for (int t = 0; t < 4; t++) { yv[t] = y0[t]; yv[4 + t] = y1[t]; }
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (j0 + q < n) {
#pragma unroll
          for (int t = 0; t < 8; t++) a[q] += yv[t] * wvv[q][t];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const float v = wave_sum(a[q]);
      if (lane == 0 && j0 + q < n) zl[j0 + q] = v;
    }
  }
  __syncthreads();
  // argmax, lowest index on ties
  float best = -INFINITY;
  int bi = 0x7fffffff;
  const int64_t orow = out_rows[item];
  for (int j = threadIdx.x; j < n; j += 256) {
    float v = zl[j];
    logits[orow * ldl + j] = v;
    if (v > best || (v == best && j < bi)) { best = v; bi = j; }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    float ob = __shfl_xor(best, o, 64);
    int oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  if (lane == 0) { red[wv] = best; redi[wv] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = red[0];
    int i = redi[0];
    for (int k = 1; k < 4; k++)
      if (red[k] > b || (red[k] == b && redi[k] < i)) { b = red[k]; i = redi[k]; }
    tok_out[orow * ldt] = lo + i;
    if (next_tok) next_tok[next_by_out ? orow : item] = lo + i;
  }
}

hipError_t head_map(int dt, const float* x, int64_t ldx, int n_items, int d, const float* g, float eps,
                    const void* head, int lo, int n, const int32_t* in_rows, const int32_t* out_rows, float* logits,
                    int64_t ld_logits, int32_t* tok_out, int64_t ld_tok, int32_t* next_tok, bool next_by_out,
                    hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (d % 8) return hipErrorInvalidValue;     // eight-value row pieces
  size_t lds = (size_t)(d + n) * sizeof(float);
  if (dt == DT_F32)
    hipLaunchKernelGGL(head_map_kernel<float>, dim3(n_items), dim3(256), lds, st, x, ldx, d, g, eps, (const float*)head,
                       lo, n, in_rows, out_rows, logits, ld_logits, tok_out, ld_tok, next_tok, next_by_out);
  else
    hipLaunchKernelGGL(head_map_kernel<bf16_t>, dim3(n_items), dim3(256), lds, st, x, ldx, d, g, eps,
                       (const bf16_t*)head, lo, n, in_rows, out_rows, logits, ld_logits, tok_out, ld_tok, next_tok, next_by_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- validation
__global__ __launch_bounds__(256) void validate_kernel(const int32_t* __restrict__ idx,
                                                       const ListCheck* __restrict__ lists, int n_lists,
                                                       int* __restrict__ bad) {
  int li = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (li >= n_lists) return;
  ListCheck l = lists[li];
  int ok = 1;
  for (int i = lane; i < l.n; i += 64) {
    int v = idx[l.off + i];
    if (v < 0 || v >= l.L) ok = 0;
    if (i > 0 && idx[l.off + i - 1] >= v) ok = 0;
  }
  ok = __all(ok);
  if (lane == 0 && !ok) atomicAdd(bad, 1);
}

hipError_t validate_lists(const int32_t* idx, const ListCheck* lists, int n_lists, int* bad, hipStream_t st) {
  if (n_lists <= 0) return hipSuccess;
  hipLaunchKernelGGL(validate_kernel, dim3((n_lists + 3) / 4), dim3(256), 0, st, idx, lists, n_lists, bad);
  return hipGetLastError();
}

// Token ids outside [0, vocab): one count per wavefront that saw any.
__global__ __launch_bounds__(256) void validate_tokens_kernel(const int32_t* __restrict__ tok, int64_t n, int vocab,
                                                              int* __restrict__ bad) {
  int ok = 1;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    int t = tok[i];
    if (t < 0 || t >= vocab) ok = 0;
  }
  ok = __all(ok);
  if ((threadIdx.x & 63) == 0 && !ok) atomicAdd(bad, 1);
}

hipError_t validate_tokens(const int32_t* tok, int64_t n, int vocab, int* bad, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(validate_tokens_kernel, dim3((unsigned)blocks), dim3(256), 0, st, tok, n, vocab, bad);
  return hipGetLastError();
}

// ---------------------------------------------------------------- weights
template <typename T>
__global__ void convert_kernel(const float* __restrict__ src, const float* __restrict__ src2, int64_t rows,
                               int64_t cols, T* __restrict__ dst, int inter) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t out_rows = inter ? 2 * rows : rows;
  if (i >= out_rows * cols) return;
  int64_t r = i / cols, c = i % cols;
  float v;
  if (inter) {
    int64_t blk = r / 32, e = r % 32;
    v = e < 16 ? src[(blk * 16 + e) * cols + c] : src2[(blk * 16 + e - 16) * cols + c];
  } else {
    v = src[i];
  }
  dst[i] = from_f32<T>(v);
}

hipError_t convert_weights(int dt, const float* src, const float* src2, int64_t rows, int64_t cols, void* dst,
                           int interleave16, hipStream_t st) {
  int64_t total = (interleave16 ? 2 * rows : rows) * cols;
  if (total <= 0) return hipSuccess;
  if (interleave16 && rows % 16) return hipErrorInvalidValue;
  dim3 grid((unsigned)((total + 255) / 256));
  if (dt == DT_F32)
    hipLaunchKernelGGL(convert_kernel<float>, grid, dim3(256), 0, st, src, src2, rows, cols, (float*)dst, interleave16);
  else
    hipLaunchKernelGGL(convert_kernel<bf16_t>, grid, dim3(256), 0, st, src, src2, rows, cols, (bf16_t*)dst, interleave16);
  return hipGetLastError();
}

template <typename TKV>
__global__ void read_cache_kernel(const uint8_t* __restrict__ region, int L, int D, int layer, int n_layers, int Hkv,
                                  int h, int kv, float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)L * D) return;
  const int64_t kv_elems = (int64_t)L * D;
  const TKV* src = reinterpret_cast<const TKV*>(region) + ((int64_t)(layer * Hkv + h) * 2 + kv) * kv_elems;
  if constexpr (sizeof(TKV) == 1) {
    int nblk = (L + 15) >> 4;
    const float* sb = reinterpret_cast<const float*>(region + (int64_t)2 * n_layers * Hkv * kv_elems);
    float sc = sb[((int64_t)(layer * Hkv + h) * 2 + kv) * nblk + (i / D) / 16];
    out[i] = e4m3_to_f32(src[i]) * sc;
  } else {
    out[i] = to_f32(src[i]);
  }
}

hipError_t read_cache(int kvdt, const uint8_t* region, int L, int D, int layer, int n_layers, int Hkv, int h, int kv,
                      float* out, hipStream_t st) {
  int64_t n = (int64_t)L * D;
  dim3 grid((unsigned)((n + 255) / 256));
  if (kvdt == DT_F32)
    hipLaunchKernelGGL(read_cache_kernel<float>, grid, dim3(256), 0, st, region, L, D, layer, n_layers, Hkv, h, kv, out);
  else if (kvdt == DT_BF16)
    hipLaunchKernelGGL(read_cache_kernel<bf16_t>, grid, dim3(256), 0, st, region, L, D, layer, n_layers, Hkv, h, kv, out);
  else
    hipLaunchKernelGGL(read_cache_kernel<fp8_t>, grid, dim3(256), 0, st, region, L, D, layer, n_layers, Hkv, h, kv, out);
  return hipGetLastError();
}

__global__ void fill_kernel(int32_t* p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

}  // namespace kvop
