// Grouped-query attention of a block of query rows over gathered cached rows plus the
// item's own (suffix / generated) rows, with an online softmax in FP32.
//
// One workgroup = one work item x one kv head.  Its query rows are the G query heads of
// that kv head times up to Pmax positions (row r -> head r / Pmax, position r % Pmax);
// each wavefront owns 16 of them.  Keys stream through LDS in tiles of KT rows taken, in
// order, from: document A's cached rows (contiguous or through a retained-row index list),
// document B's cached rows (joins: positions shifted by L_A; the matching queries are
// rotated at position - L_A), and the own rows.  A key is visible to a query iff its
// position is <= the query's position, which expresses both prefill causality and the
// suffix's view of (all retained rows) + (earlier suffix rows).
//
// MFMA layout: scores are computed transposed, S^T = K Q^T, so every accumulator a lane
// holds belongs to the same query (column lane % 16).  Softmax rescaling is then a
// per-lane scalar and the probabilities are already in the B-operand layout of the
// second product O^T = V^T P^T.  FP32 path: v_mfma_f32_16x16x4f32 with K and V row-major
// in LDS.  BF16 path: v_mfma_f32_16x16x32_bf16 with V stored transposed in LDS; FP8
// (E4M3) cache rows are widened to BF16 exactly while staging and their per-16-row FP32
// block scales are applied to the scores (K) and to the probabilities (V).
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace kvop {

template <typename TC, int D>
struct AttnCfg {
  static constexpr bool F32 = std::is_same<TC, float>::value;
  static constexpr int KT = F32 ? 32 : 64;       // keys per tile
  static constexpr int KPAD = F32 ? 4 : 8;       // LDS row padding (elements)
  static constexpr int KLD = D + KPAD;           // K row pitch (and V row pitch for f32)
  static constexpr int VTLD = KT + 8;            // transposed V row pitch (bf16)
  static constexpr int KS_ELEMS = KT * KLD;
  static constexpr int VS_ELEMS = F32 ? KT * KLD : D * VTLD;
};

// Stage one tile of keys (rows t0 .. t0+KT-1 of a source) into LDS.
//   src_k/src_v : element pointers of row 0 of the source (row pitch `pitch` elements)
//   idx         : retained-row list of the source or null (then row = t0 + j)
//   n           : rows in the source; rows past n are marked invisible
//   clampL      : rows are clamped to [0, clampL) as a guard against bad lists
//   pos_add     : key position = row + pos_add
//   ksc/vsc     : FP8 block scales of the source (per 16 rows) or null
template <typename TC, typename TS, int D, int NT>
__device__ inline void stage_tile(TC* __restrict__ Ks, TC* __restrict__ Vs, float* ksc_s, float* vsc_s,
                                  int* kpos_s, const TS* __restrict__ src_k, const TS* __restrict__ src_v,
                                  int64_t pitch, const int32_t* __restrict__ idx, int t0, int n, int clampL,
                                  int pos_add, const float* __restrict__ ksc, const float* __restrict__ vsc) {
  using C = AttnCfg<TC, D>;
  constexpr int KT = C::KT;
  const int tid = threadIdx.x;
  // row ids, positions and scales of this tile
  for (int j = tid; j < KT; j += NT) {
    int t = t0 + j;
    int row = 0, pos = 0x7fffffff;
    float ks = 1.f, vs = 1.f;
    if (t < n) {
      row = idx ? idx[t] : t;
      row = min(max(row, 0), clampL - 1);
      pos = row + pos_add;
      if (ksc) { ks = ksc[row >> 4]; vs = vsc[row >> 4]; }
    }
    kpos_s[j] = pos;
    ksc_s[j] = ks;
    vsc_s[j] = vs;
  }
  __syncthreads();
  constexpr int CPR = D * (int)sizeof(TS) / 16;  // 16-byte chunks per source row
  if constexpr (C::F32) {
    // f32 source into row-major K and V tiles
    for (int c = tid; c < KT * CPR; c += NT) {
      int j = c / CPR, cc = c % CPR;
      int t = t0 + j;
      u32x4 kv = {0, 0, 0, 0}, vv = {0, 0, 0, 0};
      if (t < n) {
        int row = kpos_s[j] - pos_add;
        kv = *reinterpret_cast<const u32x4*>(src_k + row * pitch + cc * 4);
        vv = *reinterpret_cast<const u32x4*>(src_v + row * pitch + cc * 4);
      }
      *reinterpret_cast<u32x4*>(Ks + j * C::KLD + cc * 4) = kv;
      *reinterpret_cast<u32x4*>(Vs + j * C::KLD + cc * 4) = vv;
    }
  } else {
    // K: row-major bf16
    for (int c = tid; c < KT * CPR; c += NT) {
      int j = c / CPR, cc = c % CPR;
      int t = t0 + j;
      u32x4 raw = {0, 0, 0, 0};
      if (t < n) {
        int row = kpos_s[j] - pos_add;
        raw = *reinterpret_cast<const u32x4*>(reinterpret_cast<const uint8_t*>(src_k + row * pitch) + cc * 16);
      }
      if constexpr (sizeof(TS) == 2) {
        *reinterpret_cast<u32x4*>(Ks + j * C::KLD + cc * 8) = raw;
      } else {  // 16 E4M3 codes -> 16 bf16
        u32x4 lo, hi;
#pragma unroll
        for (int w = 0; w < 4; w++) {
          uint32_t x = raw[w];
          uint32_t b0 = e4m3_to_bf16(x & 0xff), b1 = e4m3_to_bf16((x >> 8) & 0xff);
          uint32_t b2 = e4m3_to_bf16((x >> 16) & 0xff), b3 = e4m3_to_bf16(x >> 24);
          if (w < 2) { lo[2 * w] = b0 | (b1 << 16); lo[2 * w + 1] = b2 | (b3 << 16); }
          else { hi[2 * (w - 2)] = b0 | (b1 << 16); hi[2 * (w - 2) + 1] = b2 | (b3 << 16); }
        }
        *reinterpret_cast<u32x4*>(Ks + j * C::KLD + cc * 16) = lo;
        *reinterpret_cast<u32x4*>(Ks + j * C::KLD + cc * 16 + 8) = hi;
      }
    }
    // V: transposed bf16, two keys per thread so that each LDS write is a packed dword
    constexpr int EPC = 16 / (int)sizeof(TS);     // elements per chunk
    for (int c = tid; c < (KT / 2) * CPR; c += NT) {
      int jp = c / CPR, cc = c % CPR;
      int j0 = 2 * jp;
      u32x4 r0 = {0, 0, 0, 0}, r1 = {0, 0, 0, 0};
      if (t0 + j0 < n) {
        int row = kpos_s[j0] - pos_add;
        r0 = *reinterpret_cast<const u32x4*>(reinterpret_cast<const uint8_t*>(src_v + row * pitch) + cc * 16);
      }
      if (t0 + j0 + 1 < n) {
        int row = kpos_s[j0 + 1] - pos_add;
        r1 = *reinterpret_cast<const u32x4*>(reinterpret_cast<const uint8_t*>(src_v + row * pitch) + cc * 16);
      }
      uint32_t* vt = reinterpret_cast<uint32_t*>(Vs);
#pragma unroll
      for (int e = 0; e < EPC; e++) {
        uint32_t a, b;
        if constexpr (sizeof(TS) == 2) {
          a = (r0[e >> 1] >> ((e & 1) * 16)) & 0xffff;
          b = (r1[e >> 1] >> ((e & 1) * 16)) & 0xffff;
        } else {
          a = e4m3_to_bf16((r0[e >> 2] >> ((e & 3) * 8)) & 0xff);
          b = e4m3_to_bf16((r1[e >> 2] >> ((e & 3) * 8)) & 0xff);
        }
        int d = cc * EPC + e;
        vt[(d * C::VTLD + j0) >> 1] = a | (b << 16);
      }
    }
  }
}

template <typename TC, typename TKV, int D, int NW>
__global__ __launch_bounds__(NW * 64) void attn_kernel(AttnArgs a) {
  using C = AttnCfg<TC, D>;
  constexpr int KT = C::KT;
  constexpr int NT = NW * 64;
  constexpr int NB = KT / 16;                    // 16-key blocks per tile
  constexpr int ND = D / 16;                     // 16-wide d blocks of the output
  __shared__ __attribute__((aligned(16))) TC Ks[C::KS_ELEMS];
  __shared__ __attribute__((aligned(16))) TC Vs[C::VS_ELEMS];
  __shared__ float ksc_s[KT], vsc_s[KT];
  __shared__ int kpos_s[KT];

  const AttnWork w = a.work[blockIdx.x];
  const int h = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qi = lane & 15, g4 = lane >> 4;
  const int r = wave * 16 + qi;
  const int gq = r / a.Pmax, p = r % a.Pmax;
  const bool qvalid = gq < a.G && p < w.n_q;
  const int hq = h * a.G + (gq < a.G ? gq : 0);
  const int qpos = w.q_pos0 + p;
  const int64_t qrow = (int64_t)w.q_row0 + (qvalid ? p : 0);

  // ---- query fragments (B operand of S^T = K Q^T)
  constexpr int NQ = C::F32 ? D / 16 : D / 32;
  u32x4 qf[NQ], qa[NQ];
  const bool has_b = w.n_b > 0;
  {
    const TC* q = reinterpret_cast<const TC*>(a.q) + qrow * a.q_stride + hq * D;
    const TC* q2 = reinterpret_cast<const TC*>(a.q_alt ? a.q_alt : a.q) + qrow * a.q_stride + hq * D;
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      int d0 = C::F32 ? 16 * k + 4 * g4 : 32 * k + 8 * g4;
      qf[k] = qvalid ? *reinterpret_cast<const u32x4*>(q + d0) : u32x4{0, 0, 0, 0};
      qa[k] = (qvalid && has_b) ? *reinterpret_cast<const u32x4*>(q2 + d0) : u32x4{0, 0, 0, 0};
    }
  }

  float m_run = -INFINITY, l_run = 0.f;
  f32x4 o[ND];
#pragma unroll
  for (int i = 0; i < ND; i++) o[i] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int Hkv = a.Hkv;
  constexpr bool FP8 = sizeof(TKV) == 1;
  // three key sources: 0 = document A, 1 = document B, 2 = own rows
  for (int src = 0; src < 3; src++) {
    int n = src == 0 ? w.n_a : (src == 1 ? w.n_b : w.n_own);
    // document B is scored with the queries rotated at (position - L_A): swap them in for
    // source 1 and back afterwards (register moves; no dynamically indexed arrays)
    if (src >= 1 && has_b) {
#pragma unroll
      for (int k = 0; k < NQ; k++) {
        u32x4 tmp = qf[k];
        qf[k] = qa[k];
        qa[k] = tmp;
      }
    }
    if (n <= 0) continue;
    for (int t0 = 0; t0 < n; t0 += KT) {
      __syncthreads();  // previous tile fully consumed
      if (src < 2) {
        int64_t off = src == 0 ? w.off_a : w.off_b;
        int L = src == 0 ? w.L_a : w.L_b;
        int64_t il = src == 0 ? w.idx_a : w.idx_b;
        const uint8_t* base = a.pool + off;
        int64_t kv_elems = (int64_t)L * D;
        int64_t head_off = ((int64_t)(a.layer * Hkv + h) * 2) * kv_elems;  // elements
        const TKV* kp = reinterpret_cast<const TKV*>(base) + head_off;
        const TKV* vp = kp + kv_elems;
        const float *ks = nullptr, *vs = nullptr;
        if constexpr (FP8) {
          int nblk = (L + 15) >> 4;
          const float* sb = reinterpret_cast<const float*>(base + (int64_t)2 * a.n_layers * Hkv * kv_elems);
          ks = sb + ((int64_t)(a.layer * Hkv + h) * 2) * nblk;
          vs = ks + nblk;
        }
        stage_tile<TC, TKV, D, NT>(Ks, Vs, ksc_s, vsc_s, kpos_s, kp, vp, D, il >= 0 ? a.idx + il : nullptr, t0, n, L,
                                   src == 1 ? w.L_a : 0, ks, vs);
      } else {
        const TC* ob = reinterpret_cast<const TC*>(a.own) + (int64_t)w.own_row0 * a.own_stride;
        stage_tile<TC, TC, D, NT>(Ks, Vs, ksc_s, vsc_s, kpos_s, ob + a.own_kcol + h * D, ob + a.own_vcol + h * D,
                                  a.own_stride, nullptr, t0, n, n, w.own_pos0, nullptr, nullptr);
      }
      __syncthreads();

      // ---- scores S^T[key][query]: lane holds keys 16*b + 4*g4 + t of query column qi
      f32x4 s[NB];
#pragma unroll
      for (int b = 0; b < NB; b++) {
        s[b] = f32x4{0.f, 0.f, 0.f, 0.f};
        const TC* krow = Ks + (16 * b + qi) * C::KLD;
#pragma unroll
        for (int k = 0; k < NQ; k++) {
          if constexpr (C::F32) {
            u32x4 kf = *reinterpret_cast<const u32x4*>(krow + 16 * k + 4 * g4);
#pragma unroll
            for (int t = 0; t < 4; t++)
              s[b] = mfma_f32(as_f32(kf[t]), as_f32(qf[k][t]), s[b]);
          } else {
            u32x4 kf = *reinterpret_cast<const u32x4*>(krow + 32 * k + 8 * g4);
            s[b] = mfma_bf16(__builtin_bit_cast(u16x8, kf), __builtin_bit_cast(u16x8, qf[k]), s[b]);
          }
        }
      }
      // ---- mask, scale, online softmax (statistics in FP32)
      float mx = -INFINITY;
#pragma unroll
      for (int b = 0; b < NB; b++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
          int key = 16 * b + 4 * g4 + t;
          bool vis = qvalid && kpos_s[key] <= qpos;
          float v = s[b][t] * a.scale_log2;
          if constexpr (FP8) v *= ksc_s[key];
          v = vis ? v : -INFINITY;
          s[b][t] = v;
          mx = fmaxf(mx, v);
        }
      mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
      mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
      const float m_new = fmaxf(m_run, mx);
      const float alpha = (m_new == -INFINITY) ? 1.f : exp2f(m_run - m_new);
      float psum = 0.f;
#pragma unroll
      for (int b = 0; b < NB; b++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
          float pv = (s[b][t] == -INFINITY) ? 0.f : exp2f(s[b][t] - m_new);
          s[b][t] = pv;
          psum += pv;
        }
      l_run = l_run * alpha + psum;
      m_run = m_new;
#pragma unroll
      for (int i = 0; i < ND; i++) o[i] *= alpha;

      // ---- O^T[d][query] += V^T[d][key] P^T[key][query]
      if constexpr (C::F32) {
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
          for (int t = 0; t < 4; t++) {
            const float* vrow = Vs + (16 * b + 4 * g4 + t) * C::KLD;
#pragma unroll
            for (int i = 0; i < ND; i++) o[i] = mfma_f32(vrow[16 * i + qi], s[b][t], o[i]);
          }
      } else {
#pragma unroll
        for (int b2 = 0; b2 < NB / 2; b2++) {
          u16x8 pb;
#pragma unroll
          for (int t = 0; t < 4; t++) {
            float p0 = s[2 * b2][t], p1 = s[2 * b2 + 1][t];
            if constexpr (FP8) {
              p0 *= vsc_s[32 * b2 + 4 * g4 + t];
              p1 *= vsc_s[32 * b2 + 16 + 4 * g4 + t];
            }
            pb[t] = f2bf(p0);
            pb[4 + t] = f2bf(p1);
          }
#pragma unroll
          for (int i = 0; i < ND; i++) {
            const bf16_t* vt = Vs + (16 * i + qi) * C::VTLD + 32 * b2 + 4 * g4;
            u32x2 lo = *reinterpret_cast<const u32x2*>(vt);
            u32x2 hi = *reinterpret_cast<const u32x2*>(vt + 16);
            u32x4 va = {lo[0], lo[1], hi[0], hi[1]};
            o[i] = mfma_bf16(__builtin_bit_cast(u16x8, va), pb, o[i]);
          }
        }
      }
    }
  }

  // ---- normalise and store: lane holds O[query qi][d = 16*i + 4*g4 + t]
  float l_tot = l_run + __shfl_xor(l_run, 16, 64);
  l_tot += __shfl_xor(l_tot, 32, 64);
  if (!qvalid) return;
  const float inv = l_tot > 0.f ? 1.f / l_tot : 0.f;
  TC* out = reinterpret_cast<TC*>(a.out) + qrow * a.out_stride + hq * D;
#pragma unroll
  for (int i = 0; i < ND; i++) {
    int d0 = 16 * i + 4 * g4;
    if constexpr (C::F32) {
      *reinterpret_cast<f32x4*>(out + d0) = o[i] * inv;
    } else {
      u32x2 pk;
      pk[0] = (uint32_t)f2bf(o[i][0] * inv) | ((uint32_t)f2bf(o[i][1] * inv) << 16);
      pk[1] = (uint32_t)f2bf(o[i][2] * inv) | ((uint32_t)f2bf(o[i][3] * inv) << 16);
      *reinterpret_cast<u32x2*>(out + d0) = pk;
    }
  }
}

template <typename TC, typename TKV, int D>
static hipError_t launch_d(const AttnArgs& a, hipStream_t st) {
  int rows = a.G * a.Pmax;
  dim3 grid(a.n_work, a.Hkv);
  if (rows <= 16)
    hipLaunchKernelGGL((attn_kernel<TC, TKV, D, 1>), grid, dim3(64), 0, st, a);
  else if (rows <= 32)
    hipLaunchKernelGGL((attn_kernel<TC, TKV, D, 2>), grid, dim3(128), 0, st, a);
  else
    hipLaunchKernelGGL((attn_kernel<TC, TKV, D, 4>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename TC, typename TKV>
static hipError_t launch_kv(int D, const AttnArgs& a, hipStream_t st) {
  switch (D) {
    case 32: return launch_d<TC, TKV, 32>(a, st);
    case 64: return launch_d<TC, TKV, 64>(a, st);
    case 128: return launch_d<TC, TKV, 128>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t attention(int cdt, int kvdt, int D, const AttnArgs& a, hipStream_t st) {
  if (a.n_work <= 0) return hipSuccess;
  if (a.G * a.Pmax > 64 || a.G < 1 || a.Pmax < 1) return hipErrorInvalidValue;
  if (cdt == DT_F32) {
    if (kvdt != DT_F32) return hipErrorInvalidValue;
    return launch_kv<float, float>(D, a, st);
  }
  if (kvdt == DT_BF16) return launch_kv<bf16_t, bf16_t>(D, a, st);
  if (kvdt == DT_FP8) return launch_kv<bf16_t, fp8_t>(D, a, st);
  return hipErrorInvalidValue;
}

}  // namespace kvop
