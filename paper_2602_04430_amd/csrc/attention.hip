// Grouped-query attention of a block of query rows over gathered cached rows plus the
// item's own (suffix / generated) rows, with an online softmax in FP32.
//
// One workgroup (4 wavefronts) = one work item x one kv head.  Its query rows are the G
// query heads of that kv head times up to Pmax positions (row r -> head r / Pmax, position
// r % Pmax); each wavefront owns 16 of them (wavefronts without rows only help staging).  Keys stream through LDS in tiles of KT rows taken, in
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
#include <algorithm>
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

// One key source of a work item: rows of a cached document (through an optional retained
// list) or the item's own rows.  All threads of the workgroup hold the same description.
struct KeySrc {
  const uint8_t* k;      // row 0 of the keys
  const uint8_t* v;      // row 0 of the values
  int64_t pitch;         // bytes between consecutive rows
  const int32_t* idx;    // retained-row list or null (rows 0..n-1)
  const float* ksc;      // FP8 block scales (per 16 rows) or null
  const float* vsc;
  int n, clampL, pos_add;
  bool cache;            // cache dtype (else compute dtype)
};

// Register-staged tile of KT keys: each thread fetches its share of 16-byte chunks from
// global memory (fetch), then writes them to LDS, widening FP8 and transposing V for the
// BF16 path (commit).  The fetch of tile i+1 is issued before the compute of tile i.
template <typename TC, typename TKV, int D>
struct TileStage {
  using C = AttnCfg<TC, D>;
  static constexpr int KT = C::KT;
  static constexpr int NT = 256;
  static constexpr int CPR = D * (int)sizeof(TC) / 16;           // chunks per row in the compute dtype
  static constexpr int NK = (KT * CPR + NT - 1) / NT;             // K chunks per thread
  static constexpr int NVU = C::F32 ? NK : ((KT / 2) * CPR + NT - 1) / NT;  // V units per thread
  u32x4 kr[NK];
  u32x4 vr0[NVU], vr1[NVU];
  int kpos[NK];
  float ks[NK], vs[NK];
  bool fp8;                                                      // this tile came from an FP8 source

  __device__ static int row_of(const KeySrc& s, int t) {
    int row = s.idx ? s.idx[t] : t;
    return min(max(row, 0), s.clampL - 1);
  }

  __device__ void fetch(const KeySrc& s, int t0) {
    const int tid = threadIdx.x;
    fp8 = (sizeof(TKV) == 1) && s.cache;
    // an FP8 row is half as many 16-byte chunks; the widened K chunk covers 16 elements
    const int cpr_src = fp8 ? CPR / 2 : CPR;
#pragma unroll
    for (int i = 0; i < NK; i++) {
      int c = tid + i * NT;
      int j = c / CPR, cc = c % CPR;
      int t = t0 + j;
      kr[i] = u32x4{0, 0, 0, 0};
      kpos[i] = 0x7fffffff;
      ks[i] = 1.f;
      vs[i] = 1.f;
      if (c < KT * CPR && t < s.n) {
        int row = row_of(s, t);
        kpos[i] = row + s.pos_add;
        if (fp8) {
          ks[i] = s.ksc[row >> 4];
          vs[i] = s.vsc[row >> 4];
        }
        if (cc < cpr_src) kr[i] = *reinterpret_cast<const u32x4*>(s.k + row * s.pitch + cc * 16);
        if constexpr (C::F32) vr0[i] = *reinterpret_cast<const u32x4*>(s.v + row * s.pitch + cc * 16);
      } else if constexpr (C::F32) {
        vr0[i] = u32x4{0, 0, 0, 0};
      }
    }
    if constexpr (!C::F32) {
#pragma unroll
      for (int i = 0; i < NVU; i++) {
        int u = tid + i * NT;
        int jp = u / CPR, cc = u % CPR;
        int t = t0 + 2 * jp;
        vr0[i] = u32x4{0, 0, 0, 0};
        vr1[i] = u32x4{0, 0, 0, 0};
        if (u < (KT / 2) * CPR && cc < cpr_src) {
          if (t < s.n) vr0[i] = *reinterpret_cast<const u32x4*>(s.v + row_of(s, t) * s.pitch + cc * 16);
          if (t + 1 < s.n) vr1[i] = *reinterpret_cast<const u32x4*>(s.v + row_of(s, t + 1) * s.pitch + cc * 16);
        }
      }
    }
  }

  __device__ void commit(TC* __restrict__ Ks, TC* __restrict__ Vs, float* ksc_s, float* vsc_s, int* kpos_s) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NK; i++) {
      int c = tid + i * NT;
      int j = c / CPR, cc = c % CPR;
      if (c >= KT * CPR) continue;
      if (cc == 0) {
        kpos_s[j] = kpos[i];
        ksc_s[j] = ks[i];
        vsc_s[j] = vs[i];
      }
      if constexpr (C::F32) {
        *reinterpret_cast<u32x4*>(Ks + j * C::KLD + cc * 4) = kr[i];
        *reinterpret_cast<u32x4*>(Vs + j * C::KLD + cc * 4) = vr0[i];
      } else {
        if (!fp8) {
          *reinterpret_cast<u32x4*>(Ks + j * C::KLD + cc * 8) = kr[i];
        } else if (cc < CPR / 2) {  // 16 codes -> 16 bf16 (elements 16 cc .. 16 cc + 15)
          u32x4 lo, hi;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            uint32_t x = kr[i][q];
            uint32_t b0 = e4m3_to_bf16(x & 0xff), b1 = e4m3_to_bf16((x >> 8) & 0xff);
            uint32_t b2 = e4m3_to_bf16((x >> 16) & 0xff), b3 = e4m3_to_bf16(x >> 24);
            if (q < 2) { lo[2 * q] = b0 | (b1 << 16); lo[2 * q + 1] = b2 | (b3 << 16); }
            else { hi[2 * (q - 2)] = b0 | (b1 << 16); hi[2 * (q - 2) + 1] = b2 | (b3 << 16); }
          }
          *reinterpret_cast<u32x4*>(Ks + j * C::KLD + cc * 16) = lo;
          *reinterpret_cast<u32x4*>(Ks + j * C::KLD + cc * 16 + 8) = hi;
        }
      }
    }
    if constexpr (!C::F32) {
      // transposed V: element (d, key) at dword d * VTLD/2 + (key/2 ^ swz(d)), swz(d) = 2*((d/16)&7),
      // so the 16 lanes of one store (16 different d blocks) hit 16 different banks
      uint32_t* vt = reinterpret_cast<uint32_t*>(Vs);
#pragma unroll
      for (int i = 0; i < NVU; i++) {
        int u = tid + i * NT;
        int jp = u / CPR, cc = u % CPR;
        if (u >= (KT / 2) * CPR) continue;
        if (!fp8) {
#pragma unroll
          for (int e = 0; e < 8; e++) {
            const int d = cc * 8 + e;
            vt[d * (C::VTLD / 2) + (jp ^ (2 * ((d >> 4) & 7)))] = pair_halves(vr0[i][e >> 1], vr1[i][e >> 1], e & 1);
          }
        } else if (cc < CPR / 2) {
#pragma unroll
          for (int e = 0; e < 16; e++) {
            const int d = cc * 16 + e;
            uint32_t a = e4m3_to_bf16((vr0[i][e >> 2] >> ((e & 3) * 8)) & 0xff);
            uint32_t b = e4m3_to_bf16((vr1[i][e >> 2] >> ((e & 3) * 8)) & 0xff);
            vt[d * (C::VTLD / 2) + (jp ^ (2 * ((d >> 4) & 7)))] = a | (b << 16);
          }
        }
      }
    }
  }
};

template <typename TC, int D>
struct AttnSmem {
  using C = AttnCfg<TC, D>;
  __attribute__((aligned(16))) TC Ks[C::KS_ELEMS];
  __attribute__((aligned(16))) TC Vs[C::VS_ELEMS];
  float ksc_s[C::KT], vsc_s[C::KT];
  int kpos_s[C::KT];
};

// One (work item, kv head) unit, executed by a whole 256-thread workgroup.
template <typename TC, typename TKV, int D>
__device__ void attn_unit(const AttnArgs& a, int unit, AttnSmem<TC, D>& sm) {
  using C = AttnCfg<TC, D>;
  constexpr int KT = C::KT;
  constexpr int NB = KT / 16;                    // 16-key blocks per tile
  constexpr int ND = D / 16;                     // 16-wide d blocks of the output
  constexpr bool FP8 = sizeof(TKV) == 1;
  TC* Ks = sm.Ks;
  TC* Vs = sm.Vs;
  float* ksc_s = sm.ksc_s;
  float* vsc_s = sm.vsc_s;
  int* kpos_s = sm.kpos_s;

  // kv head fastest: consecutive units are the heads of one item, so the longest-first
  // order of the work list holds across heads
  const int Hkv = a.Hkv;
  const int h = unit % Hkv;
  const AttnWork w = a.work[unit / Hkv];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qi = lane & 15, g4 = lane >> 4;
  const int r = wave * 16 + qi;
  const int gq = r / a.Pmax, p = r % a.Pmax;
  const bool qvalid = gq < a.G && p < w.n_q;
  const bool wave_active = __any(qvalid);
  const int hq = h * a.G + (gq < a.G ? gq : 0);
  const int qpos = w.q_pos0 + p;
  const int64_t qrow = (int64_t)w.q_row0 + (qvalid ? p : 0);

  // ---- query fragments (B operand of S^T = K Q^T); qa: rotated for document B (joins)
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

  // ---- key sources: 0 = document A, 1 = document B, 2 = own rows
  KeySrc src[3];
#pragma unroll
  for (int sidx = 0; sidx < 2; sidx++) {
    KeySrc& s = src[sidx];
    int64_t off = sidx == 0 ? w.off_a : w.off_b;
    int L = sidx == 0 ? w.L_a : w.L_b;
    int64_t il = sidx == 0 ? w.idx_a : w.idx_b;
    s.n = sidx == 0 ? w.n_a : w.n_b;
    s.cache = true;
    s.clampL = max(L, 1);
    s.pos_add = sidx == 1 ? w.L_a : 0;
    s.idx = il >= 0 ? a.idx + il : nullptr;
    s.ksc = s.vsc = nullptr;
    s.pitch = (int64_t)D * (int64_t)sizeof(TKV);
    if (s.n > 0) {
      const uint8_t* base = a.pool + off;
      const int64_t kv_elems = (int64_t)L * D;
      const int64_t head_off = ((int64_t)(a.layer * Hkv + h) * 2) * kv_elems;
      s.k = base + head_off * (int64_t)sizeof(TKV);
      s.v = s.k + kv_elems * (int64_t)sizeof(TKV);
      if constexpr (FP8) {
        int nblk = (L + 15) >> 4;
        const float* sb = reinterpret_cast<const float*>(base + (int64_t)2 * a.n_layers * Hkv * kv_elems);
        s.ksc = sb + ((int64_t)(a.layer * Hkv + h) * 2) * nblk;
        s.vsc = s.ksc + nblk;
      }
    } else {
      s.k = s.v = a.pool;
    }
  }
  {
    KeySrc& s = src[2];
    s.n = w.n_own;
    s.cache = false;
    s.clampL = max(w.n_own, 1);
    s.pos_add = w.own_pos0;
    s.idx = nullptr;
    s.ksc = s.vsc = nullptr;
    s.pitch = a.own_stride * (int64_t)sizeof(TC);
    const uint8_t* ob = reinterpret_cast<const uint8_t*>(a.own) + (int64_t)w.own_row0 * s.pitch;
    s.k = ob + (int64_t)(a.own_kcol + h * D) * (int64_t)sizeof(TC);
    s.v = ob + (int64_t)(a.own_vcol + h * D) * (int64_t)sizeof(TC);
  }
  const int TA = (src[0].n + KT - 1) / KT, TB = (src[1].n + KT - 1) / KT, TO = (src[2].n + KT - 1) / KT;
  const int T = TA + TB + TO;

  float m_run = -INFINITY, l_run = 0.f;
  f32x4 o[ND];
#pragma unroll
  for (int i = 0; i < ND; i++) o[i] = f32x4{0.f, 0.f, 0.f, 0.f};

  TileStage<TC, TKV, D> stage;
  auto fetch_tile = [&](int ti) {
    if (ti < TA) stage.fetch(src[0], ti * KT);
    else if (ti < TA + TB) stage.fetch(src[1], (ti - TA) * KT);
    else stage.fetch(src[2], (ti - TA - TB) * KT);
  };
  if (T > 0) fetch_tile(0);
  for (int ti = 0; ti < T; ti++) {
    __syncthreads();  // the previous tile is fully consumed
    stage.commit(Ks, Vs, ksc_s, vsc_s, kpos_s);
    const bool tile_fp8 = stage.fp8;
    __syncthreads();
    if (ti + 1 < T) fetch_tile(ti + 1);  // in flight during this tile's compute
    // document B is scored with the queries rotated at (position - L_A)
    if (has_b && (ti == TA || ti == TA + TB)) {
#pragma unroll
      for (int k = 0; k < NQ; k++) {
        u32x4 tmp = qf[k];
        qf[k] = qa[k];
        qa[k] = tmp;
      }
    }
    if (!wave_active) continue;

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
          for (int t = 0; t < 4; t++) s[b] = mfma_f32(as_f32(kf[t]), as_f32(qf[k][t]), s[b]);
        } else {
          u32x4 kf = *reinterpret_cast<const u32x4*>(krow + 32 * k + 8 * g4);
          s[b] = mfma_bf16(__builtin_bit_cast(u16x8, kf), __builtin_bit_cast(u16x8, qf[k]), s[b]);
        }
      }
    }
    // ---- online softmax in FP32.  Statistics are kept on raw scores (the scale is > 0) and
    // the scale is folded into the exponent: p = 2^(s*c - m*c).  Only tiles that can hold an
    // invisible key (a partial tile, own rows, causal prefill) are masked.
    const bool need_mask = (ti >= TA + TB) || (ti < TA ? (ti + 1) * KT > src[0].n : (ti - TA + 1) * KT > src[1].n) ||
                           kpos_s[KT - 1] > w.q_pos0;
    float mx = -INFINITY;
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
      for (int t = 0; t < 4; t++) {
        float v = s[b][t];
        if (FP8 && tile_fp8) v *= ksc_s[16 * b + 4 * g4 + t];
        if (need_mask && !(kpos_s[16 * b + 4 * g4 + t] <= qpos)) v = -INFINITY;
        s[b][t] = v;
        mx = fmaxf(mx, v);
      }
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    const float c = a.scale_log2;
    const float m_new = fmaxf(m_run, mx);
    const float mc = m_new == -INFINITY ? 0.f : m_new * c;
    // rescale of the running sums: exactly 1 when the maximum did not move (the contracted
    // m_run * c - mc is then the rounding error of mc, not 0), 0 when m_run = -inf
    const float alpha = m_new > m_run ? __builtin_amdgcn_exp2f(m_run * c - mc) : 1.f;
    float psum = 0.f;
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
      for (int t = 0; t < 4; t++) {
        float pv = __builtin_amdgcn_exp2f(fmaf(s[b][t], c, -mc));  // exp2(-inf) = 0
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
        u32x4 pb;
#pragma unroll
        for (int t = 0; t < 4; t += 2) {
          float p0 = s[2 * b2][t], p0n = s[2 * b2][t + 1];
          float p1 = s[2 * b2 + 1][t], p1n = s[2 * b2 + 1][t + 1];
          if (FP8 && tile_fp8) {
            p0 *= vsc_s[32 * b2 + 4 * g4 + t];
            p0n *= vsc_s[32 * b2 + 4 * g4 + t + 1];
            p1 *= vsc_s[32 * b2 + 16 + 4 * g4 + t];
            p1n *= vsc_s[32 * b2 + 16 + 4 * g4 + t + 1];
          }
          pb[t / 2] = pack_bf16x2(p0, p0n);
          pb[2 + t / 2] = pack_bf16x2(p1, p1n);
        }
        const int jp_lo = 16 * b2 + 2 * g4;
#pragma unroll
        for (int i = 0; i < ND; i++) {
          const bf16_t* vrow = Vs + (16 * i + qi) * C::VTLD;
          const int sw = 2 * (i & 7);
          u32x2 lo = *reinterpret_cast<const u32x2*>(vrow + 2 * (jp_lo ^ sw));
          u32x2 hi = *reinterpret_cast<const u32x2*>(vrow + 2 * ((jp_lo + 8) ^ sw));
          u32x4 va = {lo[0], lo[1], hi[0], hi[1]};
          o[i] = mfma_bf16(__builtin_bit_cast(u16x8, va), __builtin_bit_cast(u16x8, pb), o[i]);
        }
      }
    }
  }

  // ---- normalise and store: lane holds O[query qi][d = 16*i + 4*g4 + t]
  float l_tot = l_run + __shfl_xor(l_run, 16, 64);
  l_tot += __shfl_xor(l_tot, 32, 64);
  __syncthreads();  // LDS reused by the workgroup's next unit
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

// One workgroup per unit.
template <typename TC, typename TKV, int D>
__global__ __launch_bounds__(256) void attn_kernel(AttnArgs a) {
  __shared__ AttnSmem<TC, D> sm;
  attn_unit<TC, TKV, D>(a, blockIdx.x, sm);
}

// Persistent form: a fixed grid of workgroups takes units from a device counter (reset to
// zero by the caller before the launch) in list order until every unit is taken; each
// workgroup exits once the counter passes the unit count, so the grid always drains.
template <typename TC, typename TKV, int D>
__global__ __launch_bounds__(256) void attn_persistent_kernel(AttnArgs a) {
  __shared__ AttnSmem<TC, D> sm;
  __shared__ int next;
  const int total = a.n_work * a.Hkv;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(a.counter, 1);
    __syncthreads();
    const int unit = next;
    __syncthreads();
    if (unit >= total) break;
    attn_unit<TC, TKV, D>(a, unit, sm);
  }
}

template <typename TC, typename TKV, int D>
static hipError_t launch_d(const AttnArgs& a, hipStream_t st) {
  const int64_t units = (int64_t)a.n_work * a.Hkv;
  if (a.counter) {
    hipLaunchKernelGGL((attn_persistent_kernel<TC, TKV, D>), dim3((unsigned)std::min<int64_t>(units, a.persistent_wgs)),
                       dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL((attn_kernel<TC, TKV, D>), dim3((unsigned)units), dim3(256), 0, st, a);
  }
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

static int g_attn_impl = 2;  // direct-load tiles, 32 keys, 3 stages (the fastest measured)
void attention_set_impl(int impl) { g_attn_impl = impl; }
int attention_get_impl() { return g_attn_impl; }

bool attention_is_dma(int cdt, int kvdt, int D) {
  return g_attn_impl >= 0 && cdt == DT_BF16 && (kvdt == DT_BF16 || kvdt == DT_FP8) && (D == 64 || D == 128);
}

hipError_t attention(int cdt, int kvdt, int D, const AttnArgs& a, hipStream_t st) {
  if (a.n_work <= 0) return hipSuccess;
  if (attention_is_dma(cdt, kvdt, D)) {
    if (a.decode && a.Pmax == 1 && attention_decode_ok(kvdt, D, a.G)) return attention_decode(kvdt, D, a, st);
    return attention_dma(kvdt, D, g_attn_impl, a, st);
  }
  if (a.counter && a.persistent_wgs < 1) return hipErrorInvalidValue;
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
