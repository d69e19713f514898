// Attention of one greedy decoding step of a map (BF16 compute, BF16 or FP8 cache).
//
// Every work item has a single query position: the G query heads of one kv head see one
// row each, so a 16x16 matrix-core block would be 1/16 used and a pass of the keys through
// LDS only adds traffic.  Keys and values therefore stream from HBM straight into
// registers.  A group of LPR = D / 8 lanes holds one cached row (8 elements per lane: a
// 16-byte load of a BF16 row, an 8-byte load of an FP8 row, so a row is one coalesced
// access), a wavefront holds KPW = 64 / LPR rows per load, and every lane keeps KB rows of
// keys and of values in flight per batch of BK = KB * KPW keys.
//
// One workgroup of four wavefronts serves one (work item, kv head).  Wavefront w takes
// batches w, w + 4, ... of each key source in turn: the document's retained rows, then the
// item's own rows (suffix and generated tokens), each source numbered from batch 0.  Each
// wavefront keeps an online softmax in FP32 with the arithmetic of the tiled kernels:
// scores from BF16 (or widened FP8) operands with exact products, the 1/sqrt(D) scale
// folded into the exponent, a rescale that is exactly 1 while the maximum stays, FP8 block
// scales multiplying scores and probabilities, probabilities rounded to BF16 where they
// weight the values while the normaliser sums the unrounded ones.  The four partial
// results are merged through LDS at the end.
//
// Padded batching: keys of the document past its retained count up to pad_a are loaded
// (its rows again, cyclically) and masked, so they cost reads and leave the result bit for
// bit unchanged; the own rows keep their batch numbering either way.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace kvop {

template <int G>
struct DecState {
  float m[G], l[G], o[G][8];
};

template <typename T> __device__ inline T dec_load(const T* p) {
  return *reinterpret_cast<const __attribute__((address_space(1))) T*>(reinterpret_cast<uintptr_t>(p));
}

// eight elements of a row -> floats (BF16: one 16-byte piece; FP8: one 8-byte piece, widened)
template <typename TE> struct DecRow;
template <> struct DecRow<bf16_t> {
  typedef u32x4 raw_t;
  __device__ static inline void unpack(const raw_t& r, float (&f)[8]) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      f[2 * i] = __builtin_bit_cast(float, r[i] << 16);
      f[2 * i + 1] = __builtin_bit_cast(float, r[i] & 0xffff0000u);
    }
  }
};
template <> struct DecRow<fp8_t> {
  typedef u32x2 raw_t;
  __device__ static inline void unpack(const raw_t& r, float (&f)[8]) {
    const u32x4 b = fp8x8_to_bf16x8(r[0], r[1]);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      f[2 * i] = __builtin_bit_cast(float, b[i] << 16);
      f[2 * i + 1] = __builtin_bit_cast(float, b[i] & 0xffff0000u);
    }
  }
};

// One key source: rows k/v + row * pitch (bytes), row = idx[key] (or key), key < n real,
// keys up to npad loaded and masked; key position = row + pos_add.  The row numbers of a
// batch arrive with one load per key (lane i: key i of the batch, spread to the row groups
// by shuffles) a batch ahead of the rows themselves, together with the FP8 block scales,
// so a batch's row loads never wait on its row numbers.
template <typename TE, int D, int G, int KB>
__device__ __attribute__((always_inline)) inline void dec_source(DecState<G>& s, const float (&q)[G][8],
                                                                 const uint8_t* kb, const uint8_t* vb, int64_t pitch,
                                                                 const int32_t* idx, int n, int npad, int clampL,
                                                                 int pos_add, const float* ksc, const float* vsc,
                                                                 int qpos, float c, int wave, int sl, int grp) {
  constexpr int LPR = D / 8, KPW = 64 / LPR, BK = KB * KPW;
  static_assert(BK <= 64, "one row number per lane");
  constexpr bool FP8 = sizeof(TE) == 1;
  using R = DecRow<TE>;
  typedef typename R::raw_t raw_t;
  const int nb = n > 0 ? (npad + BK - 1) / BK : 0;
  const int lane = __lane_id();
  // row number of key `lane` of batch bi (past the keys: the source's rows again, cyclically)
  auto row_of = [&](int bi) {
    const int key = bi * BK + (lane < BK ? lane : 0);
    const int kc = key < n ? key : key % n;
    const int rr = idx ? dec_load(idx + kc) : kc;
    return min(max(rr, 0), clampL - 1);
  };
  int rv = wave < nb ? row_of(wave) : 0;
  float ksv = 0.f, vsv = 0.f;
  if constexpr (FP8) {
    if (wave < nb) {
      ksv = dec_load(ksc + (rv >> 4));
      vsv = dec_load(vsc + (rv >> 4));
    }
  }
  for (int bi = wave; bi < nb; bi += 4) {
    int row[KB];
    bool real[KB];
    raw_t kr[KB], vr[KB];
    float ks[KB], vs[KB];
#pragma unroll
    for (int j = 0; j < KB; j++) {
      const int src = j * KPW + grp;
      row[j] = __shfl(rv, src, 64);
      real[j] = bi * BK + src < n;
      const int64_t off = (int64_t)row[j] * pitch + sl * 8 * (int)sizeof(TE);
      kr[j] = dec_load(reinterpret_cast<const raw_t*>(kb + off));
      vr[j] = dec_load(reinterpret_cast<const raw_t*>(vb + off));
      if constexpr (FP8) {
        ks[j] = __shfl(ksv, src, 64);
        vs[j] = __shfl(vsv, src, 64);
      }
    }
    // the next batch's row numbers, in flight behind this batch's rows
    const bool more = bi + 4 < nb;
    if (more) rv = row_of(bi + 4);
    // scores: the group's lanes each hold 8 products' sum, reduced over the group
    float sc[G][KB];
#pragma unroll
    for (int j = 0; j < KB; j++) {
      float kf[8];
      R::unpack(kr[j], kf);
#pragma unroll
      for (int g = 0; g < G; g++) {
        float acc = 0.f;
#pragma unroll
        for (int e = 0; e < 8; e++) acc = fmaf(q[g][e], kf[e], acc);
#pragma unroll
        for (int o = 1; o < LPR; o <<= 1) acc += __shfl_xor(acc, o, 64);
        if constexpr (FP8) acc *= ks[j];
        sc[g][j] = (real[j] && row[j] + pos_add <= qpos) ? acc : -INFINITY;
      }
    }
    // the next batch's block scales (their row numbers have arrived by now)
    if constexpr (FP8) {
      if (more) {
        ksv = dec_load(ksc + (rv >> 4));
        vsv = dec_load(vsc + (rv >> 4));
      }
    }
    // online softmax over the batch (the maximum is shared by the wavefront's groups, so
    // their partial sums stay on one scale)
#pragma unroll
    for (int g = 0; g < G; g++) {
      float bm = sc[g][0];
#pragma unroll
      for (int j = 1; j < KB; j++) bm = fmaxf(bm, sc[g][j]);
#pragma unroll
      for (int o = LPR; o < 64; o <<= 1) bm = fmaxf(bm, __shfl_xor(bm, o, 64));
      const float m_new = fmaxf(s.m[g], bm);
      const float mc = m_new == -INFINITY ? 0.f : m_new * c;
      const float alpha = m_new > s.m[g] ? __builtin_amdgcn_exp2f(s.m[g] * c - mc) : 1.f;
      float psum = 0.f;
#pragma unroll
      for (int j = 0; j < KB; j++) {
        const float pv = __builtin_amdgcn_exp2f(fmaf(sc[g][j], c, -mc));  // exp2(-inf) = 0
        sc[g][j] = pv;
        psum += pv;
      }
      s.l[g] = s.l[g] * alpha + psum;
      s.m[g] = m_new;
#pragma unroll
      for (int e = 0; e < 8; e++) s.o[g][e] *= alpha;
    }
    // values weighted by the BF16-rounded probabilities
#pragma unroll
    for (int j = 0; j < KB; j++) {
      float vf[8];
      R::unpack(vr[j], vf);
#pragma unroll
      for (int g = 0; g < G; g++) {
        float p = sc[g][j];
        if constexpr (FP8) p *= vs[j];
        const float pw = bf2f(f2bf(p));
#pragma unroll
        for (int e = 0; e < 8; e++) s.o[g][e] = fmaf(pw, vf[e], s.o[g][e]);
      }
    }
  }
}

template <typename TKV, int D, int G, int KB>
__global__ __launch_bounds__(256) void attn_decode_kernel(AttnArgs a) {
  constexpr int LPR = D / 8;
  __shared__ float red_m[4][G], red_l[4][G];
  __shared__ float red_o[4][G][D];
  const int Hkv = a.Hkv;
  const int h = blockIdx.x % Hkv;
  const AttnWork w = a.work[blockIdx.x / Hkv];
  if (w.n_q < 1) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sl = lane % LPR, grp = lane / LPR;
  const float c = a.scale_log2;
  const int64_t qrow = w.q_row0;

  float q[G][8];
#pragma unroll
  for (int g = 0; g < G; g++) {
    const u32x4 v = dec_load(reinterpret_cast<const u32x4*>(reinterpret_cast<const bf16_t*>(a.q) + qrow * a.q_stride +
                                                            (int64_t)(h * G + g) * D + 8 * sl));
    DecRow<bf16_t>::unpack(v, q[g]);
  }
  DecState<G> s;
#pragma unroll
  for (int g = 0; g < G; g++) {
    s.m[g] = -INFINITY;
    s.l[g] = 0.f;
#pragma unroll
    for (int e = 0; e < 8; e++) s.o[g][e] = 0.f;
  }

  // the document's retained rows (cache layout: per layer and kv head, K [L][D] then V [L][D];
  // FP8 block scales after all layers' rows)
  if (w.n_a > 0) {
    const uint8_t* base = a.pool + w.off_a;
    const int64_t kv_elems = (int64_t)w.L_a * D;
    const int64_t head_off = ((int64_t)(a.layer * Hkv + h) * 2) * kv_elems;
    const uint8_t* kb = base + head_off * (int64_t)sizeof(TKV);
    const uint8_t* vb = kb + kv_elems * (int64_t)sizeof(TKV);
    const float *ksc = nullptr, *vsc = nullptr;
    if constexpr (sizeof(TKV) == 1) {
      const int nblk = (w.L_a + 15) >> 4;
      const float* sbase = reinterpret_cast<const float*>(base + (int64_t)2 * a.n_layers * Hkv * kv_elems);
      ksc = sbase + ((int64_t)(a.layer * Hkv + h) * 2) * nblk;
      vsc = ksc + nblk;
    }
    dec_source<TKV, D, G, KB>(s, q, kb, vb, (int64_t)D * sizeof(TKV), w.idx_a >= 0 ? a.idx + w.idx_a : nullptr, w.n_a,
                              std::max(w.n_a, w.pad_a), std::max(w.L_a, 1), 0, ksc, vsc, w.q_pos0, c, wave, sl, grp);
  }
  // own rows (BF16, position own_pos0 + j)
  if (w.n_own > 0) {
    const int64_t pitch = a.own_stride * 2;
    const uint8_t* ob = reinterpret_cast<const uint8_t*>(a.own) + (int64_t)w.own_row0 * pitch;
    dec_source<bf16_t, D, G, KB>(s, q, ob + (int64_t)(a.own_kcol + h * D) * 2, ob + (int64_t)(a.own_vcol + h * D) * 2,
                                 pitch, nullptr, w.n_own, w.n_own, w.n_own, w.own_pos0, nullptr, nullptr, w.q_pos0, c,
                                 wave, sl, grp);
  }

  // the wavefront's groups share one scale: sum them, then merge the four wavefronts
#pragma unroll
  for (int g = 0; g < G; g++) {
    float l = s.l[g];
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1) l += __shfl_xor(l, o, 64);
#pragma unroll
    for (int e = 0; e < 8; e++) {
      float v = s.o[g][e];
#pragma unroll
      for (int o = LPR; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
      if (grp == 0) red_o[wave][g][8 * sl + e] = v;
    }
    if (lane == 0) {
      red_m[wave][g] = s.m[g];
      red_l[wave][g] = l;
    }
  }
  __syncthreads();
  bf16_t* out = reinterpret_cast<bf16_t*>(a.out) + qrow * a.out_stride + (int64_t)h * G * D;
  for (int t = tid; t < G * D; t += 256) {
    const int g = t / D, dd = t % D;
    float M = red_m[0][g];
#pragma unroll
    for (int ww = 1; ww < 4; ww++) M = fmaxf(M, red_m[ww][g]);
    float L = 0.f, O = 0.f;
#pragma unroll
    for (int ww = 0; ww < 4; ww++) {
      const float mw = red_m[ww][g];
      const float f = mw == -INFINITY ? 0.f : (mw < M ? __builtin_amdgcn_exp2f(mw * c - M * c) : 1.f);
      L = fmaf(f, red_l[ww][g], L);
      O = fmaf(f, red_o[ww][g][dd], O);
    }
    const float inv = L > 0.f ? 1.f / L : 0.f;
    out[(int64_t)g * D + dd] = f2bf(O * inv);
  }
}

template <typename TKV, int D>
static hipError_t launch_decode(const AttnArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)((int64_t)a.n_work * a.Hkv));
  switch (a.G) {
    case 1: hipLaunchKernelGGL((attn_decode_kernel<TKV, D, 1, 8>), grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((attn_decode_kernel<TKV, D, 2, 8>), grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((attn_decode_kernel<TKV, D, 4, 8>), grid, dim3(256), 0, st, a); break;
  }
  return hipGetLastError();
}

bool attention_decode_ok(int kvdt, int D, int G) {
  return (kvdt == DT_BF16 || kvdt == DT_FP8) && (D == 64 || D == 128) && (G == 1 || G == 2 || G == 4);
}

hipError_t attention_decode(int kvdt, int D, const AttnArgs& a, hipStream_t st) {
  if (a.n_work <= 0) return hipSuccess;
  if (a.Pmax != 1 || !attention_decode_ok(kvdt, D, a.G)) return hipErrorInvalidValue;
  if (kvdt == DT_BF16) return D == 128 ? launch_decode<bf16_t, 128>(a, st) : launch_decode<bf16_t, 64>(a, st);
  return D == 128 ? launch_decode<fp8_t, 128>(a, st) : launch_decode<fp8_t, 64>(a, st);
}

}  // namespace kvop
