// Attention over gathered cache rows with direct global -> LDS loads (BF16 compute path).
//
// Same work decomposition and arithmetic as the register-staged kernel in attention.hip:
// one workgroup of 4 wavefronts per (work item, kv head); scores computed transposed,
// S^T = K Q^T, so that every accumulator of a lane belongs to one query; online softmax in
// FP32 on raw scores with the 1/sqrt(D) scale folded into the exponent; O^T = V^T P^T.
// The difference is how key/value tiles reach LDS: with global_load_lds every lane names
// one 16-byte chunk of a cached row anywhere in HBM and the chunk lands in LDS at the
// lane's slot, so a gathered tile costs no registers and up to NS tiles are in flight per
// workgroup.  Completion is tracked with explicit vmcnt waits: every wavefront issues the
// same number of vector-memory operations per tile.
//
// LDS layout of a tile part (K or V): rows in the source dtype (FP8 cache rows, BF16
// cache or own rows), chunk c of row r at slot c ^ swz(r).  The K swizzle spreads the 16
// rows read at one chunk by an S^T operand over distinct banks; the V swizzle does the
// same for the 8 rows x 2 chunks of a transposed read.  V^T operands come from
// ds_read_b64_tr_b16 (BF16 rows) or ds_read_b64_tr_b8 (FP8 rows) without a transposing
// copy; FP8 values are widened with the hardware FP8 -> BF16 conversion (exact: every E4M3
// value is a BF16 value) and their per-16-row block scales multiply scores and
// probabilities as in the register-staged kernel.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace kvop {

typedef __attribute__((address_space(3))) void lds_void_t;
typedef short v4i16_t __attribute__((ext_vector_type(4)));
typedef int v2i32_t __attribute__((ext_vector_type(2)));

template <typename TKV, int D, int KT_, int NS_>
struct DmaCfg {
  static constexpr bool FP8 = sizeof(TKV) == 1;
  static constexpr int KT = KT_;                     // keys per cache tile
  static constexpr int NS = NS_;                     // stages (tiles resident in LDS)
  static constexpr int RBC = D * (int)sizeof(TKV);   // bytes per cached row
  static constexpr int RBO = D * 2;                  // bytes per own (BF16) row
  static constexpr int KTO = FP8 ? KT / 2 : KT;      // keys per own tile: the same bytes as a cache tile
  static constexpr int CHC = RBC / 16, CHO = RBO / 16;
  static constexpr int REGION = KT * RBC;            // bytes of the K (or V) part of a tile
  static_assert(KT * RBC == KTO * RBO, "cache and own tiles move the same bytes");
  static constexpr int NJ = 2 * REGION / 16 / 256;   // chunk loads per thread per tile
  static constexpr int NR = NJ / 2;                  // rows per thread per tile (K and V chunks share them)
  static_assert(NJ >= 2 && NJ % 2 == 0, "tile split");
  static constexpr int META = 3 * 64 * 4;            // ksc | vsc | unused (64 slots each)
  static constexpr int STAGE = 2 * REGION + META;
  static constexpr int RING = NS * STAGE;            // row-number ring: NS + 1 slots of 64
  static constexpr int LDS = RING + (NS + 1) * 64 * 4;
  static constexpr int LDS_TOTAL = LDS;
  // vmcnt that leaves only the newest tile's chunk + metadata loads outstanding
  static constexpr int WAIT = NS >= 3 ? NJ + 1 : 0;
  static_assert(NJ + 1 <= 15, "vmcnt immediates");
  static_assert(NS == 2 || NS == 3, "stages");
};

// log2(16 / CH): consecutive rows that share one 256-byte bank line
template <int CH> struct RowShift {
  static constexpr int v = CH >= 16 ? 0 : (CH == 8 ? 1 : (CH == 4 ? 2 : 3));
};
template <int CH> __device__ inline int swz_k(int r) { return (r >> RowShift<CH>::v) & (CH - 1); }
template <int CH> __device__ inline int swz_v(int r) { return CH >= 4 ? 2 * ((r >> RowShift<CH>::v) & (CH / 2 - 1)) : 0; }
// V swizzle of FP8 rows (read by ds_read_b64_tr_b8: rows r, r + 1, r + 2, r + 3 and the
// same + 16 at one chunk, for two lane groups): distinct (slot, bank line half) pairs
template <int CH> __device__ inline int swz_v8(int r) {
  if constexpr (CH >= 8) return ((r >> 1) & 3) | (((r >> 4) & 1) << 2);
  else return ((r >> 2) & 1) | (((r >> 4) & 1) << 1);
}

template <int N> __device__ inline void vm_wait() {
  static_assert(N >= 0 && N <= 63, "vmcnt range");
  // gfx9 s_waitcnt: vmcnt in bits 3:0 and 15:14, expcnt 6:4 (7: no wait), lgkmcnt 11:8 (15: no wait)
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// ds_read_b64_tr_b16 as inline assembly.  The builtin form makes the compiler wait for every
// direct-to-LDS load in flight (vmcnt(0)) before it, since it cannot tell which LDS bytes
// the read touches.  The assembly form is followed by an explicit lgkmcnt(0) wait; the
// caller reads V only from stages whose loads have completed (checked by the tile wait).
// The result may only be used after lgkm_wait_all() has taken it as an operand.
__device__ inline u32x2 ds_read_tr16(const uint8_t* p) {
  const uint32_t addr = (uint32_t)reinterpret_cast<uintptr_t>(p);
  u32x2 v;
  asm volatile("ds_read_b64_tr_b16 %0, %1" : "=v"(v) : "v"(addr) : "memory");
  return v;
}
__device__ inline u32x2 ds_read_tr8(const uint8_t* p) {
  const uint32_t addr = (uint32_t)reinterpret_cast<uintptr_t>(p);
  u32x2 v;
  asm volatile("ds_read_b64_tr_b8 %0, %1" : "=v"(v) : "v"(addr) : "memory");
  return v;
}
// lgkmcnt(0), tied to the values it guards so that no use is scheduled above it
template <int N> __device__ inline void lgkm_wait_all(u32x2 (&v)[N]);
template <> __device__ inline void lgkm_wait_all<4>(u32x2 (&v)[4]) {
  asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]) : : "memory");
}
template <> __device__ inline void lgkm_wait_all<8>(u32x2 (&v)[8]) {
  asm volatile("s_waitcnt lgkmcnt(0)"
               : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7])
               :
               : "memory");
}
template <> __device__ inline void lgkm_wait_all<16>(u32x2 (&v)[16]) {
  asm volatile("s_waitcnt lgkmcnt(0)"
               : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7]),
                 "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]), "+v"(v[14]), "+v"(v[15])
               :
               : "memory");
}

// plain global load (global_load, not flat: a flat load also counts in lgkmcnt)
template <typename T> __device__ inline T gload(const T* p) {
  return *reinterpret_cast<const __attribute__((address_space(1))) T*>(reinterpret_cast<uintptr_t>(p));
}

struct __attribute__((aligned(8))) DmaSrc {
  const uint8_t* k;     // row 0 of the keys (bytes)
  const uint8_t* v;
  int64_t pitch;        // bytes between rows
  const int32_t* idx;   // retained list or null (rows 0..n-1)
  const float* ksc;     // FP8 block scales (per 16 rows) or null
  const float* vsc;
  int n, clampL, pos_add;
  int npad;             // keys iterated (>= n when padded, else n); keys past n are masked
};

template <typename TKV, int D, int KT, int NS, int KC>
__device__ void attn_dma_unit(const AttnArgs& a, int unit, uint8_t* smem) {
  using C = DmaCfg<TKV, D, KT, NS>;
  constexpr int NQ = D / 32;                 // 32-deep K steps of S^T
  constexpr int ND = D / 16;                 // 16-wide d blocks of the output
  constexpr int NBC = KC / 16;               // 16-key blocks of one compute step
  constexpr int NSTEP = KT / KC;             // compute steps per cache tile
  static_assert(KT % KC == 0 && KC % 32 == 0, "compute steps of whole 32-key pairs");
  constexpr bool FP8 = C::FP8;

  const int Hkv = a.Hkv;
  const int h = unit % Hkv;
  const AttnWork w = a.work[unit / Hkv];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int qi = lane & 15, g4 = lane >> 4;
  const int r = wave * 16 + qi;
  const int gq = r / a.Pmax, p = r % a.Pmax;
  const bool qvalid = gq < a.G && p < w.n_q;
  const bool wave_active = __any(qvalid);
  const int hq = h * a.G + (gq < a.G ? gq : 0);
  const int qpos = w.q_pos0 + p;
  const int64_t qrow = (int64_t)w.q_row0 + (qvalid ? p : 0);

  // ---- query fragments (B operand of S^T); qa: rotated for document B (joins)
  // (joins: the fragments of the queries rotated at position - L_A are loaded when the
  // tiles of document B begin, and the plain ones again after them; holding both sets
  // would cost the registers of a third resident workgroup)
  u32x4 qf[NQ];
  const bool has_b = w.n_b > 0;
  const bf16_t* q_plain = reinterpret_cast<const bf16_t*>(a.q) + qrow * a.q_stride + hq * D;
  const bf16_t* q_rot = reinterpret_cast<const bf16_t*>(a.q_alt ? a.q_alt : a.q) + qrow * a.q_stride + hq * D;
  auto load_q = [&](const bf16_t* q) {
#pragma unroll
    for (int k = 0; k < NQ; k++)
      qf[k] = qvalid ? gload(reinterpret_cast<const u32x4*>(q + 32 * k + 8 * g4)) : u32x4{0, 0, 0, 0};
  };
  load_q(q_plain);

  // ---- key sources: 0 = document A, 1 = document B, 2 = own rows.  Three separate
  // variables selected field by field (a dynamically indexed local array would live in
  // scratch memory, and a scratch load waits behind every tile load in flight).
  auto init_doc = [&](DmaSrc& s, int64_t off, int L, int64_t il, int n, int pos_add, int pad) {
    s.n = n;
    s.npad = n > 0 ? max(n, pad) : 0;
    s.clampL = max(L, 1);
    s.pos_add = pos_add;
    s.idx = il >= 0 ? a.idx + il : nullptr;
    s.pitch = C::RBC;
    s.ksc = s.vsc = nullptr;
    s.k = s.v = a.pool;
    if (n > 0) {
      const uint8_t* base = a.pool + off;
      const int64_t kv_elems = (int64_t)L * D;
      const int64_t head_off = ((int64_t)(a.layer * Hkv + h) * 2) * kv_elems;
      s.k = base + head_off * (int64_t)sizeof(TKV);
      s.v = s.k + kv_elems * (int64_t)sizeof(TKV);
      if constexpr (FP8) {
        const int nblk = (L + 15) >> 4;
        const float* sb = reinterpret_cast<const float*>(base + (int64_t)2 * a.n_layers * Hkv * kv_elems);
        s.ksc = sb + ((int64_t)(a.layer * Hkv + h) * 2) * nblk;
        s.vsc = s.ksc + nblk;
      }
    }
  };
  DmaSrc src0, src1, src2;
  init_doc(src0, w.off_a, w.L_a, w.idx_a, w.n_a, 0, w.pad_a);
  init_doc(src1, w.off_b, w.L_b, w.idx_b, w.n_b, w.L_a, 0);
  {
    DmaSrc& s = src2;
    s.n = w.n_own;
    s.npad = w.n_own;
    s.clampL = max(w.n_own, 1);
    s.pos_add = w.own_pos0;
    s.idx = nullptr;
    s.ksc = s.vsc = nullptr;
    s.pitch = a.own_stride * 2;
    const uint8_t* ob = reinterpret_cast<const uint8_t*>(a.own) + (int64_t)w.own_row0 * s.pitch;
    s.k = ob + (int64_t)(a.own_kcol + h * D) * 2;
    s.v = ob + (int64_t)(a.own_vcol + h * D) * 2;
  }
  const int TA = (src0.npad + KT - 1) / KT, TB = (src1.npad + KT - 1) / KT;
  const int TO = (src2.n + C::KTO - 1) / C::KTO;
  vm_wait<0>();  // the query fragments have arrived (the loop's waits count tile loads only)
  __syncthreads();
  const int T = TA + TB + TO;
  // a valid address for loads whose value is not used (keeps the per-tile load count fixed)
  const int32_t* dummy = reinterpret_cast<const int32_t*>(a.work + unit / Hkv);

  auto tile_src = [&](int ti, int& sidx, int& t0) {
    if (ti < TA) { sidx = 0; t0 = ti * KT; }
    else if (ti < TA + TB) { sidx = 1; t0 = (ti - TA) * KT; }
    else { sidx = 2; t0 = (ti - TA - TB) * C::KTO; }
  };

  // Row numbers of retained lists reach LDS by direct loads too (one 4-byte load per key,
  // lane = key), one step before the tile's chunks are issued, into a ring of NS + 1
  // slots: the loop then holds no register-destination memory load, so the only waits on
  // memory are the explicit ones below.  Ring slot of tile X: X % (NS + 1).
  int* ring = reinterpret_cast<int*>(smem + C::RING);
  // The current source is selected field by field from the three descriptors, which are
  // uniform across the workgroup and stay in scalar registers (an indexed local array
  // would live in scratch memory, and a scratch load waits behind every tile load in
  // flight).
  auto pick = [&](int sidx) {
    DmaSrc r;
#define KVOP_PICK(f) r.f = sidx == 0 ? src0.f : (sidx == 1 ? src1.f : src2.f)
    KVOP_PICK(k); KVOP_PICK(v); KVOP_PICK(pitch); KVOP_PICK(idx); KVOP_PICK(ksc); KVOP_PICK(vsc);
    KVOP_PICK(n); KVOP_PICK(clampL); KVOP_PICK(pos_add); KVOP_PICK(npad);
#undef KVOP_PICK
    return r;
  };
  auto issue_rows = [&](int ti) {
    int sidx, t0;
    tile_src(ti, sidx, t0);
    const DmaSrc s = pick(sidx);
    // a padded tile (past the source's keys) loads the source's rows again from the start
    // of the list, cyclically: real rows, so the padded keys cost loads and multiplies
    const int tl = t0 < s.n ? t0 : t0 % s.n;
    const int32_t* g = s.idx ? s.idx + min(tl + lane, s.n - 1) : dummy;
    __builtin_amdgcn_global_load_lds(g, (lds_void_t*)(ring + (ti % (NS + 1)) * 64), 4, 0, 0);
  };
  // chunk loads of tile ti into stage st, then one metadata load per wavefront (key =
  // lane): wave 0 the K block scales, wave 1 the V block scales, waves 2-3 none (a load of
  // an unused word keeps the count per wavefront the same)
  auto issue_tile = [&](int ti, int st) {
    int sidx, t0;
    tile_src(ti, sidx, t0);
    const DmaSrc s = pick(sidx);
    const int tl = t0 < s.n ? t0 : t0 % s.n;   // as in issue_rows
    const int* rws = ring + (ti % (NS + 1)) * 64;
    uint8_t* sb = smem + st * C::STAGE;
    const bool own = sidx == 2;
    const int ch = own ? C::CHO : C::CHC;
#pragma unroll
    for (int j = 0; j < C::NJ; j++) {
      const int jr = j % C::NR;
      const bool is_v = j >= C::NR;
      const int f = 256 * jr + tid;              // chunk index inside the part
      const int rr = f / ch, slot = f % ch;
      const int t = min(tl + rr, s.n - 1);
      const int row = min(max(s.idx ? rws[rr] : t, 0), s.clampL - 1);
      int sw;
      if (own) sw = is_v ? swz_v<C::CHO>(rr) : swz_k<C::CHO>(rr);
      else if (FP8) sw = is_v ? swz_v8<C::CHC>(rr) : swz_k<C::CHC>(rr);
      else sw = is_v ? swz_v<C::CHC>(rr) : swz_k<C::CHC>(rr);
      const uint8_t* g = (is_v ? s.v : s.k) + (int64_t)row * s.pitch + (slot ^ sw) * 16;
      uint8_t* l = sb + (is_v ? C::REGION : 0) + (256 * jr + 64 * wave) * 16;
      __builtin_amdgcn_global_load_lds(g, (lds_void_t*)l, 16, 0, 0);
    }
    float* meta = reinterpret_cast<float*>(sb + 2 * C::REGION);
    const int row = min(max(s.idx ? rws[lane] : min(tl + lane, s.n - 1), 0), s.clampL - 1);
    const void* g = dummy;
    if (wave == 0 && s.ksc) g = s.ksc + (row >> 4);
    if (wave == 1 && s.vsc) g = s.vsc + (row >> 4);
    __builtin_amdgcn_global_load_lds(g, (lds_void_t*)(meta + min(wave, 2) * 64), 4, 0, 0);
  };

  float m_run = -INFINITY, l_run = 0.f;
  f32x4 o[ND];
#pragma unroll
  for (int i = 0; i < ND; i++) o[i] = f32x4{0.f, 0.f, 0.f, 0.f};

  // Prologue: rows of tile 0; then for q = 0 .. NS-2: rows of tile q + 1, chunks of tile q.
  // Waiting until only the newest chunk loads (NJ + 1) are outstanding guarantees the rows
  // issued just before them.
  if (T > 0) {
    issue_rows(0);
    vm_wait<0>();
    __builtin_amdgcn_s_barrier();
  }
#pragma unroll
  for (int q = 0; q < NS - 1; q++) {
    if (q < T) {
      if (q + 1 < T) issue_rows(q + 1);
      issue_tile(q, q);
      vm_wait<C::NJ + 1>();
      __builtin_amdgcn_s_barrier();
    }
  }

  for (int ti = 0; ti < T; ti++) {
    // Tile ti and the rows of tile ti + NS - 1 have landed once only the previous step's
    // chunk loads may be outstanding (NS = 3; NS = 2 waits for everything); if that step
    // issued no chunks, wait for everything.  Then a bare s_barrier makes every
    // wavefront's loads visible and marks tile ti - 1 consumed (a fence would wait for
    // the loads still in flight).
    if (ti + NS - 2 < T) vm_wait<C::WAIT>();
    else vm_wait<0>();
    __builtin_amdgcn_s_barrier();
    if (ti + NS < T) issue_rows(ti + NS);
    if (ti + NS - 1 < T) issue_tile(ti + NS - 1, (ti + NS - 1) % NS);

    int sidx, t0;
    tile_src(ti, sidx, t0);
    const DmaSrc s = pick(sidx);
    const bool own = sidx == 2;
    const bool tile_fp8 = FP8 && !own;
    const int nbt = (own ? C::KTO : KT) / 16;  // 16-key blocks present in this tile
    const uint8_t* sb = smem + (ti % NS) * C::STAGE;
    const uint8_t* Kp = sb;
    const uint8_t* Vp = sb + C::REGION;
    const float* ksc_s = reinterpret_cast<const float*>(sb + 2 * C::REGION);
    const float* vsc_s = ksc_s + 64;
    const int* rows_s = ring + (ti % (NS + 1)) * 64;

    // document B is scored with the queries rotated at (position - L_A)
    if (has_b && (ti == TA || ti == TA + TB)) load_q(ti == TA ? q_rot : q_plain);
    if (!wave_active) continue;

    // The tile is computed in steps of KC keys (blocks kb0 .. kb0 + NBC - 1), each with its own
    // online-softmax update: a tile may carry more keys than one step holds in registers.
#pragma unroll
    for (int hc = 0; hc < NSTEP; hc++) {
      const int kb0 = hc * NBC;
      if (kb0 >= nbt) break;
      // ---- scores S^T[key][query]: lane holds keys 16 (kb0 + b) + 4 g4 + t of query column qi
      f32x4 sc[NBC];
#pragma unroll
      for (int b = 0; b < NBC; b++) {
        sc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (kb0 + b >= nbt) continue;
        const int kr = 16 * (kb0 + b) + qi;
#pragma unroll
        for (int k = 0; k < NQ; k++) {
          u32x4 kf;
          if (tile_fp8) {
            const int pc = 4 * k + g4;  // 8-byte piece of the FP8 row
            const u32x2 raw = *reinterpret_cast<const u32x2*>(Kp + kr * C::RBC + ((pc >> 1) ^ swz_k<C::CHC>(kr)) * 16 +
                                                             (pc & 1) * 8);
            kf = fp8x8_to_bf16x8(raw[0], raw[1]);
          } else if (own) {
            kf = *reinterpret_cast<const u32x4*>(Kp + kr * C::RBO + ((4 * k + g4) ^ swz_k<C::CHO>(kr)) * 16);
          } else {
            kf = *reinterpret_cast<const u32x4*>(Kp + kr * C::RBC + ((4 * k + g4) ^ swz_k<C::CHC>(kr)) * 16);
          }
          sc[b] = mfma_bf16(__builtin_bit_cast(u16x8, kf), __builtin_bit_cast(u16x8, qf[k]), sc[b]);
        }
      }
      // ---- online softmax (FP32).  Keys past the source's end and keys after the query's
      // position are masked; only tiles that can hold such keys test positions.
      const int n_here = s.n - t0;
      const bool need_mask = own || n_here < nbt * 16 || (!s.idx && t0 + nbt * 16 - 1 + s.pos_add > w.q_pos0) ||
                             (s.idx && rows_s[nbt * 16 - 1] + s.pos_add > w.q_pos0);
      float mx = -INFINITY;
#pragma unroll
      for (int b = 0; b < NBC; b++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int key = 16 * (kb0 + b) + 4 * g4 + t;
          float v = sc[b][t];
          if (tile_fp8) v *= ksc_s[key];
          if (kb0 + b >= nbt) {
            v = -INFINITY;
          } else if (need_mask) {
            const int kpos = key < n_here ? (s.idx ? rows_s[key] : t0 + key) + s.pos_add : 0x7fffffff;
            if (!(kpos <= qpos)) v = -INFINITY;
          }
          sc[b][t] = v;
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
      for (int b = 0; b < NBC; b++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const float pv = __builtin_amdgcn_exp2f(fmaf(sc[b][t], c, -mc));  // exp2(-inf) = 0
          sc[b][t] = pv;
          psum += pv;
        }
      l_run = l_run * alpha + psum;
      m_run = m_new;
#pragma unroll
      for (int i = 0; i < ND; i++) o[i] *= alpha;

      // ---- O^T[d][query] += V^T[d][key] P^T[key][query].  K slots 0..3 of lane group g4 are
      // keys 32 b2 + 4 g4 + t, slots 4..7 keys 32 b2 + 16 + 4 g4 + t (b2: pair of the tile;
      // bl: the same pair's first block within this step).
#pragma unroll
      for (int bp = 0; bp < NBC / 2; bp++) {
        const int bl = 2 * bp, b2 = kb0 / 2 + bp;
        if (2 * b2 >= nbt) continue;
        u32x4 pb;
#pragma unroll
        for (int t = 0; t < 4; t += 2) {
          float p0 = sc[bl][t], p0n = sc[bl][t + 1];
          float p1 = sc[bl + 1][t], p1n = sc[bl + 1][t + 1];
          if (tile_fp8) {
            p0 *= vsc_s[32 * b2 + 4 * g4 + t];
            p0n *= vsc_s[32 * b2 + 4 * g4 + t + 1];
            p1 *= vsc_s[32 * b2 + 16 + 4 * g4 + t];
            p1n *= vsc_s[32 * b2 + 16 + 4 * g4 + t + 1];
          }
          pb[t / 2] = pack_bf16x2(p0, p0n);
          pb[2 + t / 2] = pack_bf16x2(p1, p1n);
        }
        // lane (qi, g4) reads V[keys 32 b2 + 4 g4 + 0..3 (+16)][d = 16 i + qi].  A tile with a
        // single 16-key block in this pair (a 16-key own tile) has no rows +16: those keys
        // carry p = 0, so any finite row will do (the tile's own rows, not bytes past it)
        const int vr0 = 32 * b2 + 4 * g4 + (qi >> 2), vr1 = 2 * b2 + 1 < nbt ? vr0 + 16 : vr0;
        if (tile_fp8) {
          // 8-bit transposed reads: within a lane group, lane qi addresses key slot qi / 2
          // (row 32 b2 + 4 g4 + (qi/2 < 4 ? qi/2 : 16 + qi/2 - 4)) at byte columns
          // 16 i + 8 (qi % 2) .. +7; lane qi receives byte column 16 i + qi of the 8 rows
          const int ks = qi >> 1;
          const int vr = 32 * b2 + 4 * g4 + (ks < 4 ? ks : 12 + ks);
          const int sv = swz_v8<C::CHC>(vr);
          u32x2 y[ND];
#pragma unroll
          for (int i = 0; i < ND; i++) y[i] = ds_read_tr8(Vp + vr * C::RBC + ((i ^ sv) * 16) + (qi & 1) * 8);
          lgkm_wait_all<ND>(y);
#pragma unroll
          for (int i = 0; i < ND; i++) {
            const u32x4 va = fp8x8_to_bf16x8(y[i][0], y[i][1]);
            o[i] = mfma_bf16(__builtin_bit_cast(u16x8, va), __builtin_bit_cast(u16x8, pb), o[i]);
          }
        } else {
          // 16-bit transposed reads: lane (qi, g4) addresses row vr (qi / 4 selects the key),
          // columns 16 i + 4 (qi % 4) .. +3; lane qi receives column 16 i + qi of 4 rows
          const int rb = own ? C::RBO : C::RBC;
          const int s0 = own ? swz_v<C::CHO>(vr0) : swz_v<C::CHC>(vr0);
          const int s1 = own ? swz_v<C::CHO>(vr1) : swz_v<C::CHC>(vr1);
          // 32-key tiles: in two halves of the d blocks (fewer live registers, for the
          // register budget of three resident workgroups)
          constexpr int NHALF = KC == 32 ? 2 : 1;
#pragma unroll
          for (int h2 = 0; h2 < NHALF; h2++) {
            constexpr int NH = ND / NHALF;
            u32x2 y[2 * NH];
#pragma unroll
            for (int ii = 0; ii < NH; ii++) {
              const int i = h2 * NH + ii;
              const int cch = (16 * i + 4 * (qi & 3)) >> 3, half = qi & 1;
              y[2 * ii] = ds_read_tr16(Vp + vr0 * rb + (cch ^ s0) * 16 + half * 8);
              y[2 * ii + 1] = ds_read_tr16(Vp + vr1 * rb + (cch ^ s1) * 16 + half * 8);
            }
            lgkm_wait_all<2 * NH>(y);
#pragma unroll
            for (int ii = 0; ii < NH; ii++) {
              const int i = h2 * NH + ii;
              const u32x4 va = u32x4{y[2 * ii][0], y[2 * ii][1], y[2 * ii + 1][0], y[2 * ii + 1][1]};
              o[i] = mfma_bf16(__builtin_bit_cast(u16x8, va), __builtin_bit_cast(u16x8, pb), o[i]);
            }
          }
        }
      }
    }  // steps
  }

  // ---- normalise and store: lane holds O[query qi][d = 16 i + 4 g4 + t]
  float l_tot = l_run + __shfl_xor(l_run, 16, 64);
  l_tot += __shfl_xor(l_tot, 32, 64);
  __syncthreads();  // LDS reused by the workgroup's next unit
  if (!qvalid) return;
  const float inv = l_tot > 0.f ? 1.f / l_tot : 0.f;
  bf16_t* out = reinterpret_cast<bf16_t*>(a.out) + qrow * a.out_stride + hq * D;
#pragma unroll
  for (int i = 0; i < ND; i++) {
    const int d0 = 16 * i + 4 * g4;
    u32x2 pk;
    pk[0] = pack_bf16x2(o[i][0] * inv, o[i][1] * inv);
    pk[1] = pack_bf16x2(o[i][2] * inv, o[i][3] * inv);
    *reinterpret_cast<u32x2*>(out + d0) = pk;
  }
}

// One workgroup per unit.
// 32-key compute steps keep three workgroups' registers per CU (and their tiles fit LDS), or
// four with two stages (128 VGPRs: four wavefronts per SIMD; 34 KB of LDS per workgroup);
// the register budget is capped to match
template <typename TKV, int D, int KT, int NS, int KC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KC == 32 ? (NS == 2 ? 4 : 3) : 1)))
void attn_dma_kernel(AttnArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t dma_smem[];
  attn_dma_unit<TKV, D, KT, NS, KC>(a, blockIdx.x, dma_smem);
}

// Persistent form: a fixed grid takes units from a device counter (zeroed by the caller
// before the launch) until every unit is taken; every workgroup exits once the counter
// passes the unit count, so the grid always drains.
template <typename TKV, int D, int KT, int NS, int KC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KC == 32 ? 3 : 1)))
void attn_dma_persistent_kernel(AttnArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t dma_smem[];
  __shared__ int next;
  const int total = a.n_work * a.Hkv;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(a.counter, 1);
    __syncthreads();
    const int unit = next;
    __syncthreads();
    if (unit >= total) break;
    attn_dma_unit<TKV, D, KT, NS, KC>(a, unit, dma_smem);
  }
}

template <typename TKV, int D, int KT, int NS, int KC = KT>
static hipError_t launch_dma(const AttnArgs& a, hipStream_t st) {
  using C = DmaCfg<TKV, D, KT, NS>;
  const int64_t units = (int64_t)a.n_work * a.Hkv;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)attn_dma_kernel<TKV, D, KT, NS, KC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_TOTAL);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)attn_dma_persistent_kernel<TKV, D, KT, NS, KC>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_TOTAL);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (a.counter) {
    // as many workgroups as are resident at once (registers and LDS decide: three per CU for
    // the 32-key compute steps); each takes units until the counter passes their number
    static int per_cu = 0;
    if (per_cu == 0) {
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, (const void*)attn_dma_persistent_kernel<TKV, D, KT, NS, KC>, 256, C::LDS_TOTAL);
      if (e != hipSuccess || per_cu < 1) per_cu = 2;
    }
    const int64_t wgs = (int64_t)per_cu * std::max(a.n_cu, 1);
    hipLaunchKernelGGL((attn_dma_persistent_kernel<TKV, D, KT, NS, KC>),
                       dim3((unsigned)std::min<int64_t>(units, wgs)), dim3(256), C::LDS_TOTAL, st, a);
  } else {
    hipLaunchKernelGGL((attn_dma_kernel<TKV, D, KT, NS, KC>), dim3((unsigned)units), dim3(256), C::LDS_TOTAL, st, a);
  }
  return hipGetLastError();
}

// variant: 0 = KT 64 / 2 stages, 1 = KT 64 / 3 stages, 2 = 32-key compute steps over tiles of
// 16 KiB of keys and values: 32-key tiles of a BF16 cache, 64-key tiles of an FP8 cache (its
// rows are half as long, so the tile moves the same bytes), each computed in 32-key steps.
// The BF16 form runs two stages and four resident workgroups per CU (one tile in flight per
// workgroup, four per CU): a step's chain of dependent operations is then hidden by four
// wavefronts per SIMD instead of three, and HBM needs no more bytes in flight per CU than
// that; its persistent form keeps three stages (at four wavefronts per SIMD it would spill).
// The FP8 form needs more registers (three workgroups per CU whatever the stages) and keeps
// three stages.  The stage count changes no arithmetic: all forms of a variant agree bit
// for bit.  (D = 64 has no 32-key variant: its FP8 tile would be under one chunk load per
// thread.)
template <typename TKV, int D>
static hipError_t launch_dma_variant(int variant, const AttnArgs& a, hipStream_t st) {
  if (variant == 0) return launch_dma<TKV, D, 64, 2>(a, st);
  if constexpr (D == 64) return launch_dma<TKV, D, 64, 3>(a, st);
  else {
    if (variant == 1) return launch_dma<TKV, D, 64, 3>(a, st);
    if constexpr (sizeof(TKV) == 1) return launch_dma<TKV, D, 64, 3, 32>(a, st);
    else if (a.counter) return launch_dma<TKV, D, 32, 3>(a, st);
    else return launch_dma<TKV, D, 32, 2>(a, st);
  }
}

// The attention kernels' FP8 -> BF16 widening applied to a code array (n a multiple of 8),
// for an exhaustive check against the format's definition.
__global__ void fp8_widen_kernel(const uint8_t* __restrict__ codes, uint16_t* __restrict__ out, int n8) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n8) return;
  const u32x2 raw = *reinterpret_cast<const u32x2*>(codes + 8 * i);
  *reinterpret_cast<u32x4*>(out + 8 * i) = fp8x8_to_bf16x8(raw[0], raw[1]);
}

hipError_t fp8_widen(const uint8_t* codes, uint16_t* out, int n, hipStream_t st) {
  if (n <= 0 || n % 8) return hipErrorInvalidValue;
  const int n8 = n / 8;
  hipLaunchKernelGGL(fp8_widen_kernel, dim3((n8 + 255) / 256), dim3(256), 0, st, codes, out, n8);
  return hipGetLastError();
}

hipError_t attention_dma(int kvdt, int D, int variant, const AttnArgs& a, hipStream_t st) {
  if (a.n_work <= 0) return hipSuccess;
  if (a.counter && a.persistent_wgs < 1) return hipErrorInvalidValue;
  if (a.G * a.Pmax > 64 || a.G < 1 || a.Pmax < 1) return hipErrorInvalidValue;
  if (kvdt == DT_BF16) {
    if (D == 128) return launch_dma_variant<bf16_t, 128>(variant, a, st);
    if (D == 64) return launch_dma_variant<bf16_t, 64>(variant, a, st);
  } else if (kvdt == DT_FP8) {
    if (D == 128) return launch_dma_variant<fp8_t, 128>(variant, a, st);
    if (D == 64) return launch_dma_variant<fp8_t, 64>(variant, a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace kvop
