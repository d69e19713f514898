// Dense projections of the decoder on MFMA: C = A B^T, both operands K-contiguous.
//
// Work split: one workgroup of NW (4 or 8) wavefronts per BM x BN output tile; each
// wavefront owns a WM x WN sub-tile built from 16x16 MFMA blocks.  Larger wavefront tiles
// read fewer LDS bytes per MFMA ((WM + WN) / (WM * WN) bytes per flop); eight wavefronts
// put two on every SIMD, so one's LDS reads overlap the other's MFMAs.  K advances in BK slabs staged in LDS
// (two buffers): the next slab is fetched from global memory into registers while the
// current one feeds the MFMAs, then written to the other buffer, one barrier per slab.
// FP32 uses v_mfma_f32_16x16x4f32 (four MFMAs per 16-byte LDS read); BF16 uses the
// gfx950 v_mfma_f32_16x16x32_bf16.  Accumulation is FP32 in every case.
// Epilogues: plain store (f32/bf16), FP32 residual add, SwiGLU over interleaved
// gate/up column blocks.  The workgroup -> tile order is XCD-aware and grouped (see the
// kernel body) so that concurrently resident workgroups of one XCD share A and B tiles.
#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace kvop {

// SWZ selects the LDS layout of a K-slab row (CPR 16-byte chunks):
//   0: padded rows (BK + one chunk) — chunk c of row r at r*LDK + c*VEC
//   1: unpadded, chunk c of row r stored at slot c ^ ((r >> 1) & (CPR-1))
//   2: unpadded, chunk c of row r stored at slot c ^ (r & (CPR-1))
// NS = 0: slabs staged through registers (two LDS buffers); NS >= 2: slabs fetched by
// direct global -> LDS loads into NS buffers, completion tracked with explicit vmcnt waits
// (every thread issues the same number of loads per slab), K a multiple of BK.
//
// SCH = 1 (direct loads): software-pipelined K loop.  The A/B fragments of the next MFMA
// step are read from LDS into a second register set while the current step's MFMAs run,
// and each slab's direct loads are issued between MFMAs; one workgroup barrier per slab,
// placed where the last fragments of a slab are already in registers.
template <typename T, typename TO, int BM, int BN, int BK, int WM, int WN, int EPI, int SWZ, int NW, int NS,
          int SCH = 0, int NSB = 0, int NSA = 0>
__global__ __launch_bounds__(64 * NW)
// pipelined 4-wavefront tiles with up to 128x64 per wavefront: registers for two resident
// workgroups, whose barriers and epilogues then overlap each other's MFMAs
__attribute__((amdgpu_waves_per_eu(SCH == 1 && NW == 4 && WM * WN <= 128 * 64 ? 2 : 1)))
void gemm_nt_kernel(const T* __restrict__ A, const T* __restrict__ B,
                                                      void* __restrict__ Cv, int M, int N, int K, int64_t lda,
                                                      int64_t ldb, int64_t ldc, int tiles_m, int gm, RopeEpi rp) {
  constexpr int VEC = 16 / (int)sizeof(T);  // elements per 16-byte chunk
  constexpr int LDK = BK + (SWZ == 0 ? VEC : 0);  // LDS row pitch (elements)
  constexpr int CPR = BK / VEC;             // chunks per tile row
  constexpr int NT = 64 * NW;               // threads
  constexpr int ACH = BM * CPR / NT;
  constexpr int BCH = BN * CPR / NT;
  constexpr int MI = WM / 16, NI = WN / 16;
  constexpr int WN_CNT = BN / WN;
  constexpr int KSUB = 4 * VEC;             // K consumed per MFMA step group
  auto slot = [](int r, int c) {            // LDS chunk slot of logical chunk c in row r
    if constexpr (SWZ == 1) return c ^ ((r >> 1) & (CPR - 1));
    else if constexpr (SWZ == 2) return c ^ (r & (CPR - 1));
    else if constexpr (SWZ == 3) return c ^ ((r >> 2) & (CPR - 1));
    else return c;
  };
  static_assert(NS == 0 || SWZ != 0, "direct loads write unpadded rows");
  static_assert((BM / WM) * (BN / WN) == NW, "one wavefront per sub-tile");
  static_assert(ACH * NT == BM * CPR && BCH * NT == BN * CPR, "tile/thread mismatch");
  static_assert(EPI != EPI_SWIGLU || (NI % 2 == 0), "swiglu needs gate/up block pairs");

  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  constexpr int STAGE = (BM + BN) * LDK;
  // NSA = NSB = 0: NS stages of [A slab | B slab].  Split stages (pipelined schedule only):
  // NA A-slab buffers followed by NB B-slab buffers, one operand fetched one slab further
  // ahead than the other (the 256x256 tile's two stages leave exactly one slab of LDS free).
  constexpr int NA = NSA ? NSA : NS, NB = NSB ? NSB : NS;
  constexpr bool SPLIT = NA != NS || NB != NS;
  static_assert(!SPLIT || (SCH == 1 && NS == 2 && NA + NB == 5), "split stages: pipelined, 2 + 3");
  auto a_base = [&](int bf) -> T* { return SPLIT ? smem + bf * BM * LDK : smem + bf * STAGE; };
  auto b_base = [&](int bf) -> T* { return SPLIT ? smem + NA * BM * LDK + bf * BN * LDK : smem + bf * STAGE + BM * LDK; };

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN_CNT, wn = wave % WN_CNT;
  // Tile order.  The dispatcher hands workgroup b to XCD b % 8; remap so that every XCD
  // owns one contiguous range of logical tiles, then walk that range in groups of GM
  // M-tiles x all N-tiles (M fastest inside a group) so that the A and B tiles of
  // concurrently resident workgroups are shared in that XCD's L2.  GM is a property of the
  // tile (4 or 8), left to the autotuner: on the 256x256 pipelined tile at M = 131072, 4 is
  // faster for gate/up, O and down and 8 for QKV.
  const int nblk = gridDim.x, bid = blockIdx.x;
  const int xcd = bid & 7, loc = bid >> 3, q = nblk >> 3, rem = nblk & 7;
  const int lt = (xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q) + loc;
  const int tiles_n = nblk / tiles_m;
  const int GM = gm;
  const int per_group = GM * tiles_n;
  const int first_m = (lt / per_group) * GM;
  const int gsz = min(tiles_m - first_m, GM);
  const int tm = first_m + (lt % per_group) % gsz, tn = (lt % per_group) / gsz;
  const int m0 = tm * BM, n0 = tn * BN;

  u32x4 ra[ACH], rb[BCH];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < ACH; i++) {
      int c = tid + i * NT, r = c / CPR, kc = (c % CPR) * VEC;
      int gm = m0 + r, gk = k0 + kc;
      ra[i] = (gm < M && gk < K) ? *reinterpret_cast<const u32x4*>(A + (int64_t)gm * lda + gk) : u32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < BCH; i++) {
      int c = tid + i * NT, r = c / CPR, kc = (c % CPR) * VEC;
      int gn = n0 + r, gk = k0 + kc;
      rb[i] = (gn < N && gk < K) ? *reinterpret_cast<const u32x4*>(B + (int64_t)gn * ldb + gk) : u32x4{0, 0, 0, 0};
    }
  };
  auto sstore = [&](int buf) {
    T* As = smem + buf * STAGE;
    T* Bs = As + BM * LDK;
#pragma unroll
    for (int i = 0; i < ACH; i++) {
      int c = tid + i * NT, r = c / CPR;
      *reinterpret_cast<u32x4*>(As + r * LDK + slot(r, c % CPR) * VEC) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BCH; i++) {
      int c = tid + i * NT, r = c / CPR;
      *reinterpret_cast<u32x4*>(Bs + r * LDK + slot(r, c % CPR) * VEC) = rb[i];
    }
  };

  // Accumulators start at zero, or for the residual add at the residual itself: its reads
  // (in the accumulator layout, lane -> C[.. + 4*(lane/16) + r][.. + lane%16]) then overlap
  // the first slabs instead of a read-modify-write pass after the last one.
  f32x4 acc[MI][NI];
  if constexpr (EPI == EPI_ADD) {
    const float* Cf = reinterpret_cast<const float*>(Cv);
    const int rb0 = m0 + wm * WM + 4 * (tid >> 4 & 3), cb0 = n0 + wn * WN + (tid & 15);
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
      for (int j = 0; j < NI; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = rb0 + 16 * i + r, col = cb0 + 16 * j;
          acc[i][j][r] = (row < M && col < N) ? Cf[(int64_t)row * ldc + col] : 0.f;
        }
  } else {
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
      for (int j = 0; j < NI; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }

  const int nk = (K + BK - 1) / BK;
  const int lrow = lane & 15, lg = lane >> 4;
  // direct loads of slab k0 into buffer buf: chunk f = i NT + 64 wave + lane lands at LDS
  // chunk f (row f / CPR, slot f % CPR) and holds logical chunk slot(row, f % CPR) (the
  // XOR swizzle is its own inverse); rows past M / N read the last row (never stored)
  auto dma_a = [&](int k0, int bf) {
    T* As = a_base(bf);
#pragma unroll
    for (int i = 0; i < ACH; i++) {
      const int f = tid + i * NT, r = f / CPR, c = slot(r, f % CPR);
      const uint8_t* g = reinterpret_cast<const uint8_t*>(
          A + (int64_t)min(m0 + r, M - 1) * lda + k0 + c * VEC);
      uint8_t* l = reinterpret_cast<uint8_t*>(As + (i * NT + 64 * wave) * VEC);
      __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)l, 16, 0, 0);
    }
  };
  auto dma_b = [&](int k0, int bf) {
    T* Bs = b_base(bf);
#pragma unroll
    for (int i = 0; i < BCH; i++) {
      const int f = tid + i * NT, r = f / CPR, c = slot(r, f % CPR);
      const uint8_t* g = reinterpret_cast<const uint8_t*>(
          B + (int64_t)min(n0 + r, N - 1) * ldb + k0 + c * VEC);
      uint8_t* l = reinterpret_cast<uint8_t*>(Bs + (i * NT + 64 * wave) * VEC);
      __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)l, 16, 0, 0);
    }
  };
  auto dma = [&](int k0, int bf) {
    dma_a(k0, bf);
    dma_b(k0, bf);
  };
  if constexpr (SCH == 1) {
    static_assert(NS >= 2 && sizeof(T) == 2 && (BK == KSUB || BK == 2 * KSUB),
                  "pipelined: direct loads, BF16, one or two MFMA steps per slab");
    constexpr int HS = BK / KSUB;                     // MFMA steps per slab
    constexpr int OPS = ACH + BCH;                    // direct loads per thread per slab
    // loads allowed in flight at the first wait (slab 0 landed) and at each slab boundary
    // (slab kt + 1 landed).  Split stages issue A0 B0 A1 B1 and the deeper operand's slab 2
    // ahead, then per boundary the shallower operand's slab kt + 2 followed by the deeper one's
    // slab kt + 3, so only that newest slab may still be in flight at a boundary
    constexpr int XOPS = NB > NA ? BCH : ACH;        // loads of the deeper operand's slab
    constexpr int VMW = SPLIT ? XOPS : (NS - 2) * OPS, VMP = SPLIT ? (NS - 1) * OPS + XOPS : (NS - 1) * OPS;
    static_assert(VMP <= 63, "vmcnt range");
    constexpr int VM_STEADY = (VMW & 15) | ((VMW >> 4) << 14) | (7 << 4) | (15 << 8);
    constexpr int VM_FIRST = (VMP & 15) | ((VMP >> 4) << 14) | (7 << 4) | (15 << 8);
    constexpr int LGKM0 = 0xC07F;
    // fragments of step hs of the slab in buffer bf
    auto rd = [&](int slab, int hs, u32x4* a_, u32x4* b_) __attribute__((always_inline)) {
      const T* As = a_base(slab % NA) + (wm * WM) * LDK;
      const T* Bs = b_base(slab % NB) + (wn * WN) * LDK;
#pragma unroll
      for (int i = 0; i < MI; i++)
        a_[i] = *reinterpret_cast<const u32x4*>(As + (i * 16 + lrow) * LDK + slot(lrow, hs * 4 + lg) * VEC);
#pragma unroll
      for (int j = 0; j < NI; j++)
        b_[j] = *reinterpret_cast<const u32x4*>(Bs + (j * 16 + lrow) * LDK + slot(lrow, hs * 4 + lg) * VEC);
    };
    // Every slab boundary issues exactly one slab of direct loads (past the last slab they
    // re-read slab nk - 1 into the buffer just freed, which is never read again), so the
    // number of loads in flight behind any slab is fixed and a step has no branches: one
    // basic block per step, free for the scheduler to interleave.
#pragma unroll
    for (int q = 0; q < NS; q++) dma(min(q, nk - 1) * BK, q);
#pragma unroll
    for (int q = NS; q < NB; q++) dma_b(min(q, nk - 1) * BK, q);
#pragma unroll
    for (int q = NS; q < NA; q++) dma_a(min(q, nk - 1) * BK, q);
    __builtin_amdgcn_s_waitcnt(VM_FIRST);             // slab 0 landed (this thread's part)
    __builtin_amdgcn_s_barrier();                     // ... and every thread's
    __builtin_amdgcn_sched_barrier(0);
    // one MFMA step: fragments c* (read during the previous step) feed the MFMAs while the
    // next step's fragments are read into n*; a step that ends a slab (HSV == HS - 1) first
    // waits for the next slab, passes the barrier and refills the buffer just consumed
    auto step = [&](int kt, auto hs_c, u32x4* ca, u32x4* cb, u32x4* na, u32x4* nb) __attribute__((always_inline)) {
      constexpr int HSV = decltype(hs_c)::value;
      int nsl = kt, nhs = HSV + 1;
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (HSV == HS - 1) {
        // slab kt + 1 visible, slab kt's buffer free (all its fragments are in registers)
        __builtin_amdgcn_s_waitcnt(VM_STEADY);
        __builtin_amdgcn_s_waitcnt(LGKM0);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (NA > NB) {
          dma_b(min(kt + NB, nk - 1) * BK, kt % NB);
          dma_a(min(kt + NA, nk - 1) * BK, kt % NA);
        } else {
          dma_a(min(kt + NA, nk - 1) * BK, kt % NA);
          dma_b(min(kt + NB, nk - 1) * BK, kt % NB);
        }
        nsl = min(kt + 1, nk - 1);
        nhs = 0;
      }
      rd(nsl, nhs, na, nb);
#pragma unroll
      for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NI; j++)
          acc[i][j] = mfma_bf16(__builtin_bit_cast(u16x8, ca[i]), __builtin_bit_cast(u16x8, cb[j]), acc[i][j]);
      // issue order: an MFMA first (its fragments are the previous step's reads), then the
      // slab's direct loads and the next step's LDS reads, one per MFMA, so that their
      // latency hides behind this step's remaining MFMAs
      if constexpr (HSV == HS - 1) {
#pragma unroll
        for (int q = 0; q < OPS; q++) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // VMEM read
        }
      }
#pragma unroll
      for (int q = 0; q < MI + NI; q++) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);     // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);     // DS read
      }
      __builtin_amdgcn_sched_group_barrier(0x008, MI * NI, 0);  // the remaining MFMAs
      __builtin_amdgcn_sched_barrier(0);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    u32x4 fa0[MI], fb0[NI], fa1[MI], fb1[NI];
    rd(0, 0, fa0, fb0);
    if constexpr (HS == 2) {
      for (int kt = 0; kt < nk; kt++) {
        step(kt, I0{}, fa0, fb0, fa1, fb1);
        step(kt, I1{}, fa1, fb1, fa0, fb0);
      }
    } else {
      for (int kt = 0; kt < nk; kt += 2) {
        step(kt, I0{}, fa0, fb0, fa1, fb1);
        if (kt + 1 < nk) step(kt + 1, I0{}, fa1, fb1, fa0, fb0);
      }
    }
  } else {
  int buf = 0;
  if constexpr (NS == 0) {
    gload(0);
    sstore(0);
    __syncthreads();
  } else {
#pragma unroll
    for (int s = 0; s < NS - 1; s++)
      if (s < nk) dma(s * BK, s);
  }
  for (int kt = 0; kt < nk; kt++) {
    if constexpr (NS == 0) {
      if (kt + 1 < nk) gload((kt + 1) * BK);
    } else {
      // slab kt has landed once only the later slabs' loads (NS - 2 of them) are in flight
      constexpr int OPS = ACH + BCH;
      constexpr int W = (NS - 2) * OPS;
      static_assert(W <= 63, "vmcnt range");
      if (kt + NS - 2 < nk) __builtin_amdgcn_s_waitcnt((W & 15) | ((W >> 4) << 14) | (7 << 4) | (15 << 8));
      else __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
      __builtin_amdgcn_s_barrier();  // all loads of slab kt visible; slab kt - 1 consumed
      buf = kt % NS;
      if (kt + NS - 1 < nk) dma((kt + NS - 1) * BK, (kt + NS - 1) % NS);
    }
    const T* As = smem + buf * STAGE + (wm * WM) * LDK;
    const T* Bs = smem + buf * STAGE + BM * LDK + (wn * WN) * LDK;
#pragma unroll
    for (int ks = 0; ks < BK; ks += KSUB) {
      u32x4 af[MI], bfr[NI];
#pragma unroll
      for (int i = 0; i < MI; i++)
        af[i] = *reinterpret_cast<const u32x4*>(As + (i * 16 + lrow) * LDK + slot(lrow, ks / VEC + lg) * VEC);
#pragma unroll
      for (int j = 0; j < NI; j++)
        bfr[j] = *reinterpret_cast<const u32x4*>(Bs + (j * 16 + lrow) * LDK + slot(lrow, ks / VEC + lg) * VEC);
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int t = 0; t < 4; t++)
#pragma unroll
          for (int i = 0; i < MI; i++)
#pragma unroll
            for (int j = 0; j < NI; j++)
              acc[i][j] = mfma_f32(as_f32(af[i][t]), as_f32(bfr[j][t]), acc[i][j]);
      } else {
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
          for (int j = 0; j < NI; j++)
            acc[i][j] = mfma_bf16(__builtin_bit_cast(u16x8, af[i]), __builtin_bit_cast(u16x8, bfr[j]), acc[i][j]);
      }
    }
    if constexpr (NS == 0) {
      if (kt + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  }
  if constexpr (NS != 0) __syncthreads();  // every wavefront is done with the slabs (LDS reused below)

  if constexpr (EPI == EPI_ROPE) {
    // ---- rotary epilogue: the tile's products, rounded to BF16, staged row-major in LDS
    // (pitch BN + 8), then each thread takes 8-pair groups (dimensions i .. i+7 and
    // i + D/2 .. i + D/2 + 7 of one head of one row) and rotates them at the row's position
    // (heads in [0, rot_cols)); the rotation reads the rounded values, as a separate pass
    // over the stored products would.  Rows are written with 16-byte stores.
    static_assert(sizeof(T) == 2 && sizeof(TO) == 2, "rotary epilogue: BF16");
    if constexpr (NS == 0) __syncthreads();
    constexpr int TP = BN + 8;
    bf16_t* Tt = reinterpret_cast<bf16_t*>(smem_raw);
    // Lanes 2c and 2c + 1 hold columns 2c and 2c + 1 of the same four rows: a swap of two
    // values between them (a DPP move) lets the even lane write rows 0-1 and the odd lane
    // rows 2-3 of the pair as packed BF16 pairs, one 4-byte store each.
    const bool odd = lane & 1;
    const int prow = 4 * (lane >> 4) + (odd ? 2 : 0), pcol = (lane & 15) & ~1;
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
      for (int j = 0; j < NI; j++) {
        const f32x4 v = acc[i][j];
        const float s0 = odd ? v[0] : v[2], s1 = odd ? v[1] : v[3];
        const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s0), 0xB1,
                                                                                0xF, 0xF, false));
        const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s1), 0xB1,
                                                                                0xF, 0xF, false));
        const uint32_t w0 = odd ? pack_bf16x2(r0, v[2]) : pack_bf16x2(v[0], r0);
        const uint32_t w1 = odd ? pack_bf16x2(r1, v[3]) : pack_bf16x2(v[1], r1);
        bf16_t* t = Tt + (wm * WM + 16 * i + prow) * TP + wn * WN + 16 * j + pcol;
        *reinterpret_cast<uint32_t*>(t) = w0;
        *reinterpret_cast<uint32_t*>(t + TP) = w1;
      }
    __syncthreads();
    const int D = rp.D, half = D >> 1, gph = half >> 3;     // 8-pair groups per head
    const int upr = (BN / D) * gph;                           // groups per tile row
    bf16_t* C = reinterpret_cast<bf16_t*>(Cv);
    bf16_t* Qa = reinterpret_cast<bf16_t*>(rp.q_alt);
    // BM * BN / 16 groups whatever D is: a fixed count per thread, fully unrolled so that the
    // position and table loads of all of them can be in flight together
    constexpr int NU = BM * BN / 16 / NT;
    static_assert(NU * 16 * NT == BM * BN, "rotary groups per thread");
    // phase 1: which group (row, head, 8 dimensions) each of this thread's NU groups is, and
    // its row's position; phase 2: the table rows at those positions; phase 3: rotate and
    // store.  No load sits behind a branch, so the loads of every group are in flight at once.
    const int ps = rp.pos_stride > 0 ? rp.pos_stride : 1;
    int gm_[NU], col_[NU], off_[NU], p_[NU];
#pragma unroll
    for (int k = 0; k < NU; k++) {
      const int u = tid + NT * k;
      const int row = u / upr, w = u - row * upr;
      const int hh = w / gph, i = (w - hh * gph) * 8;
      gm_[k] = m0 + row;
      col_[k] = n0 + hh * D + i;
      off_[k] = row * TP + hh * D + i;
      p_[k] = rp.pos[(int64_t)min(gm_[k], M - 1) * ps];
    }
    f32x4 ct_[NU][2], st_[NU][2];
#pragma unroll
    for (int k = 0; k < NU; k++) {
      const int i = col_[k] % half;
      const f32x4* cp = reinterpret_cast<const f32x4*>(rp.cos_t + (int64_t)p_[k] * half + i);
      const f32x4* sp = reinterpret_cast<const f32x4*>(rp.sin_t + (int64_t)p_[k] * half + i);
      ct_[k][0] = cp[0];
      ct_[k][1] = cp[1];
      st_[k][0] = sp[0];
      st_[k][1] = sp[1];
    }
#pragma unroll
    for (int k = 0; k < NU; k++) {
      const int gm = gm_[k], col = col_[k];
      if (gm >= M || col >= N) continue;                    // N is a multiple of D
      const u32x4 r1 = *reinterpret_cast<const u32x4*>(Tt + off_[k]);
      const u32x4 r2 = *reinterpret_cast<const u32x4*>(Tt + off_[k] + half);
      bf16_t* c1 = C + (int64_t)gm * ldc + col;
      if (col >= rp.rot_cols) {
        *reinterpret_cast<u32x4*>(c1) = r1;
        *reinterpret_cast<u32x4*>(c1 + half) = r2;
        continue;
      }
      float x1[8], x2[8];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        x1[2 * q] = __builtin_bit_cast(float, r1[q] << 16);
        x1[2 * q + 1] = __builtin_bit_cast(float, r1[q] & 0xffff0000u);
        x2[2 * q] = __builtin_bit_cast(float, r2[q] << 16);
        x2[2 * q + 1] = __builtin_bit_cast(float, r2[q] & 0xffff0000u);
      }
      auto rotate_store = [&](const f32x4& ca, const f32x4& cb, const f32x4& sa, const f32x4& sb, bf16_t* dst) {
        float y1[8], y2[8];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          rope_pair(x1[e], x2[e], ca[e], sa[e], y1[e], y2[e]);
          rope_pair(x1[4 + e], x2[4 + e], cb[e], sb[e], y1[4 + e], y2[4 + e]);
        }
        u32x4 o1, o2;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          o1[q] = pack_bf16x2(y1[2 * q], y1[2 * q + 1]);
          o2[q] = pack_bf16x2(y2[2 * q], y2[2 * q + 1]);
        }
        *reinterpret_cast<u32x4*>(dst) = o1;
        *reinterpret_cast<u32x4*>(dst + half) = o2;
      };
      if (Qa && col < rp.q_cols && rp.shift[(int64_t)gm * ps] >= 0) {
        // joins: the query rotated at position - shift (rare rows; loads taken here)
        const int p2 = p_[k] - rp.shift[(int64_t)gm * ps], i = col % half;
        const f32x4* cp = reinterpret_cast<const f32x4*>(rp.cos_t + (int64_t)p2 * half + i);
        const f32x4* sp = reinterpret_cast<const f32x4*>(rp.sin_t + (int64_t)p2 * half + i);
        rotate_store(cp[0], cp[1], sp[0], sp[1], Qa + (int64_t)gm * ldc + col);
      }
      rotate_store(ct_[k][0], ct_[k][1], st_[k][0], st_[k][1], c1);
    }
    return;
  }

  // ---- epilogue.  Lane holds C[row0 + 4*(lane/16) + r][col0 + 16*j + lane%16].  Output
  // columns of one 16-row slab are first formed in registers (SwiGLU pairs gate block j with
  // up block j+1), staged row-major through this wavefront's slice of LDS (free after the
  // last barrier), then written with 16-byte row-contiguous accesses (the residual add has
  // its sum in the accumulators already).  A ragged column edge or an unaligned C uses
  // scalar accesses.
  constexpr int OW = EPI == EPI_SWIGLU ? WN / 2 : WN;       // output columns per wavefront
  constexpr int OJ = OW / 16;                               // 16-column output blocks
  constexpr int EP = OW + 4;                                // LDS slab pitch (floats)
  constexpr bool OUT_BF16 = sizeof(TO) == 2;
  constexpr int VW = OUT_BF16 ? 8 : 4;                      // output elements per 16-byte access
  constexpr int LPR = OW / VW;                              // lanes per row
  constexpr int RPP = 64 / LPR;                             // rows per pass
  static_assert(64 % LPR == 0 && 16 % RPP == 0, "epilogue lane split");
  static_assert(NW * 16 * EP * 4 <= (NS == 0 ? 2 : NS) * (BM + BN) * LDK * (int)sizeof(T),
                "epilogue staging fits the slab buffers");
  const int n_out = EPI == EPI_SWIGLU ? N / 2 : N;
  const int col0 = (EPI == EPI_SWIGLU ? (n0 + wn * WN) / 2 : n0 + wn * WN);
  float* E = reinterpret_cast<float*>(smem_raw) + wave * 16 * EP;
  const bool vec_ok = (ldc % VW) == 0 && ((reinterpret_cast<uintptr_t>(Cv) & 15) == 0);
#pragma unroll
  for (int i = 0; i < MI; i++) {
    const int row_base = m0 + wm * WM + i * 16;
#pragma unroll
    for (int jj = 0; jj < OJ; jj++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        float v;
        if constexpr (EPI == EPI_SWIGLU) v = silu(acc[i][2 * jj][r]) * acc[i][2 * jj + 1][r];
        else v = acc[i][jj][r];
        E[(4 * (lane >> 4) + r) * EP + jj * 16 + (lane & 15)] = v;
      }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wavefront's LDS writes are done
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int pass = 0; pass < 16 / RPP; pass++) {
      const int rr = pass * RPP + lane / LPR, cc = (lane % LPR) * VW;
      const int row = row_base + rr, col = col0 + cc;
      const float* e = E + rr * EP + cc;
      if (row < M) {
        if (vec_ok && col + VW <= n_out) {
          if constexpr (OUT_BF16) {
            u32x4 pk;
#pragma unroll
            for (int q = 0; q < 4; q++) pk[q] = pack_bf16x2(e[2 * q], e[2 * q + 1]);
            *reinterpret_cast<u32x4*>(reinterpret_cast<TO*>(Cv) + (int64_t)row * ldc + col) = pk;
          } else {
            *reinterpret_cast<f32x4*>(reinterpret_cast<float*>(Cv) + (int64_t)row * ldc + col) =
                *reinterpret_cast<const f32x4*>(e);
          }
        } else {
#pragma unroll
          for (int q = 0; q < VW; q++) {
            if (col + q >= n_out) break;
            reinterpret_cast<TO*>(Cv)[(int64_t)row * ldc + col + q] = from_f32<TO>(e[q]);
          }
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // the slab's LDS reads are done before the next slab's writes
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------------ tile table
struct TileCfg {
  int BM, BN, BK, WM, WN, SWZ, NW, NS;
  const char* name;
};
static const TileCfg kF32Tiles[] = {
    {128, 128, 32, 64, 64, 0, 4, 0, "f32_128x128x32_w64x64"},
    {64, 128, 32, 32, 64, 0, 4, 0, "f32_64x128x32_w32x64"},
    {128, 64, 32, 64, 32, 0, 4, 0, "f32_128x64x32_w64x32"},
    {128, 128, 32, 64, 64, 1, 4, 0, "f32_128x128x32_w64x64_swz1"},
};
static const TileCfg kBf16Tiles[] = {
    {128, 128, 64, 64, 64, 0, 4, 0, "bf16_128x128x64_w64x64"},
    {256, 128, 64, 128, 64, 0, 4, 0, "bf16_256x128x64_w128x64"},
    {128, 256, 64, 64, 128, 0, 4, 0, "bf16_128x256x64_w64x128"},
    {64, 128, 64, 32, 64, 0, 4, 0, "bf16_64x128x64_w32x64"},
    {256, 256, 64, 128, 128, 0, 4, 0, "bf16_256x256x64_w128x128"},
    {256, 256, 32, 128, 128, 0, 4, 0, "bf16_256x256x32_w128x128"},
    {128, 128, 64, 64, 64, 1, 4, 0, "bf16_128x128x64_w64x64_swz1"},
    {128, 128, 64, 64, 64, 2, 4, 0, "bf16_128x128x64_w64x64_swz2"},
    {256, 256, 64, 128, 128, 1, 4, 0, "bf16_256x256x64_w128x128_swz1"},
    {256, 128, 64, 128, 64, 1, 4, 0, "bf16_256x128x64_w128x64_swz1"},
    {256, 256, 64, 128, 64, 1, 8, 0, "bf16_256x256x64_8w_w128x64_swz1"},
    {256, 256, 64, 64, 128, 1, 8, 0, "bf16_256x256x64_8w_w64x128_swz1"},
    {256, 256, 64, 128, 64, 2, 8, 0, "bf16_256x256x64_8w_w128x64_swz2"},
    {256, 256, 64, 128, 64, 0, 8, 0, "bf16_256x256x64_8w_w128x64"},
    {256, 128, 64, 64, 64, 1, 8, 0, "bf16_256x128x64_8w_w64x64_swz1"},
    {128, 256, 64, 64, 64, 1, 8, 0, "bf16_128x256x64_8w_w64x64_swz1"},
    {256, 256, 64, 64, 128, 1, 8, 2, "bf16_256x256x64_8w_w64x128_swz1_lds2"},
    {256, 256, 32, 64, 128, 3, 8, 3, "bf16_256x256x32_8w_w64x128_swz3_lds3"},
    {256, 256, 32, 64, 128, 3, 8, 4, "bf16_256x256x32_8w_w64x128_swz3_lds4"},
    {256, 256, 64, 128, 64, 1, 8, 2, "bf16_256x256x64_8w_w128x64_swz1_lds2"},
    {256, 256, 64, 128, 64, 1, 8, 2, "bf16_256x256x64_8w_w128x64_swz1_lds2_pipe"},
    {256, 128, 32, 128, 64, 3, 4, 3, "bf16_256x128x32_w128x64_swz3_lds3_pipe"},
    {128, 256, 32, 64, 128, 3, 4, 3, "bf16_128x256x32_w64x128_swz3_lds3_pipe"},
    {256, 128, 32, 128, 64, 3, 4, 2, "bf16_256x128x32_w128x64_swz3_lds2_pipe"},
    {256, 256, 64, 128, 64, 1, 8, 2, "bf16_256x256x64_8w_w128x64_swz1_lds2_pipe_g4"},
    {256, 256, 64, 128, 64, 1, 8, 2, "bf16_256x256x64_8w_w128x64_swz1_lds2b3_pipe_g4"},
    {256, 256, 64, 128, 64, 1, 8, 2, "bf16_256x256x64_8w_w128x64_swz1_lds2a3_pipe_g4"},
};

int gemm_num_tiles(int dt) { return dt == DT_F32 ? 4 : 27; }
const char* gemm_tile_name(int dt, int t) { return dt == DT_F32 ? kF32Tiles[t].name : kBf16Tiles[t].name; }

static const TileCfg& tile_cfg(int dt, int t) { return dt == DT_F32 ? kF32Tiles[t] : kBf16Tiles[t]; }

bool gemm_tile_ok(int dt, int t, const GemmShape& s, int epi) {
  if (t < 0 || t >= gemm_num_tiles(dt)) return false;
  const TileCfg& c = tile_cfg(dt, t);
  int vec = dt == DT_F32 ? 4 : 8;
  if (s.K % vec || s.lda % vec || s.ldb % vec) return false;
  if (epi == EPI_SWIGLU && (s.N % 32 || (c.WN % 32))) return false;
  if (epi == EPI_ROPE && (dt != DT_BF16 || c.BN % 128)) return false;   // whole heads of D <= 128 per tile
  if (c.NS && s.K % c.BK) return false;   // direct-load tiles read whole slabs only
  return true;
}

template <typename T, typename TO, int EPI, int BM, int BN, int BK, int WM, int WN, int SWZ, int NW = 4, int NS = 0,
          int SCH = 0, int NSB = 0, int NSA = 0>
static hipError_t launch_t(const void* A, const void* B, void* C, const GemmShape& s, hipStream_t st,
                           const RopeEpi& rp, int gm = 8) {
  int tiles_m = (s.M + BM - 1) / BM, tiles_n = (s.N + BN - 1) / BN;
  const size_t ldk = BK + (SWZ == 0 ? 16 / sizeof(T) : 0);
  size_t lds = (NSA || NSB) ? ((size_t)(NSA ? NSA : NS) * BM + (size_t)(NSB ? NSB : NS) * BN) * ldk * sizeof(T)
                           : (NS == 0 ? 2 : NS) * (size_t)(BM + BN) * ldk * sizeof(T);
  if (EPI == EPI_ROPE) lds = std::max(lds, (size_t)BM * (BN + 8) * 2);   // the staged BF16 tile
  auto kern = gemm_nt_kernel<T, TO, BM, BN, BK, WM, WN, EPI, SWZ, NW, NS, SCH, NSB, NSA>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3(tiles_m * tiles_n), dim3(64 * NW), lds, st, (const T*)A, (const T*)B, C, s.M, s.N, s.K,
                     s.lda, s.ldb, s.ldc, tiles_m, gm, rp);
  return hipGetLastError();
}

template <typename T, typename TO, int EPI>
static hipError_t launch_cfg(int tile, const void* A, const void* B, void* C, const GemmShape& s, hipStream_t st,
                             const RopeEpi& rp) {
  if constexpr (sizeof(T) == 4) {
    switch (tile) {
      case 0: return launch_t<T, TO, EPI, 128, 128, 32, 64, 64, 0>(A, B, C, s, st, rp);
      case 1: return launch_t<T, TO, EPI, 64, 128, 32, 32, 64, 0>(A, B, C, s, st, rp);
      case 2: return launch_t<T, TO, EPI, 128, 64, 32, 64, 32, 0>(A, B, C, s, st, rp);
      default: return launch_t<T, TO, EPI, 128, 128, 32, 64, 64, 1>(A, B, C, s, st, rp);
    }
  } else {
    switch (tile) {
      case 0: return launch_t<T, TO, EPI, 128, 128, 64, 64, 64, 0>(A, B, C, s, st, rp);
      case 1: return launch_t<T, TO, EPI, 256, 128, 64, 128, 64, 0>(A, B, C, s, st, rp);
      case 2: return launch_t<T, TO, EPI, 128, 256, 64, 64, 128, 0>(A, B, C, s, st, rp);
      case 3: return launch_t<T, TO, EPI, 64, 128, 64, 32, 64, 0>(A, B, C, s, st, rp);
      case 4: return launch_t<T, TO, EPI, 256, 256, 64, 128, 128, 0>(A, B, C, s, st, rp);
      case 5: return launch_t<T, TO, EPI, 256, 256, 32, 128, 128, 0>(A, B, C, s, st, rp);
      case 6: return launch_t<T, TO, EPI, 128, 128, 64, 64, 64, 1>(A, B, C, s, st, rp);
      case 7: return launch_t<T, TO, EPI, 128, 128, 64, 64, 64, 2>(A, B, C, s, st, rp);
      case 8: return launch_t<T, TO, EPI, 256, 256, 64, 128, 128, 1>(A, B, C, s, st, rp);
      case 9: return launch_t<T, TO, EPI, 256, 128, 64, 128, 64, 1>(A, B, C, s, st, rp);
      case 10: return launch_t<T, TO, EPI, 256, 256, 64, 128, 64, 1, 8>(A, B, C, s, st, rp);
      case 11: return launch_t<T, TO, EPI, 256, 256, 64, 64, 128, 1, 8>(A, B, C, s, st, rp);
      case 12: return launch_t<T, TO, EPI, 256, 256, 64, 128, 64, 2, 8>(A, B, C, s, st, rp);
      case 13: return launch_t<T, TO, EPI, 256, 256, 64, 128, 64, 0, 8>(A, B, C, s, st, rp);
      case 14: return launch_t<T, TO, EPI, 256, 128, 64, 64, 64, 1, 8>(A, B, C, s, st, rp);
      case 15: return launch_t<T, TO, EPI, 128, 256, 64, 64, 64, 1, 8>(A, B, C, s, st, rp);
      case 16: return launch_t<T, TO, EPI, 256, 256, 64, 64, 128, 1, 8, 2>(A, B, C, s, st, rp);
      case 17: return launch_t<T, TO, EPI, 256, 256, 32, 64, 128, 3, 8, 3>(A, B, C, s, st, rp);
      case 18: return launch_t<T, TO, EPI, 256, 256, 32, 64, 128, 3, 8, 4>(A, B, C, s, st, rp);
      case 19: return launch_t<T, TO, EPI, 256, 256, 64, 128, 64, 1, 8, 2>(A, B, C, s, st, rp);
      case 20: return launch_t<T, TO, EPI, 256, 256, 64, 128, 64, 1, 8, 2, 1>(A, B, C, s, st, rp);
      case 21: return launch_t<T, TO, EPI, 256, 128, 32, 128, 64, 3, 4, 3, 1>(A, B, C, s, st, rp);
      case 22: return launch_t<T, TO, EPI, 128, 256, 32, 64, 128, 3, 4, 3, 1>(A, B, C, s, st, rp);
      case 23: return launch_t<T, TO, EPI, 256, 128, 32, 128, 64, 3, 4, 2, 1>(A, B, C, s, st, rp);
      case 24: return launch_t<T, TO, EPI, 256, 256, 64, 128, 64, 1, 8, 2, 1>(A, B, C, s, st, rp, 4);
      case 25: return launch_t<T, TO, EPI, 256, 256, 64, 128, 64, 1, 8, 2, 1, 3>(A, B, C, s, st, rp, 4);
      default: return launch_t<T, TO, EPI, 256, 256, 64, 128, 64, 1, 8, 2, 1, 0, 3>(A, B, C, s, st, rp, 4);
    }
  }
}

bool gemm_rope_supported(int D) { return D >= 16 && D % 16 == 0 && 128 % D == 0; }

hipError_t gemm(int dt, int out_dt, int epi, int tile, const void* A, const void* B, void* C, const GemmShape& s,
                hipStream_t st, const RopeEpi* rope) {
  if (s.M <= 0 || s.N <= 0) return hipSuccess;
  if (!gemm_tile_ok(dt, tile, s, epi)) return hipErrorInvalidValue;
  const RopeEpi none{};
  if (epi == EPI_ROPE) {
    // whole heads per tile (every BF16 tile is 128 or 256 columns wide: D divides 128), 8-pair
    // groups (D a multiple of 16) and 16-byte rows
    if (!rope || dt != DT_BF16 || out_dt != DT_BF16 || !gemm_rope_supported(rope->D) || s.N % rope->D ||
        s.ldc % 8 || (reinterpret_cast<uintptr_t>(C) & 15) || (rope->q_alt && !rope->shift) || !rope->pos ||
        (reinterpret_cast<uintptr_t>(rope->q_alt) & 15))
      return hipErrorInvalidValue;
    return launch_cfg<bf16_t, bf16_t, EPI_ROPE>(tile, A, B, C, s, st, *rope);
  }
  if (dt == DT_F32) {
    if (epi == EPI_ADD) return launch_cfg<float, float, EPI_ADD>(tile, A, B, C, s, st, none);
    if (epi == EPI_SWIGLU) return launch_cfg<float, float, EPI_SWIGLU>(tile, A, B, C, s, st, none);
    return launch_cfg<float, float, EPI_STORE>(tile, A, B, C, s, st, none);
  }
  if (epi == EPI_ADD) return launch_cfg<bf16_t, float, EPI_ADD>(tile, A, B, C, s, st, none);
  if (epi == EPI_SWIGLU) return launch_cfg<bf16_t, bf16_t, EPI_SWIGLU>(tile, A, B, C, s, st, none);
  if (out_dt == DT_F32) return launch_cfg<bf16_t, float, EPI_STORE>(tile, A, B, C, s, st, none);
  return launch_cfg<bf16_t, bf16_t, EPI_STORE>(tile, A, B, C, s, st, none);
}

// ------------------------------------------------------------------ tile choice
// Tuned winners keyed by (dtype, epilogue, N, K, M bucket); filled by the autotuner.
static std::map<std::tuple<int, int, int, int, int>, int>& tuned() {
  static std::map<std::tuple<int, int, int, int, int>, int> t;
  return t;
}
static int mbucket(int M) {
  int b = 0;
  while ((1 << (b + 1)) <= M && b < 30) b++;
  return b;
}
void gemm_set_tuned(int dt, int epi, int N, int K, int mb, int tile) { tuned()[{dt, epi, N, K, mb}] = tile; }
int gemm_mbucket(int M) { return mbucket(M); }

std::string gemm_tuned_export() {
  std::string out;
  for (auto& kv : tuned()) {
    int dt, epi, N, K, mb;
    std::tie(dt, epi, N, K, mb) = kv.first;
    out += std::to_string(dt) + " " + std::to_string(epi) + " " + std::to_string(N) + " " + std::to_string(K) + " " +
           std::to_string(mb) + " " + gemm_tile_name(dt, kv.second) + "\n";
  }
  return out;
}

bool gemm_tuned_import_line(int dt, int epi, int N, int K, int mb, const std::string& name) {
  for (int t = 0; t < gemm_num_tiles(dt); t++)
    if (name == gemm_tile_name(dt, t)) {
      gemm_set_tuned(dt, epi, N, K, mb, t);
      return true;
    }
  return false;
}

int gemm_pick_tile(int dt, int epi, const GemmShape& s) {
  if (epi == EPI_ROPE) epi = EPI_STORE;   // same main loop; the store epilogue's tuning applies
  auto it = tuned().find({dt, epi, s.N, s.K, mbucket(s.M)});
  if (it != tuned().end() && gemm_tile_ok(dt, it->second, s, epi)) return it->second;
  if (dt == DT_F32) return s.M <= 64 ? 1 : 0;
  if (s.M <= 128) return 3;        // 64x128
  if (s.M < 8192) return 7;        // 128x128, 4 wavefronts
  if (gemm_tile_ok(dt, 26, s, epi)) return 26;  // 256x256, 8 wavefronts of 128x64, direct loads, pipelined,
                                                // groups of 4 M-tiles, a third A-slab stage
  return 11;                       // 256x256, 8 wavefronts of 64x128
}

}  // namespace kvop
