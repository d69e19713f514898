// Shared device helpers for the gfx950 kernels: number formats, MFMA wrappers,
// wavefront reductions.  Wavefronts are 64 lanes wide.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kvop {

typedef uint16_t bf16_t;  // bfloat16 bit pattern in memory
typedef uint8_t fp8_t;    // OCP E4M3 (fn) code in memory

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// float -> bfloat16, round to nearest even (NaN kept quiet).  On the device this is the
// hardware conversion (v_cvt_pk_bf16_f32); the host keeps the same rounding in integer code.
__device__ __host__ inline bf16_t f2bf(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_bit_cast(bf16_t, (__bf16)f);
#else
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
#endif
}
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
// two floats -> packed bfloat16 pair (low = a), one v_cvt_pk_bf16_f32
__device__ inline uint32_t pack_bf16x2(float a, float b) {
  bf16x2_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
// low 16 bits from lo's half h, high 16 bits from hi's half h (one v_perm_b32)
__device__ inline uint32_t pair_halves(uint32_t lo, uint32_t hi, int h) {
  return __builtin_amdgcn_perm(hi, lo, h ? 0x07060302u : 0x05040100u);
}
__device__ __host__ inline float bf2f(bf16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// E4M3 (fn) code -> float.  Normal codes: exponent bias 7, 3 mantissa bits, placed in
// binary32 bit positions and rescaled by 2^120; subnormal codes (exponent 0): m * 2^-9.
__device__ inline float e4m3_to_f32(uint32_t c) {
  float mag = ((c & 0x78u) == 0) ? (float)(c & 7u) * 0x1p-9f
                                 : __builtin_bit_cast(float, (c & 0x7fu) << 20) * 0x1p120f;
  return (c & 0x80u) ? -mag : mag;
}
// E4M3 code -> bfloat16 bits (exact: every E4M3 value is a bfloat16 value)
__device__ inline uint32_t e4m3_to_bf16(uint32_t c) {
  return __builtin_bit_cast(uint32_t, e4m3_to_f32(c)) >> 16;
}

// eight E4M3 codes (two dwords, code 0 in the low byte of lo) -> eight bfloat16 values,
// by the hardware conversion (exact: every E4M3 value is a bfloat16 value)
__device__ inline u32x4 fp8x8_to_bf16x8(uint32_t lo, uint32_t hi) {
  u32x4 r;
  r[0] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 1.0f, false));
  r[1] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 1.0f, true));
  r[2] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 1.0f, false));
  r[3] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 1.0f, true));
  return r;
}

// float -> E4M3 (fn) code, round to nearest even, saturating to +-448.
__device__ inline uint32_t f32_to_e4m3(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  uint32_t sign = (u >> 24) & 0x80u;
  float a = fabsf(x);
  uint32_t code;
  if (!(a < 448.0f)) {                      // also catches +inf; NaN never reaches here in use
    code = 0x7eu;
  } else if (a < 0x1p-6f) {                 // subnormal range: multiples of 2^-9
    code = (uint32_t)rintf(a * 512.0f);     // 0..8 (8 is the smallest normal, code 0x08)
  } else {
    uint32_t ua = __builtin_bit_cast(uint32_t, a);
    int e = (int)((ua >> 23) & 0xff) - 127;  // -6..8
    uint32_t m = ua & 0x7fffffu;
    uint32_t m3 = m >> 20, rem = m & 0xfffffu;
    if (rem > 0x80000u || (rem == 0x80000u && (m3 & 1u))) m3++;
    if (m3 == 8u) { m3 = 0; e++; }
    code = ((uint32_t)(e + 7) << 3) | m3;
    if (code > 0x7eu) code = 0x7eu;
  }
  return code | sign;
}

// Rotary embedding of one pair (x1 at dimension i, x2 at i + D/2) by the angle with cosine c
// and sine s.  The roundings are spelled out (one product rounded, then a fused multiply-add)
// so that every kernel that rotates gives the same bits.
__device__ inline void rope_pair(float x1, float x2, float c, float s, float& y1, float& y2) {
  y1 = __builtin_fmaf(x1, c, -(x2 * s));
  y2 = __builtin_fmaf(x2, c, x1 * s);
}

// Reinterpret a 32-bit lane value as float.  Takes the value by copy: a bit_cast applied
// directly to an ext-vector element subscript reads element 0 of the vector.
__device__ inline float as_f32(uint32_t v) { return __builtin_bit_cast(float, v); }

__device__ inline float silu(float x) { return x / (1.0f + __expf(-x)); }

// wavefront reductions (64 lanes)
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// MFMA wrappers.  16x16 output blocks; lane l holds C[4*(l/16) + r][l % 16], r = 0..3.
// f32: A lane value A[l%16][k], B lane value B[k][l%16], k = l/16 (4 deep).
__device__ inline f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// bf16: A lane values A[l%16][8*(l/16) + 0..7], B lane values B[8*(l/16) + 0..7][l%16] (32 deep).
__device__ inline f32x4 mfma_bf16(u16x8 a, u16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

template <typename T> struct elem_bytes;
template <> struct elem_bytes<float> { static constexpr int v = 4; };
template <> struct elem_bytes<bf16_t> { static constexpr int v = 2; };
template <> struct elem_bytes<fp8_t> { static constexpr int v = 1; };

__device__ inline float to_f32(float v) { return v; }
__device__ inline float to_f32(bf16_t v) { return bf2f(v); }
template <typename T> __device__ inline T from_f32(float v);
template <> __device__ inline float from_f32<float>(float v) { return v; }
template <> __device__ inline bf16_t from_f32<bf16_t>(float v) { return f2bf(v); }

}  // namespace kvop
