"""Reference number codecs for the reduced-precision forms (test infrastructure only).

* bfloat16: the upper 16 bits of an IEEE binary32, rounded to nearest, ties to even.
* FP8 E4M3 in the OCP "fn" flavour: 1 sign bit, 4 exponent bits (bias 7), 3 mantissa
  bits, no infinities, only S.1111.111 is NaN, largest finite magnitude 448, subnormals
  m/8 * 2^-6.  Encoding rounds to nearest, ties to the even code, and saturates finite
  values beyond 448 to +-448.
* Block quantisation of the KV cache: one FP32 scale per block (amax / 448, or 1 when the
  block is all zero); codes are the E4M3 encoding of x / scale; decoding is code * scale.
  A cache block is 16 consecutive rows of one (layer, kv head, K or V) array.

Written from the format definitions; pinned against library casts in the tests.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (RNE), returned as float32."""
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(x), x, out)


def e4m3_decode_table() -> np.ndarray:
    """Value of every one of the 256 codes (NaN for 0x7F and 0xFF)."""
    vals = np.empty(256, np.float64)
    for c in range(256):
        s = -1.0 if c & 0x80 else 1.0
        e = (c >> 3) & 0xF
        mnt = c & 0x7
        if e == 0xF and mnt == 0x7:
            vals[c] = np.nan
        elif e == 0:
            vals[c] = s * (mnt / 8.0) * 2.0 ** -6
        else:
            vals[c] = s * (1.0 + mnt / 8.0) * 2.0 ** (e - 7)
    return vals


_TABLE = e4m3_decode_table()
_POS_CODES = np.arange(0, 0x7F)            # finite non-negative codes, increasing values
_POS_VALS = _TABLE[_POS_CODES]


def e4m3_decode(codes: np.ndarray) -> np.ndarray:
    return _TABLE[np.asarray(codes, np.uint8)]


def e4m3_encode(x: np.ndarray) -> np.ndarray:
    """Nearest E4M3 code, ties to even (even mantissa LSB), saturating to +-448."""
    x = np.asarray(x, np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    hi = np.searchsorted(_POS_VALS, a, side="left")          # first value >= a
    hi = np.minimum(hi, len(_POS_VALS) - 1)
    lo = np.maximum(hi - 1, 0)
    d_lo = a - _POS_VALS[lo]
    d_hi = _POS_VALS[hi] - a
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & ((_POS_CODES[hi] & 1) == 0))
    code = np.where(pick_hi, _POS_CODES[hi], _POS_CODES[lo]).astype(np.uint8)
    code = np.where(a == _POS_VALS[hi], _POS_CODES[hi], code).astype(np.uint8)
    neg = np.signbit(x)
    code = np.where(neg, code | 0x80, code).astype(np.uint8)
    return np.where(np.isnan(x), np.uint8(0x7F), code).astype(np.uint8)


def block_scale(block: np.ndarray) -> np.float32:
    """FP32 scale of one block: amax / 448, or 1 when the block is all zero."""
    amax = np.float32(np.max(np.abs(np.asarray(block, np.float32)))) if np.size(block) else np.float32(0)
    return np.float32(1.0) if amax == 0 else np.float32(amax / np.float32(E4M3_MAX))


def quantize_block(block: np.ndarray):
    """Encode one block in FP32 arithmetic: x / scale rounded to E4M3.  Returns (codes, scale)."""
    sc = block_scale(block)
    q = (np.asarray(block, np.float32) / sc).astype(np.float32)
    return e4m3_encode(q), sc


CACHE_BLOCK_ROWS = 16


def fp8_cache_roundtrip(a: np.ndarray) -> np.ndarray:
    """What an FP8-E4M3 cache holds for one layer's keys or values a [Hkv, L, D]: each block
    of 16 rows of one head is quantised on its own (quantize_block) and decoded as
    code * scale.  Returned in float64."""
    a = np.asarray(a, np.float64)
    out = np.empty_like(a)
    for h in range(a.shape[0]):
        for r0 in range(0, a.shape[1], CACHE_BLOCK_ROWS):
            codes, sc = quantize_block(a[h, r0:r0 + CACHE_BLOCK_ROWS])
            out[h, r0:r0 + CACHE_BLOCK_ROWS] = e4m3_decode(codes) * np.float64(sc)
    return out
