"""Row-scaled reduced-precision matrix storage (BF16, OCP FP8-E4M3).

A float64 matrix is stored as codes plus one FP32 scale per row: element
(i, j) stands for scale[i] * decode(code_ij). Rounding is to nearest, ties to
even, directly from float64. BF16 rows keep scale 1 (BF16 has the FP32
exponent range); FP8 rows use scale = amax_i / 448 (448 is the largest finite
E4M3 value) and saturate at +-448.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def _round_to(x: np.ndarray, mbits: int, emin: int) -> np.ndarray:
    """x rounded to the nearest value with `mbits` fraction bits (ties to even),
    exponents below `emin` falling on the subnormal grid 2**(emin - mbits)."""
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)                     # x = m 2**e, 0.5 <= |m| < 1
    e = np.maximum(e - 1, emin)            # floor(log2 |x|), clamped to the subnormal range
    q = np.ldexp(1.0, (e - mbits).astype(np.int64))
    return np.rint(x / q) * q


def _rne_bits(b: np.ndarray, drop: int) -> np.ndarray:
    """Round the float64 bit patterns b (non-negative values) to nearest, ties
    to even, keeping 52 - drop fraction bits; a carry moves into the exponent."""
    one = np.uint64(1)
    half = (one << np.uint64(drop - 1)) - one
    lsb = (b >> np.uint64(drop)) & one
    return ((b + half + lsb) >> np.uint64(drop)) << np.uint64(drop)


def to_bf16_codes(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    r = _rne_bits(a.view(np.uint64), 45).view(np.float64)      # 7 fraction bits
    tiny = a < 2.0 ** -126                                     # BF16 subnormal range
    if np.any(tiny):
        r = np.where(tiny, np.rint(a / 2.0 ** -133) * 2.0 ** -133, r)
    r32 = np.copysign(r, x).astype(np.float32)                 # exact: <= 8 significant bits
    return (r32.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def to_e4m3_codes(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    b = _rne_bits(a.view(np.uint64), 49)                       # 3 fraction bits (normal range)
    sub = a < 2.0 ** -6                                        # subnormals: multiples of 2**-9
    m_sub = np.rint(a * 2.0 ** 9)                              # 0..8 (8 = smallest normal)
    e = (b >> np.uint64(52)).astype(np.int64) - 1023
    m = ((b >> np.uint64(49)) & np.uint64(7)).astype(np.int64)
    code = ((e + 7) << 3) | m
    code = np.where(sub, m_sub.astype(np.int64), code)         # m_sub = 8 encodes 0x08 = 2**-6
    code = np.minimum(code, 0x7E)                               # saturate at 448 (0x7E)
    code = np.where(np.isnan(x), 0x7F, code)
    return (code.astype(np.uint8) | (np.signbit(x).astype(np.uint8) << np.uint8(7))).astype(np.uint8)


def quantize_rows(A: np.ndarray, fmt: str, ld: int | None = None):
    """(storage rows x ld, scales float32 rows) of a float64 matrix."""
    A = np.asarray(A, dtype=np.float64)
    rows, cols = A.shape
    if fmt == "f32":
        ld = ld or (cols + 3) // 4 * 4
        out = np.zeros((rows, ld), np.float32)
        out[:, :cols] = A.astype(np.float32)
        return out, np.ones(rows, np.float32)
    if fmt == "bf16":
        ld = ld or (cols + 7) // 8 * 8
        out = np.zeros((rows, ld), np.uint16)
        out[:, :cols] = to_bf16_codes(A)
        return out, np.ones(rows, np.float32)
    if fmt == "fp8":
        ld = ld or (cols + 15) // 16 * 16
        amax = np.max(np.abs(A), axis=1)
        scale = np.where(amax > 0, amax / E4M3_MAX, 1.0).astype(np.float32)
        out = np.zeros((rows, ld), np.uint8)
        out[:, :cols] = to_e4m3_codes(A / scale.astype(np.float64)[:, None])
        return out, scale
    raise ValueError(fmt)
