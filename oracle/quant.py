"""Decoding of the reduced-precision storage formats (test infrastructure).

Written from the format definitions, independently of the library:
* BF16: the 16 high bits of an IEEE-754 binary32 value.
* OCP FP8-E4M3: bit 7 sign, bits 6..3 exponent (bias 7), bits 2..0 fraction;
  exponent field 0 encodes subnormals f * 2**-9; the all-ones pattern
  S.1111.111 is NaN; there are no infinities (largest finite 1.75 * 2**8 = 448).
"""
from __future__ import annotations

import numpy as np


def decode_bf16(codes) -> np.ndarray:
    c = np.asarray(codes, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return c.view(np.float32).astype(np.float64)


def decode_e4m3(codes) -> np.ndarray:
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    sign = np.where((c >> 7) & 1, -1.0, 1.0)
    e = (c >> 3) & 15
    f = c & 7
    mag = np.where(e == 0, f * 2.0 ** -9, (1.0 + f / 8.0) * np.exp2(e - 7.0))
    out = sign * mag
    return np.where((e == 15) & (f == 7), np.nan, out)


def dequantize(storage, scales, fmt: str, cols: int) -> np.ndarray:
    """float64 matrix scale[i] * decode(code_ij)."""
    if fmt == "f32":
        v = np.asarray(storage[:, :cols], dtype=np.float64)
    elif fmt == "bf16":
        v = decode_bf16(storage[:, :cols])
    elif fmt == "fp8":
        v = decode_e4m3(storage[:, :cols])
    else:
        raise ValueError(fmt)
    return v * np.asarray(scales, dtype=np.float64)[:, None]
