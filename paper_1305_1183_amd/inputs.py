"""Seeded synthetic inputs shared by the tests, the benchmark and the examples.

This module only draws numbers: it holds none of the fused-BLAS arithmetic.
The paper states no problem sizes or value distributions for its Table 2-5
experiments, so every operand is synthetic and counter-based:

* the stream for (seed, tensor_id) starts from the state
  ``key = (seed * 0x9E3779B97F4A7C15 + tensor_id * 0xD1B54A32D192ED03) mod 2**64``;
* element ``i`` is ``h_i = mix64(key + (i + 1) * 0x9E3779B97F4A7C15)``, i.e. the
  i-th output of Steele, Lea and Flood's SplitMix64 generator seeded with ``key``;
* a uniform[-1, 1) value is ``(h_i >> 40) * 2**-23 - 1``: 24 random bits, so it
  is exactly representable in float32 and independent of how it is computed.

Matrix element (i, j) of a rows x cols matrix uses counter ``i * cols + j``
regardless of the leading dimension, so padding never changes the values.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_K2 = 0xD1B54A32D192ED03
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1
_CHUNK = 1 << 17


def stream_key(seed: int, tensor_id: int) -> int:
    return (int(seed) * GAMMA + int(tensor_id) * _K2) & _MASK


def mix64_int(z: int) -> int:
    """SplitMix64 output mix on a Python int (reference for the array version)."""
    z &= _MASK
    z = ((z ^ (z >> 30)) * _M1) & _MASK
    z = ((z ^ (z >> 27)) * _M2) & _MASK
    return z ^ (z >> 31)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * np.uint64(_M1)
        z = z ^ (z >> np.uint64(27))
        z = z * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return z


def raw_bits(seed: int, tensor_id: int, start: int, count: int) -> np.ndarray:
    """Hashes h_start .. h_{start+count-1} of stream (seed, tensor_id) as uint64."""
    key = np.uint64(stream_key(seed, tensor_id))
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(key + idx * np.uint64(GAMMA))


def _threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _fill_pm1(out: np.ndarray, seed: int, tensor_id: int, start: int) -> None:
    # (h >> 40) - 2**23 is an integer in [-2**23, 2**23), exact in float32;
    # scaling by 2**-23 is exact too, so the value equals (h >> 40) 2**-23 - 1.
    bits = raw_bits(seed, tensor_id, start, out.size) >> np.uint64(40)
    k = bits.astype(np.int64) - (1 << 23)
    np.multiply(k.astype(np.float32), np.float32(2.0 ** -23), out=out)


def uniform_pm1(seed: int, tensor_id: int, count: int, start: int = 0) -> np.ndarray:
    """float32 values uniform on [-1, 1) with 24 random bits each."""
    out = np.empty(count, dtype=np.float32)
    offs = list(range(0, count, _CHUNK))
    if len(offs) <= 1:
        if count:
            _fill_pm1(out, seed, tensor_id, start)
        return out
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda o: _fill_pm1(out[o:o + _CHUNK], seed, tensor_id, start + o), offs))
    return out


def scalar_uniform(seed: int, tensor_id: int, lo: float = 0.5, hi: float = 2.0) -> float:
    """One value uniform on [lo, hi), drawn in float64 and rounded to float32."""
    u = float(raw_bits(seed, tensor_id, 0, 1)[0] >> np.uint64(40)) * 2.0 ** -24
    return float(np.float32(lo + (hi - lo) * u))


def vector(seed: int, tensor_id: int, n: int) -> np.ndarray:
    return uniform_pm1(seed, tensor_id, n)


def matrix(seed: int, tensor_id: int, rows: int, cols: int, ld: int | None = None,
           pad_value: float = np.nan) -> np.ndarray:
    """rows x ld float32 array; columns >= cols hold ``pad_value``.

    NaN padding is the default so that any kernel that lets a padding element
    into a result is caught by the comparison.
    """
    ld = cols if ld is None else int(ld)
    if ld < cols:
        raise ValueError("ld < cols")
    a = np.empty((rows, ld), dtype=np.float32)
    if ld > cols:
        a[:, cols:] = pad_value
    if ld == cols:
        a.reshape(-1)[:] = uniform_pm1(seed, tensor_id, rows * cols)
        return a
    rows_per_chunk = max(1, _CHUNK // max(cols, 1))

    def fill(r0):
        r1 = min(rows, r0 + rows_per_chunk)
        tmp = np.empty((r1 - r0) * cols, dtype=np.float32)
        _fill_pm1(tmp, seed, tensor_id, r0 * cols)
        a[r0:r1, :cols] = tmp.reshape(r1 - r0, cols)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fill, range(0, rows, rows_per_chunk)))
    return a


def small_ints(seed: int, tensor_id: int, count: int, lo: int, hi: int) -> np.ndarray:
    """float32 integers uniform on [lo, hi] (for exactly-representable pins)."""
    bits = raw_bits(seed, tensor_id, 0, count) >> np.uint64(32)
    span = hi - lo + 1
    return (lo + (bits % np.uint64(span)).astype(np.int64)).astype(np.float32)


def padded_ld(cols: int, multiple: int = 4) -> int:
    return ((cols + multiple - 1) // multiple) * multiple


def loguniform_int(seed: int, tensor_id: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Integers floor(exp(U(ln lo, ln(hi + 1)))) clipped to [lo, hi]."""
    bits = raw_bits(seed, tensor_id, 0, count) >> np.uint64(11)
    u = bits.astype(np.float64) * 2.0 ** -53
    v = np.floor(np.exp(np.log(lo) + u * (np.log(hi + 1) - np.log(lo)))).astype(np.int64)
    return np.clip(v, lo, hi)


def _normal_from_bits(h1: np.ndarray, h2: np.ndarray) -> np.ndarray:
    # Box-Muller: u1 in (0, 1], u2 in [0, 1) from 53 random bits each
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def normal_at(seed: int, tensor_id: int, idx: np.ndarray) -> np.ndarray:
    """float64 N(0, 1) values of element indices idx (element k uses hashes 2k, 2k + 1)."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = np.uint64(stream_key(seed, tensor_id))
    with np.errstate(over="ignore"):
        h1 = _mix64(key + (np.uint64(2) * idx + np.uint64(1)) * np.uint64(GAMMA))
        h2 = _mix64(key + (np.uint64(2) * idx + np.uint64(2)) * np.uint64(GAMMA))
    return _normal_from_bits(h1, h2)


def normal(seed: int, tensor_id: int, count: int, start: int = 0) -> np.ndarray:
    """float64 N(0, 1) values of elements start .. start + count - 1."""
    out = np.empty(count, dtype=np.float64)

    def fill(o):
        c = min(_CHUNK, count - o)
        out[o:o + c] = normal_at(seed, tensor_id, np.arange(start + o, start + o + c, dtype=np.uint64))

    offs = list(range(0, count, _CHUNK))
    if len(offs) <= 1:
        if count:
            fill(0)
        return out
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fill, offs))
    return out
