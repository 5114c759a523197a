"""The library's row quantiser on the GPU (kf_quantize_rows) against brute
force over the oracle's decoders: every stored code is the nearest
representable value of the exact number it stands for (a_ij for BF16, the
exact quotient a_ij / scale_i for FP8-E4M3), ties to the even code, FP8
saturating at +-448; FP8 scales are the correctly rounded amax_i / 448; the
padding codes are zero. Rows with planted exact ties, zero rows, negative
zeros, tiny scales and subnormal inputs are included."""
import numpy as np
import pytest
import torch

from oracle import quant as OQ
from paper_1305_1183_amd import inputs as I
from paper_1305_1183_amd import kf
from paper_1305_1183_amd import quant as Q

pytestmark = pytest.mark.gpu

E4M3_CODES = np.arange(0x7F, dtype=np.uint8)                 # non-negative finite codes 0 .. 0x7e
E4M3_VALS = OQ.decode_e4m3(E4M3_CODES)


def setup_module():
    assert torch.cuda.is_available()
    kf.lib()


def _matrix(rows, cols, seed):
    """FP32 test matrix: random rows at assorted magnitudes, and rows whose
    amax makes the FP8 scale a power of two so that planted E4M3 midpoints
    are exact ties."""
    A = (I.normal(seed, 0, rows * cols).reshape(rows, cols) *
         np.exp2(I.uniform_pm1(seed, 1, rows).astype(np.float64) * 20)[:, None]).astype(np.float32)
    mids = ((E4M3_VALS[:-1] + E4M3_VALS[1:]) / 2).astype(np.float32)        # 126 exact midpoints
    for r, t in ((0, 0), (1, -3), (2, 5)):
        row = np.resize(np.concatenate([mids, -mids, E4M3_VALS.astype(np.float32)]), cols).astype(np.float32)
        row[0] = 448.0
        A[r] = row * np.float32(2.0 ** t)
    A[3] = 0.0                                                  # all-zero row: scale 1
    A[4] = -0.0
    A[5] = A[5] * np.float32(2.0 ** -100)                      # tiny scale (the scaled tie test)
    A[6, :] = np.float32(2.0 ** -140) * np.arange(cols, dtype=np.float32)   # FP32 subnormals
    # BF16 midpoints (9 significant bits, exact in FP32) in row 7
    base = I.uniform_pm1(seed, 2, cols).astype(np.float32)
    b = base.view(np.uint32) & np.uint32(0xFFFF0000)
    A[7] = (b | np.uint32(0x8000)).view(np.float32)
    return A


def _run(A, dtype, ldq):
    rows, cols = A.shape
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    es = 2 if dtype == kf.KF_BF16 else 1
    codes = torch.full((rows, ldq * es), 0x5A, dtype=torch.uint8, device="cuda")   # padding must be overwritten
    scales = torch.full((rows,), float("nan"), dtype=torch.float32, device="cuda")
    kf.kf_quantize_rows(Ad.data_ptr(), rows, cols, cols, dtype, codes.data_ptr(), ldq, scales.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    c = codes.cpu().numpy()
    return (c.view(np.uint16) if es == 2 else c), scales.cpu().numpy()


def _nearest_e4m3(x, s):
    """Brute force over every finite E4M3 magnitude: the code whose value
    times s is nearest to |x| (float64 differences, exact for the nearest
    candidates), ties to the even code; the sign bit from x."""
    ax = np.abs(x.astype(np.float64))
    d = np.abs(E4M3_VALS[None, :] * np.float64(s) - ax[:, None])
    best = d.min(axis=1)
    out = np.empty(len(x), np.uint8)
    for i in range(len(x)):
        cand = np.flatnonzero(d[i] == best[i])
        if len(cand) > 1:
            cand = [c for c in cand if c % 2 == 0] or cand
        out[i] = cand[0]
    return out | (np.signbit(x).astype(np.uint8) << np.uint8(7))


def test_fp8_codes_and_scales_match_brute_force():
    rows, cols = 12, 1000
    A = _matrix(rows, cols, 5)
    ldq = 1008                                     # 16-byte rows, ragged tail of padding
    codes, scales = _run(A, kf.KF_FP8_E4M3, ldq)
    amax = np.max(np.abs(A), axis=1)
    want_s = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    assert np.array_equal(scales.view(np.uint32), want_s.view(np.uint32))
    assert scales[0] == 1.0 and scales[1] == 2.0 ** -3 and scales[2] == 32.0 and scales[3] == 1.0
    assert np.all(codes[:, cols:] == 0)
    for r in range(rows):
        want = _nearest_e4m3(A[r], scales[r])
        bad = np.flatnonzero(codes[r, :cols] != want)
        assert len(bad) == 0, (r, bad[:5], A[r, bad[:5]], codes[r, bad[:5]], want[bad[:5]])
    # the planted midpoints are exact ties: half of them round up (to an even code)
    assert np.array_equal(OQ.decode_e4m3(codes[0, :cols]) * scales[0], OQ.decode_e4m3(_nearest_e4m3(A[0], 1.0)))
    # the host quantiser (float64 quotient) agrees on every finite row
    for r in range(rows):
        if scales[r] > 0:
            host = Q.to_e4m3_codes(A[r].astype(np.float64) / np.float64(scales[r]))
            assert np.array_equal(host, codes[r, :cols]), r


def test_fp8_saturation_and_nan():
    A = np.array([[448.0, -448.0, 1.0, np.nan]], np.float32)
    codes, scales = _run(A, kf.KF_FP8_E4M3, 16)
    assert scales[0] == 1.0
    assert list(codes[0, :4]) == [0x7E, 0xFE, 0x38, 0x7F]


def test_bf16_codes_match_brute_force():
    rows, cols = 12, 777
    A = _matrix(rows, cols, 9)
    ldq = 784
    codes, scales = _run(A, kf.KF_BF16, ldq)
    assert np.all(scales == 1.0) and np.all(codes[:, cols:] == 0)
    allc = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    vals = OQ.decode_bf16(allc)
    fin = np.isfinite(vals)
    tv, tc = vals[fin], allc[fin]
    order = np.argsort(tv, kind="stable")
    tv, tc = tv[order], tc[order]
    x = A.reshape(-1).astype(np.float64)
    got = codes[:, :cols].reshape(-1)
    # brute force on a sample of every row plus every planted tie (row 7)
    pick = np.unique(np.concatenate([np.arange(0, x.size, 37), np.arange(7 * cols, 8 * cols)]))
    for i in pick:
        d = np.abs(tv - x[i])
        cand = tc[d == d.min()]
        if len(cand) > 1:                                     # +0 / -0, or an exact tie
            if x[i] == 0:
                cand = [np.uint16(0x8000 if np.signbit(x[i]) else 0)]
            else:
                cand = [c for c in cand if c % 2 == 0] or list(cand)
        assert got[i] == cand[0], (i, x[i], hex(got[i]), hex(cand[0]))
    # every element agrees with the host quantiser (the same exact rounding from binary32)
    assert np.array_equal(Q.to_bf16_codes(x), got)


def test_quantize_rows_rejects_bad_arguments():
    L = kf.lib()
    t = torch.zeros(64, dtype=torch.float32, device="cuda")
    c = torch.zeros(256, dtype=torch.uint8, device="cuda")
    p = t.data_ptr()
    assert L.kf_quantize_rows(p, 2, 8, 8, 7, c.data_ptr(), 16, p + 128, None) == kf.KF_ERR_ARG
    assert L.kf_quantize_rows(p, 2, 8, 8, kf.KF_FP8_E4M3, c.data_ptr(), 12, p + 128, None) == kf.KF_ERR_ALIGN
    assert L.kf_quantize_rows(p, 2, 8, 8, kf.KF_FP8_E4M3, p + 16, 16, p + 200, None) == kf.KF_ERR_ALIAS
    assert L.kf_quantize_rows(p, 2, 8, 4, kf.KF_BF16, c.data_ptr(), 8, p + 128, None) == kf.KF_ERR_ARG
