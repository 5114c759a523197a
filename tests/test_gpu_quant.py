"""Reduced-precision A on the GPU: exhaustive decoding of every FP8-E4M3 and
BF16 code through the library, and BiCGK / GEMVER against the FP64 oracle
evaluated on the dequantised matrix (relative L2 <= 1e-5 log2 n)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import quant as OQ
from paper_1305_1183_amd import inputs as I
from paper_1305_1183_amd import quant as Q
from paper_1305_1183_amd import sequences as S
from paper_1305_1183_amd import workloads as WL

pytestmark = pytest.mark.gpu


def dev(a, fmt=None):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).cuda()


def run(q, arrays, mode="fused", **params):
    prog = q.compile(mode=mode, **params)
    prog.bind(**{k: dev(v) for k, v in arrays.items()})
    outs = prog.run()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in outs.items()}


@pytest.mark.parametrize("fmt,ncodes", [("fp8", 256), ("bf16", 1 << 16)])
def test_exhaustive_decode(fmt, ncodes):
    codes = np.arange(ncodes, dtype=np.uint8 if fmt == "fp8" else np.uint16)
    q = S.decode_probe(ncodes, fmt)
    ld = q.shapes["A"][1]
    st = np.zeros((1, ld), codes.dtype)
    st[0, :ncodes] = codes
    h = run(q, {"A": st, "A_scale": np.ones(1, np.float32), "x": np.ones(1, np.float32)})
    got = h["y"].astype(np.float64)
    want = OQ.decode_e4m3(codes) if fmt == "fp8" else OQ.decode_bf16(codes)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    fin = ~np.isnan(want)
    assert np.array_equal(got[fin], want[fin]), np.where(got[fin] != want[fin])[0][:10]


def quant_oracle_bicgk(D, p, r):
    return oracle.gemv(1.0, D, p.astype(np.float64)), oracle.gemtv(1.0, D, r.astype(np.float64))


def quant_oracle_gemver(D, v, alpha, beta):
    f = lambda a: a.astype(np.float64)
    B = oracle.ger(1.0, oracle.ger(1.0, D, f(v["u1"]), f(v["v1"])), f(v["u2"]), f(v["v2"]))
    x = oracle.gemtv(beta, B, f(v["y"]), 1.0, f(v["z"]))
    return B, x, oracle.gemv(alpha, B, x)


@pytest.mark.parametrize("fmt", ["bf16", "fp8", "f32"])
@pytest.mark.parametrize("mn", [(1000, 1001), (257, 2050), (33, 17)])
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_bicgk_quantised(fmt, mn, mode):
    m, n = mn
    print("case bicgk", fmt, m, n, mode, flush=True)
    A = I.normal(31, 0, m * n).reshape(m, n)
    st, sc = Q.quantize_rows(A, fmt)
    p, r = I.vector(31, 1, n), I.vector(31, 2, m)
    h = run(S.bicgk_q(m, n, fmt), {"A": st, "A_scale": sc, "p": p, "r": r}, mode)
    D = OQ.dequantize(st, sc, fmt, n)
    qr, sr = quant_oracle_bicgk(D, p, r)
    tol = WL.tolerance("bicgk", m, n)
    assert WL.rel_l2(h["q"], qr) <= tol and WL.rel_l2(h["s"], sr) <= tol


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_gemver_quantised(fmt, mode):
    m, n = 700, 1500
    A = I.normal(32, 0, m * n).reshape(m, n)
    st, sc = Q.quantize_rows(A, fmt)
    v = {k: I.vector(32, i + 1, m if k in ("u1", "u2", "y") else n)
         for i, k in enumerate(["u1", "v1", "u2", "v2", "y", "z"])}
    h = run(S.gemver_q(m, n, 1.5, 0.75, fmt), dict(v, A=st, A_scale=sc), mode)
    B, x, w = quant_oracle_gemver(OQ.dequantize(st, sc, fmt, n), v, 1.5, 0.75)
    tol = WL.tolerance("gemver", m, n)
    assert WL.rel_l2(h["B"][:, :n], B) <= tol
    assert WL.rel_l2(h["x"], x) <= tol and WL.rel_l2(h["w"], w) <= tol


def test_quantised_param_grid():
    m, n = 513, 3000
    A = I.normal(33, 0, m * n).reshape(m, n)
    for fmt in ("bf16", "fp8"):
        st, sc = Q.quantize_rows(A, fmt)
        p, r = I.vector(33, 1, n), I.vector(33, 2, m)
        D = OQ.dequantize(st, sc, fmt, n)
        qr, sr = quant_oracle_bicgk(D, p, r)
        for params in (dict(mat_k=1, mat_waves=1, mat_group=1, mat_rows=1), dict(mat_k=2, mat_waves=4, mat_group=8, mat_rows=64)):
            print("case", fmt, params, flush=True)
            h = run(S.bicgk_q(m, n, fmt), {"A": st, "A_scale": sc, "p": p, "r": r}, "fused", **params)
            tol = WL.tolerance("bicgk", m, n)
            assert WL.rel_l2(h["q"], qr) <= tol and WL.rel_l2(h["s"], sr) <= tol


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
@pytest.mark.parametrize("unit", [4, 16])
def test_quantised_load_units(fmt, unit):
    """Both load widths for quantised matrices (four elements per lane, or one
    16-byte load per lane), in BiCGK and in GEMVER's ger kernel, with ragged
    edges in both dimensions."""
    m, n = 259, 1031
    A = I.normal(34, 0, m * n).reshape(m, n)
    st, sc = Q.quantize_rows(A, fmt)
    D = OQ.dequantize(st, sc, fmt, n)
    p, r = I.vector(34, 1, n), I.vector(34, 2, m)
    print("case units", fmt, unit, flush=True)
    h = run(S.bicgk_q(m, n, fmt), {"A": st, "A_scale": sc, "p": p, "r": r}, "fused", mat_unit=unit)
    qr, sr = quant_oracle_bicgk(D, p, r)
    tol = WL.tolerance("bicgk", m, n)
    assert WL.rel_l2(h["q"], qr) <= tol and WL.rel_l2(h["s"], sr) <= tol
    v = {k: I.vector(34, i + 3, m if k in ("u1", "u2", "y") else n)
         for i, k in enumerate(["u1", "v1", "u2", "v2", "y", "z"])}
    h = run(S.gemver_q(m, n, 1.5, 0.75, fmt), dict(v, A=st, A_scale=sc), "fused", mat_unit=unit)
    B, x, w = quant_oracle_gemver(D, v, 1.5, 0.75)
    tol = WL.tolerance("gemver", m, n)
    assert WL.rel_l2(h["B"][:, :n], B) <= tol
    assert WL.rel_l2(h["x"], x) <= tol and WL.rel_l2(h["w"], w) <= tol
