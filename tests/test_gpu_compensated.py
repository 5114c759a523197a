"""Compensated final reductions on the GPU.

Every final reduction that adds partial sums of different workgroups (or of
different waves, where that merge is the last step of a dot) uses TwoSum
compensation. Each case here places partials +2^24, a random partial x and
-2^24 so that plain FP32 addition in the kernel's fixed order rounds x to an
even integer (2^24 + x has a spacing of 2) and misses the tolerance
1e-5 log2 n against the FP64 oracle, while the compensated sum keeps x. Every
case first shows, on the host, that plain FP32 addition of the block partials
in the kernel's order fails the bound, so the case can tell the two apart.

The layouts follow the kernels' documented decompositions: row blocks of
mat_rows rows, column strips of 256 k columns, row-resident waves of 256 kp
columns, BLAS-1 workgroups of threads x unroll float4 chunks, batched row
blocks of opts.rows rows and batched wave rows (row r in wave r mod 4 for
whole-row tiles of 64 lanes)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import quant as OQ
from paper_1305_1183_amd import batched as B
from paper_1305_1183_amd import inputs as I
from paper_1305_1183_amd import kf
from paper_1305_1183_amd import quant as Q
from paper_1305_1183_amd import sequences as S
from paper_1305_1183_amd import workloads as WL
from tests import seqcheck as SC

pytestmark = pytest.mark.gpu

BIG = float(2 ** 24)


def setup_module():
    assert torch.cuda.is_available()
    kf.lib()


def plain_f32(parts):
    """Plain FP32 sum of the partials (arrays) in the given order."""
    acc = np.asarray(parts[0], np.float32).copy()
    for p in parts[1:]:
        acc = (acc + np.asarray(p, np.float32)).astype(np.float32)
    return acc.astype(np.float64)


def assert_teeth(plain, ref, tol):
    e = WL.rel_l2(plain, ref)
    assert e > 10 * tol, ("case cannot separate plain from compensated sums", e, tol)


def rows_cancel_matrix(m, n, big_rows, rand_rows, seed):
    """A (m x ld, zero padding), r: rows big_rows[0] = +2^24 and big_rows[1]
    = -2^24 with r = 1 there; rand_rows random with random r; the rest zero."""
    ld = I.padded_ld(n)
    A = np.zeros((m, ld), np.float32)
    r = np.zeros(m, np.float32)
    A[big_rows[0], :n] = BIG
    A[big_rows[1], :n] = -BIG
    r[list(big_rows)] = 1.0
    rr = np.asarray(rand_rows)
    A[rr, :n] = I.matrix(seed, 0, len(rr), n, ld=n)
    r[rr] = I.vector(seed, 1, len(rr))
    return A, r


def cols_cancel_matrix(m, n, big_cols, rand_cols, seed):
    """A, p: column big_cols[0] = +2^24, big_cols[1] = -2^24 with p = 1
    there; rand_cols random with random p; the rest zero."""
    ld = I.padded_ld(n)
    A = np.zeros((m, ld), np.float32)
    p = np.zeros(n, np.float32)
    A[:, big_cols[0]] = BIG
    A[:, big_cols[1]] = -BIG
    p[list(big_cols)] = 1.0
    cc = np.asarray(rand_cols)
    A[:, cc] = I.matrix(seed, 2, m, len(cc), ld=len(cc))
    p[cc] = I.vector(seed, 3, len(cc))
    return A, p


@pytest.mark.parametrize("sched", [0, 1])
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_gemtv_row_block_partials_cancel(sched, mode):
    """s = A^T r over three row blocks of 64 rows: block 0 holds +2^24 r_0,
    block 1 random rows, block 2 -2^24 r_128 (strip and row-resident schedules)."""
    R, m, n = 64, 192, 300
    print("case gemtv blocks sched", sched, mode, flush=True)
    A, r = rows_cancel_matrix(m, n, (0, 2 * R), range(R, 2 * R), seed=41)
    p = I.vector(41, 4, n)
    ref = SC.oracle_outputs("bicgk", {"A": A, "p": p, "r": r}, {}, n)
    tol = WL.tolerance("bicgk", m, n)
    parts = [A[b * R:(b + 1) * R, :n].astype(np.float64).T @ r[b * R:(b + 1) * R] for b in range(3)]
    assert_teeth(plain_f32(parts), ref["s"], tol)
    params = dict(mat_rows=R, mat_sched=sched)
    if sched == 0:
        params.update(mat_waves=4, mat_group=4)
    _, prog, h = SC.run_gpu("bicgk", m, n, {"A": A, "p": p, "r": r}, {}, mode=mode, **params)
    # the gemtv partials of the three row blocks go through a finishing launch
    assert max(kf.kf_plan_num_launches(prog.plan, k) for k in range(prog.num_kernels)) == 2
    SC.check_against_oracle("bicgk", m, n, h, ref)


def test_gemv_strip_partials_cancel():
    """q = A p over three column strips of 256 columns (mat_k = 1): strip 0
    holds +2^24 p_0, strip 1 random columns, strip 2 -2^24 p_512."""
    m, n = 200, 768
    print("case gemv strips", flush=True)
    A, p = cols_cancel_matrix(m, n, (0, 512), range(256, 512), seed=42)
    r = I.vector(42, 5, m)
    ref = SC.oracle_outputs("bicgk", {"A": A, "p": p, "r": r}, {}, n)
    tol = WL.tolerance("bicgk", m, n)
    parts = [A[:, s * 256:(s + 1) * 256].astype(np.float64) @ p[s * 256:(s + 1) * 256] for s in range(3)]
    assert_teeth(plain_f32(parts), ref["q"], tol)
    for mode in ("fused", "unfused"):
        _, _, h = SC.run_gpu("bicgk", m, n, {"A": A, "p": p, "r": r}, {}, mode=mode,
                             mat_k=1, mat_waves=4, mat_group=4, mat_rows=64)
        SC.check_against_oracle("bicgk", m, n, h, ref)


def test_rowres_gemv_wave_partials_cancel():
    """Row-resident q = A p with four waves of 256 columns each: the wave
    partials +2^24, x, -2^24, 0 are merged in wave order inside the workgroup."""
    m, n = 100, 1024
    print("case rowres waves", flush=True)
    A, p = cols_cancel_matrix(m, n, (0, 512), range(256, 512), seed=43)
    r = I.vector(43, 5, m)
    ref = SC.oracle_outputs("bicgk", {"A": A, "p": p, "r": r}, {}, n)
    tol = WL.tolerance("bicgk", m, n)
    parts = [A[:, w * 256:(w + 1) * 256].astype(np.float64) @ p[w * 256:(w + 1) * 256] for w in range(4)]
    assert_teeth(plain_f32(parts), ref["q"], tol)
    _, _, h = SC.run_gpu("bicgk", m, n, {"A": A, "p": p, "r": r}, {}, mode="fused",
                         mat_sched=1, mat_waves=4, mat_group=1)
    SC.check_against_oracle("bicgk", m, n, h, ref)


def test_strip_wave_merge_cancel():
    """One row block of four rows and four waves of one row each (the strip
    kernel's in-workgroup merge of wave column partials is the final sum):
    rows +2^24, random, -2^24, random."""
    m, n = 4, 520
    print("case strip wave merge", flush=True)
    A, r = rows_cancel_matrix(m, n, (0, 2), [1, 3], seed=44)
    p = I.vector(44, 4, n)
    ref = SC.oracle_outputs("bicgk", {"A": A, "p": p, "r": r}, {}, n)
    tol = WL.tolerance("bicgk", m, n)
    parts = [A[i, :n].astype(np.float64) * r[i] for i in range(4)]
    assert_teeth(plain_f32(parts), ref["s"], tol)
    _, _, h = SC.run_gpu("bicgk", m, n, {"A": A, "p": p, "r": r}, {}, mode="fused",
                         mat_k=1, mat_waves=4, mat_group=1, mat_rows=4)
    SC.check_against_oracle("bicgk", m, n, h, ref)


def test_blas1_dot_workgroup_partials_cancel():
    """AXPYDOT r = z^T u with three workgroups of 64 threads x one float4
    (256 entries each): partials +2^24, -2^24, x. The finishing launch's lanes
    0, 1, 2 hold them and its butterfly first adds lanes 0 and 2, so plain
    FP32 computes (2^24 + x) - 2^24."""
    n = 768
    print("case blas1 dot", flush=True)
    w = np.zeros(n, np.float32)
    u = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    w[0], u[0] = BIG, 1.0
    w[256], u[256] = -BIG, 1.0
    w[512:] = I.vector(45, 0, 256)
    u[512:] = I.vector(45, 1, 256)
    arrays, scal = {"w": w, "v": v, "u": u}, {"alpha": 1.5}
    ref = SC.oracle_outputs("axpydot", arrays, scal, n)
    tol = WL.tolerance("axpydot", n, n)
    P = [np.array([np.dot(w[b * 256:(b + 1) * 256].astype(np.float64), u[b * 256:(b + 1) * 256])]) for b in range(3)]
    assert_teeth(plain_f32([plain_f32([P[0], P[2]]), P[1]]), ref["r"], tol)
    _, _, h = SC.run_gpu("axpydot", n, n, arrays, scal, mode="fused", vec_unroll=1, vec_threads=64, vec_grid=3)
    SC.check_against_oracle("axpydot", n, n, h, ref)


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_quantised_gemtv_row_block_partials_cancel(fmt):
    """Reduced-precision A: the column partials of A^T r over three row
    blocks cancel as in the FP32 case (BF16 stores 2^24 exactly; FP8 rows
    +d and -d with the same row scale cancel exactly)."""
    R, m, n = 64, 192, 300
    print("case quantised gemtv", fmt, flush=True)
    A, r = rows_cancel_matrix(m, n, (0, 2 * R), range(R, 2 * R), seed=46)
    st, sc = Q.quantize_rows(A[:, :n].astype(np.float64), fmt)
    D = OQ.dequantize(st, sc, fmt, n)
    p = I.vector(46, 4, n)
    s_ref = oracle.gemtv(1.0, D, r.astype(np.float64))
    tol = WL.tolerance("bicgk", m, n)
    parts = [D[b * R:(b + 1) * R].T @ r[b * R:(b + 1) * R].astype(np.float64) for b in range(3)]
    assert_teeth(plain_f32(parts), s_ref, tol)
    q = S.bicgk_q(m, n, fmt)
    prog = q.compile(mode="fused", mat_rows=R, mat_waves=4, mat_group=4)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a.view(np.int16) if a.dtype == np.uint16 else a)).cuda()
    prog.bind(A=dev(st), A_scale=dev(sc), p=dev(p), r=dev(r))
    outs = prog.run()
    torch.cuda.synchronize()
    assert WL.rel_l2(outs["s"].cpu().numpy(), s_ref) <= tol


def test_batched_partials_cancel():
    """Batched launch: a BiCGK and a GEMVER instance of n = 1500 cut into
    three row blocks of 500 rows (the last block adds the column partials in
    block order), and a BiCGK instance of n = 200 whose four waves hold rows
    0, 1, 2, 3 mod 4 (the whole-row tiles merge the wave partials in wave
    order)."""
    kinds = np.array([B.BICGK, B.GEMVER, B.BICGK], np.int32)
    ns = np.array([1500, 1500, 200])
    rows = {B.BICGK: [0, 0, 0, 0, 0, 500], B.GEMVER: [0, 0, 0, 0, 0, 500]}
    bt = B.Batch(kinds, ns, np.array([1.0, 1.25, 1.0], np.float32), np.array([1.0, 0.75, 1.0], np.float32),
                 kf.batch_opts(rows=rows))
    host = np.full(bt.elems, np.nan, np.float32)
    refs, plains = [], []

    def put(i, name, arr):
        o, _ = bt.offset(i, name)
        host[o:o + arr.size] = arr.ravel()

    for i, (kind, n) in enumerate(zip(kinds, ns)):
        n = int(n)
        off, ld = bt.offset(i, "A")
        if n == 1500:
            A, rr = rows_cancel_matrix(n, n, (0, 1000), range(500, 1000), seed=47 + i)
            blocks = [(0, 500), (500, 1000), (1000, 1500)]
        else:
            A, rr = rows_cancel_matrix(n, n, (0, 2), range(1, n, 4), seed=47 + i)
            blocks = [(w, None) for w in range(4)]
        Ap = np.full((n, ld), np.nan, np.float32)
        Ap[:, :n] = A[:, :n]
        put(i, "A", Ap)
        if kind == B.BICGK:
            p = I.vector(50 + i, 0, n)
            put(i, "p", p)
            put(i, "r", rr)
            q, s = oracle.bicgk(Ap, p, rr, cols=n)
            refs.append((i, "s", s, WL.tolerance("bicgk", n, n)))
            refs.append((i, "q", q, WL.tolerance("bicgk", n, n)))
            target, weights = s, rr
        else:
            z = I.vector(50 + i, 1, n)
            yv = rr
            vals = {"u1": np.zeros(n, np.float32), "v1": I.vector(50 + i, 2, n), "u2": np.zeros(n, np.float32),
                    "v2": I.vector(50 + i, 3, n), "y": yv, "z": z}
            for k2, v2 in vals.items():
                put(i, k2, v2)
            Bm, x, w = oracle.gemver(1.25, 0.75, Ap, vals["u1"], vals["v1"], vals["u2"], vals["v2"], yv, z, cols=n)
            refs.append((i, "x", x, WL.tolerance("gemver", n, n)))
            target, weights = (x - z.astype(np.float64)) / 0.75, yv
        D = A[:, :n].astype(np.float64)
        if blocks[0][1] is not None:
            parts = [D[a:b].T @ weights[a:b] for a, b in blocks]
        else:
            parts = [D[w::4].T @ weights[w::4] for w, _ in blocks]
        plains.append((plain_f32(parts), target, refs[-1][3] if kind == B.GEMVER else refs[-2][3]))
    for plain, target, tol in plains:
        assert_teeth(plain, target, tol)
    bt.upload(host)
    bt.run(0)
    torch.cuda.synchronize()
    assert bt.error() == 0
    out = bt.arena.cpu().numpy()
    for i, name, ref, tol in refs:
        got = bt.outputs(out, i)[name]
        e = WL.rel_l2(got, ref)
        assert e <= tol, (i, name, e, tol)


@pytest.mark.parametrize("params", [dict(mat_k=1, mat_waves=4, mat_group=2, mat_rows=64),
                                    dict(mat_sched=1, mat_waves=4, mat_group=2, mat_rows=16)])
def test_infinite_terms_give_infinity_not_nan(params):
    """A sum with an infinite term is that infinity, as plain addition gives:
    the compensation of an infinite partial (inf - inf) must not turn it into
    NaN. BiCGK with one +inf entry of A and positive p, r: the row dot of that
    row and the column sum of that column are +inf, every other result finite
    and within tolerance of the oracle."""
    m, n = 300, 700
    ld = I.padded_ld(n)
    A = (np.abs(I.uniform_pm1(5, 0, m * ld)).reshape(m, ld) + 0.5).astype(np.float32)
    A[:, n:] = 0.0
    A[123, 456] = np.inf
    p = (np.abs(I.uniform_pm1(5, 1, n)) + 0.5).astype(np.float32)
    r = (np.abs(I.uniform_pm1(5, 2, m)) + 0.5).astype(np.float32)
    q_seq = S.bicgk(m, n, ld=ld)
    prog = q_seq.compile(mode="fused", **params)
    prog.bind(A=torch.from_numpy(A).cuda(), p=torch.from_numpy(p).cuda(), r=torch.from_numpy(r).cuda())
    outs = prog.run()
    torch.cuda.synchronize()
    q, s = outs["q"].cpu().numpy(), outs["s"].cpu().numpy()
    assert np.isposinf(q[123]) and np.isposinf(s[456])
    fq, fs = np.delete(np.arange(m), 123), np.delete(np.arange(n), 456)
    assert np.all(np.isfinite(q[fq])) and np.all(np.isfinite(s[fs]))
    Af = A.copy()
    Af[123, 456] = 1.0
    qr, sr = oracle.bicgk(Af, p, r, cols=n)
    tol = WL.tolerance("bicgk", m, n)
    assert WL.rel_l2(q[fq], qr[fq]) <= tol and WL.rel_l2(s[fs], sr[fs]) <= tol


def test_infinite_dot_term_gives_infinity():
    """AXPYDOT's r = z^T u with one infinite u entry is +inf (z > 0 there)."""
    n = (1 << 20) + 3
    w = (np.abs(I.uniform_pm1(6, 0, n)) + 1.0).astype(np.float32)
    v = (np.abs(I.uniform_pm1(6, 1, n)) * 0.25).astype(np.float32)
    u = I.uniform_pm1(6, 2, n).astype(np.float32)
    u[777777] = np.inf
    q_seq = S.axpydot(n, 1.5)
    prog = q_seq.compile(mode="fused")
    prog.bind(w=torch.from_numpy(w).cuda(), v=torch.from_numpy(v).cuda(), u=torch.from_numpy(u).cuda())
    outs = prog.run()
    torch.cuda.synchronize()
    assert np.isposinf(outs["r"].cpu().numpy()[0])
