"""GPU parity: every fused and unfused plan of the Table 1 sequences against
the FP64 oracle (relative L2 error <= 1e-5 log2 n), exact special cases that
must match bit for bit, fused == unfused bit for bit at equal parameters, and
run-to-run determinism."""
import numpy as np
import pytest
import torch

from paper_1305_1183_amd import inputs as I
from paper_1305_1183_amd import kf
from paper_1305_1183_amd import workloads as WL
from tests import seqcheck as SC

pytestmark = pytest.mark.gpu

SMALL = [  # (m, n): several tiles and ragged tails in both dimensions
    (1000, 1001), (257, 2050), (64, 64), (3, 5), (1, 1), (4099, 300),
]
VEC_N = [1, 3, 4, 1000, 65539, 1 << 20]


def setup_module():
    assert torch.cuda.is_available()
    kf.lib()


@pytest.mark.parametrize("name", ["bicgk", "atax", "gesummv", "gemver", "sgemvt"])
@pytest.mark.parametrize("mn", SMALL)
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_blas2_sequences(name, mn, mode):
    m, n = mn
    print("case", name, m, n, mode, flush=True)
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(7, name))
    q, prog, host = SC.run_gpu(name, m, n, arrays, scal, mode=mode)
    ref = SC.oracle_outputs(name, arrays, scal, n)
    SC.check_against_oracle(name, m, n, host, ref)


@pytest.mark.parametrize("name", ["axpydot", "waxpby", "vadd"])
@pytest.mark.parametrize("n", VEC_N)
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_blas1_sequences(name, n, mode):
    print("case", name, n, mode, flush=True)
    arrays, scal = WL.make(name, n, n, seed=WL.seed_for(7, name))
    q, prog, host = SC.run_gpu(name, n, n, arrays, scal, mode=mode)
    ref = SC.oracle_outputs(name, arrays, scal, n)
    SC.check_against_oracle(name, n, n, host, ref)


@pytest.mark.parametrize("params", [
    dict(mat_k=1, mat_waves=1, mat_group=1, mat_rows=1),
    dict(mat_k=2, mat_waves=2, mat_group=8, mat_rows=16),
    dict(mat_k=4, mat_waves=8, mat_group=16, mat_rows=128),
    dict(mat_k=2, mat_waves=4, mat_group=4, mat_rows=512),
])
def test_blas2_param_grid(params):
    m, n = 777, 1555
    for name in ("bicgk", "gemver", "gesummv"):
        print("case", name, params, flush=True)
        arrays, scal = WL.make(name, m, n, seed=11)
        q, prog, host = SC.run_gpu(name, m, n, arrays, scal, mode="fused", **params)
        SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))


@pytest.mark.parametrize("params", [dict(vec_unroll=1, vec_threads=64, vec_grid=1),
                                    dict(vec_unroll=8, vec_threads=1024, vec_grid=7),
                                    dict(vec_unroll=2, vec_threads=128, vec_grid=4096)])
def test_blas1_param_grid(params):
    n = 300007
    for name in ("axpydot", "waxpby"):
        print("case", name, params, flush=True)
        arrays, scal = WL.make(name, n, n, seed=12)
        q, prog, host = SC.run_gpu(name, n, n, arrays, scal, mode="fused", **params)
        SC.check_against_oracle(name, n, n, host, SC.oracle_outputs(name, arrays, scal, n))


def test_fused_equals_unfused_bitwise():
    """Same tile parameters give the same per-element operation order, so
    fusion changes no bit of any output (it only removes HBM traffic)."""
    m, n = 1500, 2300
    for name in ("bicgk", "gemver", "gesummv", "axpydot", "waxpby"):
        arrays, scal = WL.make(name, m, n, seed=13)
        _, _, hf = SC.run_gpu(name, m, n, arrays, scal, mode="fused")
        _, _, hu = SC.run_gpu(name, m, n, arrays, scal, mode="unfused")
        for k in hf:
            assert np.array_equal(hf[k], hu[k], equal_nan=True), (name, k)


def test_rerun_bitwise_deterministic():
    m, n = 2048, 3000
    for name in ("bicgk", "gemver", "axpydot"):
        arrays, scal = WL.make(name, m, n, seed=14)
        q, prog, h0 = SC.run_gpu(name, m, n, arrays, scal, mode="fused")
        for _ in range(5):
            outs = prog.run()
            torch.cuda.synchronize()
            for k, v in outs.items():
                assert np.array_equal(v.cpu().numpy(), h0[k], equal_nan=True), (name, k)


# ---- exact special cases (bit for bit) --------------------------------------------
def test_bicgk_identity_and_integer_exact():
    n = 1030
    A = np.zeros((n, I.padded_ld(n)), np.float32)
    A[:, :n] = np.eye(n, dtype=np.float32)
    p = I.vector(1, 0, n)
    r = I.vector(1, 1, n)
    _, _, h = SC.run_gpu("bicgk", n, n, {"A": A, "p": p, "r": r}, {})
    assert np.array_equal(h["q"], p) and np.array_equal(h["s"], r)
    # small integers: every partial sum is an exact integer < 2**24 in FP32
    m, n = 700, 900
    Ai = np.zeros((m, I.padded_ld(n)), np.float32)
    Ai[:, :n] = I.small_ints(2, 0, m * n, -3, 3).reshape(m, n)
    pi = I.small_ints(2, 1, n, -3, 3)
    ri = I.small_ints(2, 2, m, -3, 3)
    _, _, h = SC.run_gpu("bicgk", m, n, {"A": Ai, "p": pi, "r": ri}, {})
    ref = SC.oracle_outputs("bicgk", {"A": Ai, "p": pi, "r": ri}, {}, n)
    assert np.array_equal(h["q"].astype(np.float64), ref["q"])
    assert np.array_equal(h["s"].astype(np.float64), ref["s"])


def test_gemver_exact_chain():
    """A = 0, small-integer vectors and power-of-two scalars make every stage
    of GEMVER exact, so the GPU must equal the oracle exactly."""
    m, n = 513, 1027
    arrays = {"A": np.zeros((m, I.padded_ld(n)), np.float32)}
    for tid, k in enumerate(["u1", "v1", "u2", "v2", "y", "z"]):
        ln = m if k in ("u1", "u2", "y") else n
        arrays[k] = I.small_ints(3, tid, ln, -2, 2)
    arrays["A"][:, n:] = np.nan
    scal = {"alpha": 0.5, "beta": 2.0}
    _, _, h = SC.run_gpu("gemver", m, n, arrays, scal)
    ref = SC.oracle_outputs("gemver", arrays, scal, n)
    assert np.array_equal(h["B"][:, :n].astype(np.float64), ref["B"])
    assert np.array_equal(h["x"].astype(np.float64), ref["x"])
    assert np.array_equal(h["w"].astype(np.float64), ref["w"])


def test_axpydot_exact_zero_and_integers():
    n = 100003
    v = I.vector(4, 0, n)
    u = I.vector(4, 1, n)
    _, _, h = SC.run_gpu("axpydot", n, n, {"w": 2 * v, "v": v, "u": u}, {"alpha": 2.0})
    assert np.all(h["z"] == 0) and h["r"][0] == 0
    w = I.small_ints(4, 2, n, -4, 4)
    vi = I.small_ints(4, 3, n, -4, 4)
    ui = I.small_ints(4, 4, n, -4, 4)
    _, _, h = SC.run_gpu("axpydot", n, n, {"w": w, "v": vi, "u": ui}, {"alpha": 1.0})
    ref = SC.oracle_outputs("axpydot", {"w": w, "v": vi, "u": ui}, {"alpha": 1.0}, n)
    assert h["r"][0] == ref["r"][0]


def test_padding_never_read_or_written():
    """NaN in the padding columns of A must not reach any result, and the
    padding of the output matrix B must be left untouched."""
    m, n = 300, 1001
    arrays, scal = WL.make("gemver", m, n, seed=15, ld=1012)
    q = SC.build_sequence("gemver", m, n, scal, ld=1012)
    prog = q.compile(mode="fused")
    dev = {k: torch.from_numpy(v).cuda() for k, v in arrays.items()}
    ldb = kf.kf_value_info(q.script, q.values["B"])[3]
    B = torch.full((m, ldb), 7.0, device="cuda")
    prog.bind(B=B, **dev)
    prog.run()
    torch.cuda.synchronize()
    Bh = B.cpu().numpy()
    assert np.all(Bh[:, n:] == 7.0)
    assert np.all(np.isfinite(Bh[:, :n]))
    ref = SC.oracle_outputs("gemver", arrays, scal, n)
    SC.check_against_oracle("gemver", m, n, {"B": Bh, "x": prog.tensors["x"].cpu().numpy(),
                                             "w": prog.tensors["w"].cpu().numpy()}, ref)


def test_set_const_without_recompile():
    m, n = 256, 512
    arrays, scal = WL.make("gesummv", m, n, seed=16)
    q, prog, h = SC.run_gpu("gesummv", m, n, arrays, scal)
    prog.set_const("alpha", 2 * scal["alpha"])
    outs = prog.run()
    torch.cuda.synchronize()
    ref = SC.oracle_outputs("gesummv", arrays, dict(scal, alpha=2 * scal["alpha"]), n)
    SC.check_against_oracle("gesummv", m, n, {"y": outs["y"].cpu().numpy()}, ref)


def test_enumerated_plans_agree():
    """Every legal partition of GEMVER computes the same result."""
    m, n = 400, 700
    arrays, scal = WL.make("gemver", m, n, seed=17)
    ref = SC.oracle_outputs("gemver", arrays, scal, n)
    q = SC.build_sequence("gemver", m, n, scal)
    dev = {k: torch.from_numpy(v).cuda() for k, v in arrays.items()}
    for part in kf.kf_enumerate(q.script):
        print("case gemver partition", part, flush=True)
        prog = q.compile(mode="partition", partition=part)
        prog.bind(**dev)
        outs = prog.run()
        torch.cuda.synchronize()
        SC.check_against_oracle("gemver", m, n, {k: v.cpu().numpy() for k, v in outs.items()}, ref)


@pytest.mark.parametrize("params", [dict(mat_sched=1), dict(mat_sched=1, mat_waves=4, mat_group=2, mat_rows=6),
                                    dict(mat_sched=1, mat_waves=16, mat_group=1, mat_rows=64),
                                    dict(mat_sched=1, mat_waves=8, mat_group=4, mat_rows=4)])
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_row_resident_schedule(params, mode):
    """Row-resident kernels (whole rows per workgroup): ATAX in one pass over A,
    and every other sequence under the same schedule."""
    for name, (m, n) in [("atax", (777, 1555)), ("bicgk", (777, 1555)), ("gemver", (513, 1027)),
                         ("gesummv", (300, 2049)), ("atax", (5, 3)), ("atax", (2049, 4097))]:
        print("case", name, m, n, params, mode, flush=True)
        arrays, scal = WL.make(name, m, n, seed=18)
        q, prog, host = SC.run_gpu(name, m, n, arrays, scal, mode=mode, **params)
        SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))


def test_atax_single_pass_reads_a_once():
    """The fused ATAX plan is one kernel that moves A through HBM once."""
    m, n = 2048, 2048
    arrays, scal = WL.make("atax", m, n, seed=19)
    q, prog, host = SC.run_gpu("atax", m, n, arrays, scal, mode="fused")
    assert prog.num_kernels == 1
    r, w = prog.bytes()
    assert r == m * n * 4 + n * 4 and w == n * 4
    SC.check_against_oracle("atax", m, n, host, SC.oracle_outputs("atax", arrays, scal, n))


@pytest.mark.parametrize("name", ["gemver", "bicgk", "atax", "axpydot"])
def test_plan_graph_replays_match_eager(name):
    """kf_run captured into a HIP graph (through torch's graph capture on its
    side stream): every replay, with eager work and synchronisation between
    replays, reproduces the eager result bit for bit."""
    m, n = 1500, 2300
    arrays, scal = WL.make(name, m, n, seed=16)
    q, prog, h0 = SC.run_gpu(name, m, n, arrays, scal, mode="fused")
    outs = {k: prog.tensors[k] for k in q.outputs}
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        prog.run(stream=s.cuda_stream)        # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        kf.kf_run(prog.plan, s.cuda_stream)
    for rep in range(3):
        for v in outs.values():
            v.fill_(float("nan"))             # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            got, ref = v.cpu().numpy(), h0[k]
            if got.ndim == 2:                  # padding columns are never written
                got, ref = got[:, :n], ref[:, :n]
            assert np.array_equal(got, ref), (name, k, rep)
