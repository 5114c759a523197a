"""Host-side tests of the C ABI: exports, validation, legality, enumeration,
byte accounting and code generation (hipRTC compile for gfx950, no GPU)."""
import json
import os
import re

import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "kf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kf_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = kf.lib()
    names = header_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(kf.EXPORTED), set(names) ^ set(kf.EXPORTED)


def test_version():
    assert "gfx950" in kf.kf_version()


def err(fn, *a):
    with pytest.raises(kf.KFError) as e:
        fn(*a)
    return e.value.name


def test_validation_errors():
    s = kf.kf_script_create()
    assert err(kf.kf_vector, s, 0) == "KF_ERR_SHAPE"
    assert err(kf.kf_matrix, s, 4, 5, 6) == "KF_ERR_ALIGN"
    assert err(kf.kf_matrix, s, 4, 9, 8) == "KF_ERR_SHAPE"
    A = kf.kf_matrix(s, 8, 6)
    assert kf.kf_value_info(s, A) == (1, 8, 6, 8)
    x = kf.kf_vector(s, 6)
    y = kf.kf_vector(s, 8)
    one = kf.kf_const(s, 1.0)
    # declared values must be marked input before use
    assert err(kf.kf_gemv, s, one, A, x) == "KF_ERR_STATE"
    kf.kf_input(s, A)
    kf.kf_input(s, x)
    kf.kf_input(s, y)
    assert err(kf.kf_gemv, s, one, A, y) == "KF_ERR_SHAPE"      # x must have cols entries
    assert err(kf.kf_gemtv, s, one, A, x) == "KF_ERR_SHAPE"     # x must have rows entries
    assert err(kf.kf_gemv, s, one, x, x) == "KF_ERR_DTYPE"      # A must be a matrix
    assert err(kf.kf_axpy, s, one, x, y) == "KF_ERR_SHAPE"
    assert err(kf.kf_gemv, s, one, A, x, kf.KF_NONE, y) == "KF_ERR_ARG"  # y0 without beta
    assert err(kf.kf_ger, s, one, A, x, y) == "KF_ERR_SHAPE"    # u has rows, v has cols
    q = kf.kf_gemv(s, one, A, x)
    assert err(kf.kf_input, s, q) == "KF_ERR_STATE"             # SSA: computed, not input
    assert err(kf.kf_output, s, x) == "KF_ERR_STATE"            # declared values are inputs
    assert err(kf.kf_scal, s, x, x) == "KF_ERR_DTYPE"           # alpha must be a scalar
    assert err(kf.kf_compile, kf.kf_script_create()) == "KF_ERR_STATE"  # no calls
    kf.kf_output(s, q)
    # an illegal explicit partition is refused
    q2 = S.gemver(16, 12, 1.5, 0.5)   # keep the Sequence alive: it owns the script
    s2 = q2.script
    with pytest.raises(kf.KFError) as e:   # gemtv result feeding gemv in one kernel
        kf.kf_compile(s2, mode="partition", partition=[0, 1, 2, 2], flags=kf.KF_COMPILE_NO_LOAD)
    assert e.value.name == "KF_ERR_UNSUPPORTED" and "R3" in str(e.value)
    with pytest.raises(kf.KFError) as e:   # {ger1, gemtv} without ger2 between them
        kf.kf_compile(s2, mode="partition", partition=[0, 1, 0, 2], flags=kf.KF_COMPILE_NO_LOAD)
    assert "R1" in str(e.value)
    with pytest.raises(kf.KFError):
        kf.kf_compile(s2, mode="partition", partition=[0], flags=kf.KF_COMPILE_NO_LOAD)
    with pytest.raises(kf.KFError):
        kf.kf_compile(s2, mode="fused", mat_k=3, flags=kf.KF_COMPILE_NO_LOAD)
    with pytest.raises(kf.KFError):
        kf.kf_compile(s2, mode="fused", mat_waves=4, mat_group=4, mat_rows=24, flags=kf.KF_COMPILE_NO_LOAD)
    with pytest.raises(kf.KFError):
        kf.kf_compile(s2, mode="fused", mat_sched=1, mat_group=4, mat_rows=6, flags=kf.KF_COMPILE_NO_LOAD)


def test_run_without_gpu_state_errors():
    q = S.bicgk(64, 48)
    p = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD)
    assert err(kf.kf_run, p, 0) == "KF_ERR_STATE"       # compiled without loading
    assert err(kf.kf_bind_workspace, p, 256, 16) == "KF_ERR_WORKSPACE" or kf.kf_plan_workspace_bytes(p) <= 16
    assert err(kf.kf_bind, p, q.values["A"], 8) == "KF_ERR_ALIGN"
    # outputs must not overlap other operands
    kf.kf_bind(p, q.values["A"], 1 << 20)
    assert err(kf.kf_bind, p, q.values["q"], (1 << 20) + 256) == "KF_ERR_ALIAS"
    kf.kf_bind(p, q.values["q"], 1 << 30)
    kf.kf_plan_destroy(p)


# ---- legality facts of Section 3.2 and Section 5.1 ------------------------------
EXPECTED_PLANS = {
    "bicgk": 2,     # fused (Algorithm 3) or two kernels
    "atax": 2,      # A^T (A x): fused only by the row-resident schedule (R3'')
    "gemver": 4,
    "gesummv": 2,
    "axpydot": 2,
    "waxpby": 2,
}


def build(name, small=True):
    n = 96
    return {"axpydot": lambda: S.axpydot(1000, 1.5), "waxpby": lambda: S.waxpby(1000, 1.5, 0.5),
            "bicgk": lambda: S.bicgk(n, 80), "atax": lambda: S.atax(n, 80),
            "gesummv": lambda: S.gesummv(n, 80, 1.5, 0.5), "gemver": lambda: S.gemver(n, 80, 1.5, 0.5)}[name]()


@pytest.mark.parametrize("name", sorted(EXPECTED_PLANS))
def test_plan_counts(name):
    q = build(name)
    parts = kf.kf_enumerate(q.script)
    assert len(parts) == EXPECTED_PLANS[name]
    # unfused is always legal and listed last (most kernels)
    nc = kf.kf_script_num_calls(q.script)
    assert parts[-1] == list(range(nc))


def test_gemver_partitions_exact():
    q = build("gemver")
    got = sorted(tuple(p) for p in kf.kf_enumerate(q.script))
    # calls: ger1, ger2, gemtv, gemv
    assert got == sorted([(0, 0, 0, 1), (0, 0, 1, 2), (0, 1, 1, 2), (0, 1, 2, 3)])


def test_fused_plans():
    for name, nk in [("bicgk", 1), ("atax", 1), ("gemver", 2), ("gesummv", 1), ("axpydot", 1), ("waxpby", 1)]:
        q = build(name)
        p = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD)
        assert kf.kf_plan_num_kernels(p) == nk, name
        kf.kf_plan_destroy(p)


# ---- byte accounting ----------------------------------------------------------
N2 = 16384


@pytest.mark.parametrize("name,fused,unfused", [
    ("axpydot", 1073741824 + 4, 1342177280 + 4),   # + the 4-byte scalar r
    ("waxpby", 805306368, 1342177280),
    ("bicgk", 1074003968, 2147745792),
    ("atax", 1073872896, 2147745792),   # fused: one pass over A (row-resident)
    ("gesummv", 2147614720, 2147811328),
    ("gemver", 3221815296, 6443040768),
])
def test_algorithmic_bytes_full_size(name, fused, unfused):
    n = N2
    q = {"axpydot": lambda: S.axpydot(1 << 26, 1.5), "waxpby": lambda: S.waxpby(1 << 26, 1.5, 0.5),
         "bicgk": lambda: S.bicgk(n, n), "atax": lambda: S.atax(n, n),
         "gesummv": lambda: S.gesummv(n, n, 1.5, 0.5), "gemver": lambda: S.gemver(n, n, 1.5, 0.5)}[name]()
    for mode, want in (("fused", fused), ("unfused", unfused)):
        p = kf.kf_compile(q.script, mode=mode, flags=kf.KF_COMPILE_NO_LOAD)
        r, w = kf.kf_plan_bytes(p)
        assert r + w == want, (name, mode, r + w, want)
        kf.kf_plan_destroy(p)


def test_bytes_per_flop_match_paper_tables():
    """Table 3 GB/s / Table 2 GFlops equals fused bytes / flops of our plans
    (flops: 2 per multiply-add, GEMVER counted as the paper's 7 n^2)."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables_2_3.json")))["rows"]
    n = N2
    flops = {"AXPYDOT": 4.0 * n * n, "ATAX": 4.0 * n * n, "BiCGK": 4.0 * n * n,
             "GEMVER": 7.0 * n * n, "GESUMMV": 4.0 * n * n, "WAXPBY": 3.0 * n * n}
    seqs = {"AXPYDOT": S.axpydot(n * n, 1.5), "ATAX": S.atax(n, n), "BiCGK": S.bicgk(n, n),
            "GEMVER": S.gemver(n, n, 1.5, 0.5), "GESUMMV": S.gesummv(n, n, 1.5, 0.5),
            "WAXPBY": S.waxpby(n * n, 1.5, 0.5)}
    for key, q in seqs.items():
        # the paper's ATAX plan is two kernels (it cannot fuse it); ours also has
        # a one-pass plan, so the paper's plan is the unfused one here
        mode = "unfused" if key == "ATAX" else "fused"
        p = kf.kf_compile(q.script, mode=mode, flags=kf.KF_COMPILE_NO_LOAD)
        r, w = kf.kf_plan_bytes(p)
        ours = (r + w) / flops[key]
        paper = g[key]["gbps"] / g[key]["gflops"]
        assert abs(ours - paper) / paper < 0.01, (key, ours, paper)
        kf.kf_plan_destroy(p)


# ---- code generation ------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(EXPECTED_PLANS))
def test_every_plan_compiles_for_gfx950(name):
    q = build(name)
    for part in kf.kf_enumerate(q.script):
        p = kf.kf_compile(q.script, mode="partition", partition=part, flags=kf.KF_COMPILE_NO_LOAD)
        d = json.loads(kf.kf_plan_describe(p))
        assert len(d["kernels"]) == max(part) + 1
        for k in range(len(d["kernels"])):
            src = kf.kf_plan_source(p, k)
            assert "extern \"C\" __global__" in src
        kf.kf_plan_destroy(p)


def test_param_grid_compiles():
    q = S.gemver(300, 517, 1.5, 0.5)
    for k_, w, g in [(1, 1, 1), (2, 2, 2), (4, 4, 8), (2, 8, 16), (1, 16, 4)]:
        p = kf.kf_compile(q.script, mode="fused", mat_k=k_, mat_waves=w, mat_group=g,
                          flags=kf.KF_COMPILE_NO_LOAD)
        kf.kf_plan_destroy(p)
    q = S.axpydot(12345, 1.5)
    for u, t, gr in [(1, 64, 1), (8, 1024, 3), (2, 256, 0)]:
        p = kf.kf_compile(q.script, mode="fused", vec_unroll=u, vec_threads=t, vec_grid=gr,
                          flags=kf.KF_COMPILE_NO_LOAD)
        kf.kf_plan_destroy(p)


def test_values_written_only_when_needed():
    """R6: a fused kernel keeps B1 of GEMVER on chip; the unfused plan stores it
    in the workspace because the next kernel reads it."""
    q = S.gemver(64, 64, 1.5, 0.5)
    pf = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD)
    pu = kf.kf_compile(q.script, mode="unfused", flags=kf.KF_COMPILE_NO_LOAD)
    assert kf.kf_plan_workspace_bytes(pu) >= 64 * 64 * 4
    src = kf.kf_plan_source(pf, 0)
    assert src.count("kf_st4_nt(O") == 1     # only B is stored, not B1


def test_ranking_modes_check_their_inputs():
    """Learned mode without a model and exhaustive mode without buffers are
    refused before any GPU work."""
    from paper_1305_1183_amd import sequences as S
    q = S.bicgk(64, 64)
    with pytest.raises(kf.KFError, match="KF_ERR_ARG"):
        kf.kf_compile(q.script, mode="learned")
    with pytest.raises(kf.KFError, match="KF_ERR_UNBOUND"):
        kf.kf_compile(q.script, mode="exhaustive")


def test_stream_reference_checks_its_arguments():
    """Rejected on the host before any device work (runs without a GPU)."""
    a, b = 1 << 20, 1 << 30                           # 16-byte aligned stand-in addresses
    for args in [(2, a, b, 65536), (1, a, b, 65536 + 16), (0, a, b, 12), (0, a + 4, b, 64), (1, 0, b, 65536)]:
        with pytest.raises(kf.KFError) as e:
            kf.kf_util_stream(*args)
        assert e.value.name == "KF_ERR_ARG", args
    with pytest.raises(kf.KFError) as e:
        kf.kf_util_stream(1, a, a + 65536, 2 * 65536)  # overlapping copy
    assert e.value.name == "KF_ERR_ALIAS"


def test_noalloc_entry_checks_before_any_gpu_call():
    """kf_run_noalloc: the array size in kf.h and the binding agree; a null plan,
    a plan too large for the array and a plan compiled without loading are
    refused on the host."""
    text = open(os.path.join(ROOT, "include", "kf.h")).read()
    m = re.search(r"#define KF_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == kf.KF_NOALLOC_SCRATCH_BYTES
    assert kf.lib().kf_run_noalloc(None, None) == kf.KF_ERR_ARG
    big = S.gemver(3072, 3072, 1.5, 0.75)              # unfused: B1 (36 MiB) lives in the workspace
    p = kf.kf_compile(big.script, mode="unfused", flags=kf.KF_COMPILE_NO_LOAD)
    try:
        assert kf.kf_plan_workspace_bytes(p) > kf.KF_NOALLOC_SCRATCH_BYTES
        assert kf.lib().kf_run_noalloc(p, None) == kf.KF_ERR_WORKSPACE
        assert "workspace" in kf.kf_last_error()
    finally:
        kf.kf_plan_destroy(p)
    small = S.bicgk(1000, 1000)
    p = kf.kf_compile(small.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD)
    try:
        assert kf.lib().kf_run_noalloc(p, None) == kf.KF_ERR_STATE
    finally:
        kf.kf_plan_destroy(p)


def test_script_handle_outlives_its_sequence():
    """The Python handle owns the script: compiling from the handle of a
    temporary sequence object (collected before the call runs) is safe, and a
    destroyed handle reaches the library as a null script (KF_ERR_ARG)."""
    p = kf.kf_compile(S.bicgk(64, 96).script, mode="fused", flags=kf.KF_COMPILE_CODEGEN_ONLY)
    assert kf.kf_plan_num_kernels(p) == 1
    kf.kf_plan_destroy(p)
    s = S.bicgk(64, 96).script
    kf.kf_script_destroy(s)
    assert err(kf.kf_compile, s) == "KF_ERR_ARG"
    kf.kf_script_destroy(s)                      # a second destroy does nothing
