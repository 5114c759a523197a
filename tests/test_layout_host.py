"""Column-major matrices (Section 3.3: a matrix is a list of rows or a list of
columns, and operations on the transpose are expressed the same way).

A column-major m x n matrix is the row-major n x m matrix A^T in the same
memory, so the recorder stores that form: gemv and gemtv swap, ger swaps u and
v. These host tests check the recorded calls, the shapes the API reports, the
errors, and that plan enumeration, bytes and features are those of the
row-major transpose (no GPU)."""
import json

import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S


def err(fn, *a):
    with pytest.raises(kf.KFError) as e:
        fn(*a)
    return e.value.name


def test_declaration_shape_ld_and_errors():
    s = kf.kf_script_create()
    A = kf.kf_matrix_layout(s, 5, 7, kf.KF_COL_MAJOR)
    assert kf.kf_value_info(s, A) == (1, 5, 7, 8)          # rows, cols as declared; ld = round_up(5, 4)
    assert kf.kf_value_layout(s, A) == kf.KF_COL_MAJOR
    R = kf.kf_matrix_layout(s, 5, 7, kf.KF_ROW_MAJOR)
    assert kf.kf_value_info(s, R) == (1, 5, 7, 8)
    assert kf.kf_value_layout(s, R) == kf.KF_ROW_MAJOR
    assert kf.kf_value_info(s, kf.kf_matrix_layout(s, 5, 7, kf.KF_COL_MAJOR, 12))[3] == 12
    assert err(kf.kf_matrix_layout, s, 5, 7, 2) == "KF_ERR_ARG"
    assert err(kf.kf_matrix_layout, s, 9, 3, kf.KF_COL_MAJOR, 8) == "KF_ERR_SHAPE"   # ld < rows
    assert err(kf.kf_matrix_layout, s, 5, 3, kf.KF_COL_MAJOR, 6) == "KF_ERR_ALIGN"
    assert err(kf.kf_matrix_layout, s, 0, 3, kf.KF_COL_MAJOR) == "KF_ERR_SHAPE"
    v = kf.kf_vector(s, 7)
    assert err(kf.kf_value_layout, s, v) == "KF_ERR_DTYPE"
    kf.kf_script_destroy(s)


def test_calls_recorded_on_the_storage_form():
    m, n = 6, 10
    s = kf.kf_script_create()
    A = kf.kf_matrix_layout(s, m, n, kf.KF_COL_MAJOR)
    u, v, p, r = kf.kf_vector(s, m), kf.kf_vector(s, n), kf.kf_vector(s, n), kf.kf_vector(s, m)
    for x in (A, u, v, p, r):
        kf.kf_input(s, x)
    one = kf.kf_const(s, 1.0)
    q = kf.kf_gemv(s, one, A, p)           # logical A p: length m
    t = kf.kf_gemtv(s, one, A, r)          # logical A^T r: length n
    B = kf.kf_ger(s, one, A, u, v)         # logical m x n
    assert kf.kf_value_info(s, q)[1] == m and kf.kf_value_info(s, t)[1] == n
    assert kf.kf_value_info(s, B)[:3] == (1, m, n)
    assert kf.kf_value_info(s, B)[3] == 8                  # column-major B: ld = round_up(m, 4)
    assert kf.kf_value_layout(s, B) == kf.KF_COL_MAJOR
    calls = [kf.kf_script_call(s, i) for i in range(3)]
    assert [c["op"] for c in calls] == ["gemtv", "gemv", "ger"]
    assert calls[2]["in"] == [A, v, u]                     # u and v swap on the transpose
    # shapes are checked against the declared matrix
    assert err(kf.kf_gemv, s, one, A, r) == "KF_ERR_SHAPE"
    assert err(kf.kf_gemtv, s, one, A, p) == "KF_ERR_SHAPE"
    assert err(kf.kf_ger, s, one, A, v, u) == "KF_ERR_SHAPE"
    # a result of the column-major B keeps flipping
    w = kf.kf_gemv(s, one, B, p)
    assert kf.kf_value_info(s, w)[1] == m
    kf.kf_script_destroy(s)


def storage_twin(q):
    """Replay the recorded (storage-form) calls of sequence q on row-major
    matrices with the storage shapes: the script a caller would write for
    A^T. Returns the twin script."""
    s = q.script
    t = kf.kf_script_create()
    produced = {}
    for i in range(kf.kf_script_num_calls(s)):
        c = kf.kf_script_call(s, i)
        produced[c["out"]] = c
    outputs = {q.values[nm] for nm in q.outputs}
    consts = {v: val for v, val in q.consts.values()}
    h = {}
    for v in range(max(produced) + 1):
        if v in produced:
            c = produced[v]
            a = [h[x] if x >= 0 else kf.KF_NONE for x in c["in"]]
            al = h[c["alpha"]] if c["alpha"] >= 0 else kf.KF_NONE
            be = h[c["beta"]] if c["beta"] >= 0 else kf.KF_NONE
            op = c["op"]
            if op in ("gemv", "gemtv"):
                h[v] = getattr(kf, "kf_" + op)(t, al, a[0], a[1], be, a[2])
            elif op == "ger":
                h[v] = kf.kf_ger(t, al, a[0], a[1], a[2])
            elif op == "scal":
                h[v] = kf.kf_scal(t, al, a[0])
            elif op == "axpy":
                h[v] = kf.kf_axpy(t, al, a[0], a[1])
            else:
                h[v] = kf.kf_dot(t, a[0], a[1])
            if v in outputs:
                kf.kf_output(t, h[v])
            continue
        kind, d0, d1, d2 = kf.kf_value_info(s, v)
        if kind == 0:
            h[v] = kf.kf_vector(t, d0)
        elif kind == 1:
            col = kf.kf_value_layout(s, v) == kf.KF_COL_MAJOR
            h[v] = kf.kf_matrix(t, d1, d0, d2) if col else kf.kf_matrix(t, d0, d1, d2)
        elif kind == 2:
            h[v] = kf.kf_const(t, consts[v])
            continue
        else:
            h[v] = kf.kf_scalar(t)
        kf.kf_input(t, h[v])
    return t


@pytest.mark.parametrize("name,m,n", [("bicgk", 300, 1000), ("atax", 1000, 300),
                                      ("gemver", 257, 2050), ("gesummv", 100, 64),
                                      ("sgemvt", 65, 33), ("gemver", 1, 7)])
def test_same_plans_as_the_storage_form(name, m, n):
    """A column-major m x n sequence has the partitions, bytes and kernel
    code of its storage-form calls recorded on n x m row-major matrices."""
    scal = {"alpha": 1.5, "beta": 0.75}
    qc = S.by_name(name, m, n, scal, layout=kf.KF_COL_MAJOR)
    row = S.by_name(name, m, n, scal)
    twin = storage_twin(qc)
    assert kf.kf_enumerate(qc.script) == kf.kf_enumerate(twin)
    for mode in ("fused", "unfused"):
        pc = kf.kf_compile(qc.script, mode=mode, flags=kf.KF_COMPILE_CODEGEN_ONLY)
        pt = kf.kf_compile(twin, mode=mode, flags=kf.KF_COMPILE_CODEGEN_ONLY)
        assert kf.kf_plan_bytes(pc) == kf.kf_plan_bytes(pt)
        assert kf.kf_plan_num_kernels(pc) == kf.kf_plan_num_kernels(pt)
        for k in range(kf.kf_plan_num_kernels(pc)):
            assert kf.kf_plan_source(pc, k) == kf.kf_plan_source(pt, k)
    # every matrix call is the other form of the row-major sequence's call
    flip = {"gemv": "gemtv", "gemtv": "gemv", "ger": "ger"}
    for i in range(kf.kf_script_num_calls(qc.script)):
        assert kf.kf_script_call(qc.script, i)["op"] == flip[kf.kf_script_call(row.script, i)["op"]]


def test_layout_decides_fusibility():
    """On column-major storage the roles of gemv and gemtv swap, so the
    dependence that blocks fusion moves: ATAX (t = A x, y = A^T t) needs two
    kernels, while GEMVER and SGEMVT, whose gemtv result feeds a gemv on
    row-major storage, become one row-resident kernel each; GEMVER's B is then
    written once and not read back."""
    scal = {"alpha": 1.5, "beta": 0.75}
    m = n = 1024
    counts = {}
    for name in ("atax", "gemver", "sgemvt", "bicgk", "gesummv"):
        for lay in (kf.KF_ROW_MAJOR, kf.KF_COL_MAJOR):
            q = S.by_name(name, m, n, scal, layout=lay)
            p = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_CODEGEN_ONLY)
            counts[name, lay] = (kf.kf_plan_num_kernels(p), kf.kf_plan_bytes(p))
    R, C = kf.KF_ROW_MAJOR, kf.KF_COL_MAJOR
    assert counts["atax", R][0] == 1 and counts["atax", C][0] == 2
    assert counts["gemver", R][0] == 2 and counts["gemver", C][0] == 1
    assert counts["sgemvt", R][0] == 2 and counts["sgemvt", C][0] == 1
    assert counts["bicgk", C][0] == 1 and counts["gesummv", C][0] == 1
    # GEMVER: A read once and B written once (plus vectors) against 12 n^2 bytes
    rd, wr = counts["gemver", C][1]
    assert rd + wr < 8 * n * n + 64 * n
    rd, wr = counts["gemver", R][1]
    assert rd + wr >= 12 * n * n


def test_bind_shapes_of_column_major_sequences():
    q = S.gemver(10, 6, 1.0, 1.0, layout=kf.KF_COL_MAJOR)
    assert q.shapes["A"] == (6, 12)      # storage: cols x ld, ld = round_up(10, 4)
    assert q.shapes["B"] == (6, 12)
    assert q.shapes["x"] == (6,) and q.shapes["w"] == (10,)
