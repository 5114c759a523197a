"""GPU parity of column-major matrices (Section 3.3: a matrix viewed as a list
of columns) against the FP64 oracle. The oracle works on the declared m x n
matrix; the library gets its column-major storage (element (i, j) at
j * ld + i). Fused and unfused plans, ragged shapes, every BLAS-2 sequence,
including the one-kernel column-major GEMVER and SGEMVT."""
import numpy as np
import pytest
import torch

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S
from paper_1305_1183_amd import workloads as WL
from tests import seqcheck as SC

pytestmark = pytest.mark.gpu

SHAPES = [(1000, 1001), (257, 2050), (4099, 300), (64, 64), (3, 5), (1, 1)]


def setup_module():
    assert torch.cuda.is_available()
    kf.lib()


def to_colmajor(a, m, n):
    """Column-major storage of the m x n matrix held in the first n columns of a."""
    ld = (m + 3) // 4 * 4
    st = np.zeros((n, ld), dtype=np.float32)
    st[:, :m] = a[:m, :n].T
    return st


def run_colmajor(name, m, n, arrays, scal, mode, **params):
    q = S.by_name(name, m, n, scal, layout=kf.KF_COL_MAJOR)
    prog = q.compile(mode=mode, **params)
    dev = {}
    for k, v in arrays.items():
        h = to_colmajor(v, m, n) if v.ndim == 2 else v
        dev[k] = torch.from_numpy(np.ascontiguousarray(h)).cuda()
    prog.bind(**dev)
    outs = prog.run()
    torch.cuda.synchronize()
    host = {}
    for k, v in outs.items():
        h = v.cpu().numpy()
        host[k] = np.ascontiguousarray(h[:, :m].T) if h.ndim == 2 else h
    return prog, host


@pytest.mark.parametrize("name", ["bicgk", "atax", "gesummv", "gemver", "sgemvt"])
@pytest.mark.parametrize("mn", SHAPES)
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_colmajor_sequences(name, mn, mode):
    m, n = mn
    print("case colmajor", name, m, n, mode, flush=True)
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(23, name))
    prog, host = run_colmajor(name, m, n, arrays, scal, mode)
    ref = SC.oracle_outputs(name, arrays, scal, n)
    SC.check_against_oracle(name, m, n, host, ref)


@pytest.mark.parametrize("params", [
    dict(mat_sched=1, mat_waves=4, mat_group=1),
    dict(mat_sched=1, mat_waves=16, mat_group=4, mat_rows=64),
])
def test_colmajor_gemver_one_kernel(params):
    """Column-major GEMVER runs as one row-resident kernel (x complete per row
    before its gemtv update) and matches the oracle."""
    m, n = 1500, 777
    print("case colmajor gemver one kernel", params, flush=True)
    arrays, scal = WL.make("gemver", m, n, seed=29)
    prog, host = run_colmajor("gemver", m, n, arrays, scal, "fused", **params)
    assert prog.num_kernels == 1
    ref = SC.oracle_outputs("gemver", arrays, scal, n)
    SC.check_against_oracle("gemver", m, n, host, ref)


def test_colmajor_equals_row_major_transpose_bitwise():
    """BiCGK on a column-major A and on the row-major A^T (p and r swapped)
    run the same kernels on the same memory: outputs equal bit for bit."""
    m, n = 900, 1300
    print("case colmajor bitwise", m, n, flush=True)
    arrays, scal = WL.make("bicgk", m, n, seed=31)
    prog, host = run_colmajor("bicgk", m, n, arrays, scal, "fused")
    # row-major A^T is n x m; its q = A^T p' and s = A r' with p' = r, r' = p
    qt = S.bicgk(n, m)
    st = to_colmajor(arrays["A"], m, n)
    pt = qt.compile(mode="fused").bind(A=torch.from_numpy(st).cuda(),
                                       p=torch.from_numpy(arrays["r"]).cuda(),
                                       r=torch.from_numpy(arrays["p"]).cuda())
    out = pt.run()
    torch.cuda.synchronize()
    assert np.array_equal(host["q"], out["s"].cpu().numpy())
    assert np.array_equal(host["s"], out["q"].cpu().numpy())


@pytest.mark.parametrize("name", WL.LAYOUT_SEQ)
def test_colmajor_measured_points(name):
    """The parameter points the layout measurement uses, on a ragged shape."""
    m, n = 2001, 1503
    print("case colmajor measured point", name, m, n, flush=True)
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(37, name))
    prog, host = run_colmajor(name, m, n, arrays, scal, "fused", **WL.LAYOUT_TUNED[name])
    ref = SC.oracle_outputs(name, arrays, scal, n)
    SC.check_against_oracle(name, m, n, host, ref)
