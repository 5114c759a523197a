"""Row-resident kernels on rows of 32760 and 32768 columns (eight float4 per
lane per row) against the FP64 oracle. At that width the library's own
geometry would not fit the registers, so the generator halves the rows per
group, stages column vectors in LDS and reads the rest from global memory at
each use; every case checks that the remedy it is meant to cover is present in
the generated source, then compares with the oracle (fused and unfused
plans, ragged and exact widths, row- and column-major storage)."""
import json

import numpy as np
import pytest
import torch

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import workloads as WL
from tests import seqcheck as SC
from tests.test_gpu_layout import run_colmajor

pytestmark = pytest.mark.gpu


def setup_module():
    assert torch.cuda.is_available()
    kf.lib()


def _row_kernels(prog):
    """(params, main-launch source) of each row-resident kernel of a plan."""
    d = json.loads(kf.kf_plan_describe(prog.plan))
    return [(kk["params"], kf.kf_plan_source(prog.plan, k).split("_fin")[0])
            for k, kk in enumerate(d["kernels"]) if kk["name"].startswith("kf_row")]


def _markers(prog):
    out = set()
    for params, src in _row_kernels(prog):
        if params["group"] == 1:
            out.add("g1")
        if "cbg" in src:
            out.add("global")
        if "__shared__ kf_f4 xs" in src:
            out.add("lds")
    return out


# (sequence, m, n, layout, params, remedies expected in the fused plan)
CASES = [
    ("atax", 67, 32760, "row", {}, {"g1", "lds"}),
    ("atax", 64, 32768, "row", {}, {"g1", "lds"}),
    ("bicgk", 67, 32760, "row", dict(mat_sched=1), {"g1", "lds"}),
    ("gesummv", 67, 32760, "row", dict(mat_sched=1), {"g1"}),
    ("gemver", 67, 32760, "row", dict(mat_sched=1), {"g1", "lds", "global"}),
    ("gemver", 32760, 67, "col", {}, {"g1", "lds", "global"}),
    ("gemver", 32768, 64, "col", {}, {"g1", "lds", "global"}),
    ("sgemvt", 32760, 67, "col", {}, {"g1", "lds"}),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%dx%d-%s" % c[:4])
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_wide_rows_against_oracle(case, mode):
    name, m, n, layout, params, want = case
    print("case", name, m, n, layout, params, mode, flush=True)
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(41, name))
    if layout == "row":
        q, prog, host = SC.run_gpu(name, m, n, arrays, scal, mode=mode, **params)
    else:
        prog, host = run_colmajor(name, m, n, arrays, scal, mode, **params)
    if mode == "fused":
        assert want <= _markers(prog), (_markers(prog), want)
    SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))


def test_requested_geometry_is_kept():
    """Parameters the caller gives are generated as asked: the remedies only
    adjust the geometry the library picks itself."""
    name, m, n = "atax", 67, 32760
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(42, name))
    q, prog, host = SC.run_gpu(name, m, n, arrays, scal, mode="fused", mat_sched=1, mat_waves=16, mat_group=2)
    (params, src), = _row_kernels(prog)
    assert params["group"] == 2 and "cbg" not in src
    SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))


@pytest.mark.parametrize("name", ["gemver", "atax"])
def test_wide_rows_with_padded_leading_dimension(name):
    """Rows of 32760 columns stored 32776 floats apart, the padding NaN (a
    read of it would reach the results): the adjusted geometry's loads and
    column-vector reads stay within each row's columns."""
    m, n, ld = 67, 32760, 32776
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(43, name), ld=ld)
    params = dict(mat_sched=1) if name == "gemver" else {}
    q, prog, host = SC.run_gpu(name, m, n, arrays, scal, mode="fused", ld=ld, **params)
    assert "g1" in _markers(prog)
    if name == "gemver":
        assert "global" in _markers(prog)
    SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))
