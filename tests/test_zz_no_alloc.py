"""kf_run_noalloc on the GPU: a plan run on the library's fixed per-device
workspace gives the same bits as kf_run on a caller workspace and meets the
FP64 oracle's tolerance, call after call, with a later call on a smaller
input than an earlier one (the array keeps the earlier call's contents); a
plan whose workspace exceeds the array is refused before any launch; repeated
calls leave the device's free memory unchanged."""
import numpy as np
import pytest
import torch

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S
from paper_1305_1183_amd import workloads as WL
from tests import seqcheck as SC

pytestmark = pytest.mark.gpu
SCAL = {"alpha": 1.5, "beta": 0.75}


def setup_module():
    assert torch.cuda.is_available()
    kf.lib()


def _prepare(name, n, mode="fused"):
    """Fused plan of `name` at n x n (BLAS-1: n entries), bound to seeded inputs
    and outputs, with its reference outputs from kf_run on a caller workspace."""
    m = n
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(41, name) + n)
    q = S.by_name(name, m, n, scal)
    prog = q.compile(mode=mode)
    prog.bind(**{k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in arrays.items()})
    ref = {k: v.clone() for k, v in prog.run().items()}
    torch.cuda.synchronize()
    return q, prog, arrays, scal, {k: v.cpu().numpy() for k, v in ref.items()}


def _fresh_outputs(q, prog):
    """Rebind every output to a NaN-filled tensor; return them."""
    outs = {}
    for name in q.outputs:
        t = torch.full(tuple(prog.tensors[name].shape), float("nan"), device="cuda")
        kf.kf_bind(prog.plan, q.values[name], t.data_ptr())
        outs[name] = t
    return outs


def _noalloc_matches(name, n, q, prog, arrays, scal, ref):
    outs = _fresh_outputs(q, prog)
    print("kf_run_noalloc", name, n, flush=True)
    kf.kf_run_noalloc(prog.plan, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in outs.items()}
    for k in ref:
        assert np.array_equal(got[k], ref[k], equal_nan=False), (name, n, k, "differs from kf_run")
    m = n
    SC.check_against_oracle(name, m, n, got, SC.oracle_outputs(name, arrays, scal, n))


def test_noalloc_equals_kf_run_then_smaller_input():
    # the largest first: its partials fill more of the array than the later calls
    cases = [("atax", 3000), ("bicgk", 700), ("gemver", 1500), ("axpydot", (1 << 20) + 3),
             ("gesummv", 257), ("bicgk", 33)]
    prepared = [(name, n) + _prepare(name, n) for name, n in cases]
    need = [kf.kf_plan_workspace_bytes(p[3].plan) for p in prepared]
    assert need[0] > need[1] > 0, need            # the second call's input is smaller
    for name, n, q, prog, arrays, scal, ref in prepared:
        _noalloc_matches(name, n, q, prog, arrays, scal, ref)
    # again in reverse order: small partials first, then the larger ones over them
    for name, n, q, prog, arrays, scal, ref in reversed(prepared):
        _noalloc_matches(name, n, q, prog, arrays, scal, ref)


def test_noalloc_allocates_nothing():
    q, prog, arrays, scal, ref = _prepare("bicgk", 2048)
    outs = _fresh_outputs(q, prog)
    st = torch.cuda.current_stream().cuda_stream
    kf.kf_run_noalloc(prog.plan, st)       # first call on this device looks up the array
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        kf.kf_run_noalloc(prog.plan, st)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert np.array_equal(outs["q"].cpu().numpy(), ref["q"]) and np.array_equal(outs["s"].cpu().numpy(), ref["s"])


def test_noalloc_refuses_oversized_workspace():
    # unfused GEMVER keeps B1 = A + u1 v1^T (n x n FP32) in the workspace
    n = 3072
    q = S.gemver(n, n, 1.5, 0.75)
    plan = kf.kf_compile(q.script, mode="unfused")
    try:
        need = kf.kf_plan_workspace_bytes(plan)
        assert need > kf.KF_NOALLOC_SCRATCH_BYTES
        with pytest.raises(kf.KFError) as ei:
            kf.kf_run_noalloc(plan, torch.cuda.current_stream().cuda_stream)
        assert ei.value.status == kf.KF_ERR_WORKSPACE
        assert "workspace" in str(ei.value)
    finally:
        kf.kf_plan_destroy(plan)
