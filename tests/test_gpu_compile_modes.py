"""kf_compile's learned and exhaustive modes through the C ABI: the chosen
plans compute the right results, exhaustive search picks a plan no slower
than the other candidates it timed, and a cost model survives a save/load
round trip bit for bit."""
import os

import numpy as np
import pytest
import torch

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import workloads as WL
from paper_1305_1183_amd.costmodel import CostModel
from tests import seqcheck as SC

pytestmark = pytest.mark.gpu
MODEL = os.path.join(os.path.dirname(kf.__file__), "data", "plan_cost_model.npz")


def bound(name, m, n):
    arrays, scal = WL.make(name, m, n, seed=WL.seed_for(8, name))
    q = SC.build_sequence(name, m, n, scal)
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in arrays.items()}
    outs = {}
    for o in q.outputs:
        shape = q.shapes[o]
        outs[o] = torch.empty(shape, dtype=torch.float32, device="cuda")
    bind = {q.values[k]: t.data_ptr() for k, t in list(dev.items()) + list(outs.items())}
    return q, arrays, scal, dev, outs, bind


def run_plan(q, plan, dev):
    from paper_1305_1183_amd.sequences import Program
    prog = Program(q, plan)
    prog.bind(**dev)
    outs = prog.run()
    torch.cuda.synchronize()
    return prog, {k: v.cpu().numpy() for k, v in outs.items()}


@pytest.mark.parametrize("name", ["gemver", "bicgk"])
def test_exhaustive_mode(name):
    m = n = 2048
    q, arrays, scal, dev, outs, bind = bound(name, m, n)
    st = torch.cuda.current_stream().cuda_stream
    plan = kf.kf_compile(q.script, mode="exhaustive", bind=bind, stream=st)
    prog, host = run_plan(q, plan, dev)
    SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))
    t_best = prog.time(3, 20)
    # no slower (beyond timing noise) than the all-fused and unfused plans
    for mode in ("fused", "unfused"):
        other = q.compile(mode=mode).bind(**dev)
        assert t_best <= other.time(3, 20) * 1.10, (mode, t_best)


@pytest.mark.parametrize("top_k", [0, 3])
def test_learned_mode(top_k):
    name, m, n = "gemver", 2048, 2048
    q, arrays, scal, dev, outs, bind = bound(name, m, n)
    cm = CostModel.load(MODEL)
    cm.set_launch_us(0.41)
    st = torch.cuda.current_stream().cuda_stream
    plan = kf.kf_compile(q.script, mode="learned", model=cm.handle, stream=st, top_k=top_k,
                         bind=bind if top_k else None)
    prog, host = run_plan(q, plan, dev)
    SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))


def test_learned_top_k_needs_buffers():
    q, *_ = bound("bicgk", 256, 256)
    cm = CostModel.load(MODEL)
    with pytest.raises(kf.KFError):
        kf.kf_compile(q.script, mode="learned", model=cm.handle, stream=torch.cuda.current_stream().cuda_stream,
                      top_k=3)
    with pytest.raises(kf.KFError):
        kf.kf_compile(q.script, mode="learned")


def test_costmodel_save_load_roundtrip(tmp_path):
    cm = CostModel.load(MODEL)
    X = np.random.default_rng(0).standard_normal((500, kf.FEATURE_DIM)).astype(np.float32)
    a = cm.predict_log(X)
    p = str(tmp_path / "m.kfcm")
    cm.set_launch_us(0.5)
    cm.save(p)
    cm2 = CostModel.load(p)
    assert np.array_equal(a, cm2.predict_log(X))
    assert cm2.state()[4] == np.float32(0.5)
    for x, y in zip(cm.state()[:3], cm2.state()[:3]):
        assert np.array_equal(x, y)


def test_shipped_library_format_model_predicts_like_npz():
    a = CostModel.load(MODEL)
    b = CostModel.load(MODEL.replace(".npz", ".kfcm"))
    X = np.random.default_rng(1).standard_normal((300, kf.FEATURE_DIM)).astype(np.float32)
    assert np.array_equal(a.predict_log(X), b.predict_log(X))


@pytest.mark.parametrize("name", ["gemver", "atax"])
def test_per_kernel_parameters_parity(name):
    """A plan whose kernels use different parameter points computes the same
    results; per-kernel times add up to about the plan time."""
    m = n = 3000   # ragged against every strip width and row block
    q, arrays, scal, dev, outs, bind = bound(name, m, n)
    kp = [dict(mat_k=2, mat_waves=4, mat_group=2, mat_rows=2048), dict(mat_k=1, mat_waves=4, mat_group=2, mat_rows=1024)]
    plan = kf.kf_compile(q.script, mode="unfused" if name == "atax" else "fused", kernel_params=kp)
    assert [kf.kf_plan_kernel_params(plan, k) for k in range(2)] == kp
    prog, host = run_plan(q, plan, dev)
    SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))
    ks = prog.time_kernels(2, 10)
    assert len(ks) == 2 and all(t > 0 for t in ks)
    whole = prog.time(2, 10)
    assert 0.5 * whole < sum(ks) < 1.5 * whole + 20.0


def test_time_budget_stops_timing_early():
    """With a 1 ms budget the exhaustive mode times one candidate (plus the ones
    already under way) and still returns a correct plan, sooner than without."""
    import time
    name, m, n = "gemver", 2048, 2048
    q, arrays, scal, dev, outs, bind = bound(name, m, n)
    st = torch.cuda.current_stream().cuda_stream
    kf.kf_compile(q.script, mode="exhaustive", bind=bind, stream=st)   # compile caches warm for both runs
    t0 = time.perf_counter()
    full = kf.kf_compile(q.script, mode="exhaustive", bind=bind, stream=st)
    t_full = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = kf.kf_compile(q.script, mode="exhaustive", bind=bind, stream=st, time_budget_ms=1)
    t_budget = time.perf_counter() - t0
    kf.kf_plan_destroy(full)
    prog, host = run_plan(q, plan, dev)
    SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))
    assert t_budget < t_full
    with pytest.raises(kf.KFError):
        kf.kf_compile(q.script, mode="exhaustive", bind=bind, stream=st, time_budget_ms=-1)


def test_blas1_unfused_kernels_with_their_own_parameters():
    n = (1 << 20) + 3                                 # ragged against every unroll
    q, arrays, scal, dev, outs, bind = bound("axpydot", n, n)
    kp = [dict(vec_unroll=8, vec_threads=256, vec_grid=64), dict(vec_unroll=1, vec_threads=1024, vec_grid=4096)]
    plan = kf.kf_compile(q.script, mode="unfused", kernel_params=kp)
    got = [kf.kf_plan_kernel_params(plan, k) for k in range(2)]
    assert got[0]["vec_unroll"] == 8 and got[1]["vec_threads"] == 1024
    prog, host = run_plan(q, plan, dev)
    SC.check_against_oracle("axpydot", n, n, host, SC.oracle_outputs("axpydot", arrays, scal, n))


def test_learned_top_k_with_a_time_budget():
    name, m, n = "bicgk", 2048, 2048
    q, arrays, scal, dev, outs, bind = bound(name, m, n)
    cm = CostModel.load(MODEL.replace(".npz", ".kfcm"))
    st = torch.cuda.current_stream().cuda_stream
    plan = kf.kf_compile(q.script, mode="learned", model=cm.handle, stream=st, top_k=5, bind=bind, time_budget_ms=1)
    prog, host = run_plan(q, plan, dev)
    SC.check_against_oracle(name, m, n, host, SC.oracle_outputs(name, arrays, scal, n))
