"""Runtime-shape plans on the GPU: one plan declared at its largest shape runs
smaller shapes (kf_plan_set_shape, kf_bind_matrix) and matches the FP64
oracle; it gives the same bits as a plan compiled for that exact shape with
the same parameters; kf_plan_run_many over many instances; and the batched
configuration's per-instance plan loop, instance by instance."""
import numpy as np
import pytest
import torch

import oracle
from paper_1305_1183_amd import batched as B
from paper_1305_1183_amd import inputs as I
from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S
from paper_1305_1183_amd import workloads as WL
from tests import seqcheck as SC

pytestmark = pytest.mark.gpu
RS = kf.KF_COMPILE_RUNTIME_SHAPE
PARAMS = dict(mat_k=1, mat_waves=4, mat_group=2, mat_rows=64)


def setup_module():
    assert torch.cuda.is_available()
    kf.lib()


def _run_at(q, plan, m, n, arrays, ld):
    """Bind arrays (matrices with leading dimension ld) at shape m x n, run.
    Output vectors declared with the matrix's rows get m entries, the others n."""
    decl_rows = next(kf.kf_value_info(q.script, q.values[k])[1] for k in q.inputs
                     if kf.kf_value_info(q.script, q.values[k])[0] == 1)
    kf.kf_plan_set_shape(plan, m, n)
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in arrays.items()}
    for k, t in dev.items():
        v = q.values[k]
        if kf.kf_value_info(q.script, v)[0] == 1:
            kf.kf_bind_matrix(plan, v, t.data_ptr(), ld)
        else:
            kf.kf_bind(plan, v, t.data_ptr())
    outs = {}
    for name in q.outputs:
        kind, d0, d1, d2 = kf.kf_value_info(q.script, q.values[name])
        shape = (m, ld) if kind == 1 else ((m if d0 == decl_rows else n),) if kind == 0 else (1,)
        outs[name] = torch.full(shape, float("nan"), device="cuda")
        if kind == 1:
            kf.kf_bind_matrix(plan, q.values[name], outs[name].data_ptr(), ld)
        else:
            kf.kf_bind(plan, q.values[name], outs[name].data_ptr())
    kf.kf_run(plan, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in outs.items()}


def _workspace(plan):
    need = kf.kf_plan_workspace_bytes(plan)
    ws = torch.empty(need // 4 + 64, dtype=torch.float32, device="cuda")
    kf.kf_bind_workspace(plan, (ws.data_ptr() + 255) // 256 * 256, need)
    return ws


@pytest.mark.parametrize("name", ["bicgk", "gesummv", "gemver"])
@pytest.mark.parametrize("mode", ["fused", "unfused"])
def test_runtime_shapes_match_oracle_and_static_plans(name, mode):
    M = N = 1024
    scal = {"alpha": 1.5, "beta": 0.75}
    q = S.by_name(name, M, N, scal)
    plan = kf.kf_compile(q.script, mode=mode, flags=RS, **PARAMS)
    ws = _workspace(plan)
    for n in (1, 3, 64, 257, 1000, 1024):
        print("case", name, mode, n, flush=True)
        ld = I.padded_ld(n, 32)
        arrays, _ = WL.make(name, n, n, seed=WL.seed_for(31, name) + n, ld=ld, pad_value=np.nan)
        got = _run_at(q, plan, n, n, arrays, ld)
        for k in got:
            if got[k].ndim == 2:
                got[k] = got[k][:, :n]
        SC.check_against_oracle(name, n, n, got, SC.oracle_outputs(name, arrays, scal, n))
        # a plan compiled for exactly this shape, same parameters: same bits
        qs = S.by_name(name, n, n, scal, ld=ld)
        prog = qs.compile(mode=mode, **PARAMS)
        prog.bind(**{k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in arrays.items()})
        ref = {k: v.cpu().numpy() for k, v in prog.run().items()}
        torch.cuda.synchronize()
        for k in got:
            r = ref[k][:, :n] if ref[k].ndim == 2 else ref[k]
            assert np.array_equal(got[k], r, equal_nan=True), (name, mode, n, k)
        del prog
    kf.kf_plan_destroy(plan)
    del ws


def test_non_square_runtime_shapes():
    M, N = 700, 1500
    q = S.bicgk(M, N)
    plan = kf.kf_compile(q.script, mode="fused", flags=RS, **PARAMS)
    ws = _workspace(plan)
    for m, n in ((700, 1500), (1, 1500), (700, 1), (333, 1029)):
        print("case bicgk", m, n, flush=True)
        ld = I.padded_ld(n)
        arrays, _ = WL.make("bicgk", m, n, seed=41 + m + n, ld=ld)
        got = _run_at(q, plan, m, n, arrays, ld)
        SC.check_against_oracle("bicgk", m, n, got, SC.oracle_outputs("bicgk", arrays, {}, n))
    kf.kf_plan_destroy(plan)
    del ws


def test_run_many_and_batched_plan_loop():
    """The per-instance plan loop of the batched configuration against the
    oracle, instance by instance (edge sizes of every bucket included)."""
    k, n, a, b = B.make_instances(16, 16, seed=9, lo=1, hi=2048)
    edge = np.array([1, 2, 63, 64, 65, 511, 512, 513, 2047, 2048])
    kinds = np.concatenate([k, np.zeros(len(edge), np.int32), np.ones(len(edge), np.int32)])
    ns = np.concatenate([n, edge, edge])
    al = np.concatenate([a, np.ones(len(edge), np.float32), np.full(len(edge), 1.25, np.float32)])
    be = np.concatenate([b, np.ones(len(edge), np.float32), np.full(len(edge), 0.75, np.float32)])
    bt = B.Batch(kinds, ns, al, be)
    host_in = bt.host_arena(seed=12)
    bt.upload(host_in)
    loop = B.PlanLoop(bt)
    st = torch.cuda.current_stream().cuda_stream
    print("case plan loop: %d instances, %d launches" % (len(ns), loop.launches()), flush=True)
    loop.run(st)
    torch.cuda.synchronize()
    out = bt.arena.cpu().numpy()
    for i in range(len(ns)):
        nn, kind = int(ns[i]), int(kinds[i])
        off, ld = bt.offset(i, "A")
        A = host_in[off:off + nn * ld].reshape(nn, ld)
        v = {name: host_in[bt.offset(i, name)[0]:bt.offset(i, name)[0] + nn] for name in B.INPUTS[kind]}
        got = bt.outputs(out, i)
        if kind == B.BICGK:
            q, s = oracle.bicgk(A, v["p"], v["r"], cols=nn)
            ref = {"q": q, "s": s}
        else:
            Bm, x, w = oracle.gemver(float(al[i]), float(be[i]), A, v["u1"], v["v1"], v["u2"], v["v2"], v["y"], v["z"],
                                     cols=nn)
            ref = {"B": Bm, "x": x, "w": w}
        tol = WL.tolerance("bicgk" if kind == B.BICGK else "gemver", nn, nn)
        for key, r in ref.items():
            g = got[key][:, :nn] if key == "B" else got[key]
            e = WL.rel_l2(g, r)
            assert np.all(np.isfinite(g)) and e <= tol, (i, nn, kind, key, e, tol)
