"""Batched uneven-size BiCGK / GEMVER on the GPU against the FP64 oracle,
instance by instance: the persistent launch, the per-instance launch loop,
graph replays of both, forced block splitting, a tiny persistent grid, the
device-side input fill, and the full 4096 + 4096 configuration on sampled
instances."""
import numpy as np
import pytest
import torch

import oracle
from paper_1305_1183_amd import batched as B
from paper_1305_1183_amd import kf
from paper_1305_1183_amd import workloads as WL

pytestmark = pytest.mark.gpu

RPS = kf.BATCH_ROWS_PER_STEP
EDGE = [1, 2, 3, 4, 5, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2048]


def small_batch(seed=5, opts=None):
    k, n, a, b = B.make_instances(24, 24, seed=seed, lo=1, hi=2048)
    kinds = np.concatenate([k, np.zeros(len(EDGE), np.int32), np.ones(len(EDGE), np.int32)])
    ns = np.concatenate([n, EDGE, EDGE])
    al = np.concatenate([a, np.ones(len(EDGE), np.float32), np.full(len(EDGE), 1.25, np.float32)])
    be = np.concatenate([b, np.ones(len(EDGE), np.float32), np.full(len(EDGE), 0.75, np.float32)])
    return B.Batch(kinds, ns, al, be, opts)


def reference(bt, host_in, i):
    n, kind = int(bt.ns[i]), int(bt.kinds[i])
    off, ld = bt.offset(i, "A")
    A = host_in[off:off + n * ld].reshape(n, ld)
    v = {name: host_in[bt.offset(i, name)[0]:bt.offset(i, name)[0] + n] for name in B.INPUTS[kind]}
    if kind == B.BICGK:
        q, s = oracle.bicgk(A, v["p"], v["r"], cols=n)
        return {"q": q, "s": s}
    Bm, x, w = oracle.gemver(float(bt.alpha[i]), float(bt.beta[i]), A, v["u1"], v["v1"], v["u2"], v["v2"],
                             v["y"], v["z"], cols=n)
    return {"B": Bm, "x": x, "w": w}


def check(bt, host_in, host_out, idx=None, refs=None):
    worst = 0.0
    for i in (range(len(bt.ns)) if idx is None else idx):
        n, kind = int(bt.ns[i]), int(bt.kinds[i])
        ref = refs[i] if refs is not None else reference(bt, host_in, i)
        got = bt.outputs(host_out, i)
        tol = WL.tolerance("bicgk" if kind == B.BICGK else "gemver", n, n)
        for name, r in ref.items():
            g = got[name][:, :n] if name == "B" else got[name]
            assert np.all(np.isfinite(g)), (i, n, kind, name)
            e = WL.rel_l2(g, r)
            worst = max(worst, e / tol)
            assert e <= tol, (i, n, kind, name, e, tol)
    return worst


def run_case(bt, which, graph=False, reps=1):
    host_in = bt.host_arena(seed=77)
    bt.upload(host_in)
    st = torch.cuda.Stream()
    refs = {i: reference(bt, host_in, i) for i in range(len(bt.ns))}
    with torch.cuda.stream(st):
        if graph:
            kf.kf_batch_capture(bt.h, which, st.cuda_stream)
        for r in range(reps):
            if graph:
                kf.kf_batch_graph_launch(bt.h, which, st.cuda_stream)
            else:
                kf.kf_batch_run(bt.h, which, st.cuda_stream)
            st.synchronize()
            assert kf.kf_batch_error(bt.h, st.cuda_stream) == 0
            out = bt.arena.cpu().numpy()
            check(bt, host_in, out, refs=refs)
            # eager work and a clear of the outputs between replays
            bt.arena.copy_(torch.from_numpy(host_in).cuda())
            torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("which", [0, 1])
def test_batch_matches_oracle(which):
    print("case batch which=%d" % which, flush=True)
    run_case(small_batch(), which)


@pytest.mark.parametrize("which", [0, 1])
def test_batch_graph_replays(which):
    print("case batch graph which=%d" % which, flush=True)
    run_case(small_batch(), which, graph=True, reps=3)


def _menu(kind, bucket):
    return [kf.kf_batch_tile_info(kind, bucket, t)[1] for t in range(kf.kf_batch_tile_info(kind, bucket, 0)[0])]


@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("split", [False, True])
def test_every_tile_on_the_menus(tile, split):
    """Each non-default tile of every bucket's menu, on whole instances and on
    instances split into blocks of one tile step, matches the oracle."""
    tiles = {k: [min(tile, len(_menu(k, b)) - 1) for b in range(6)] for k in (0, 1)}
    rows = {k: [(_menu(k, b)[tiles[k][b]]["rows_per_step"] if split else 2048) for b in range(6)] for k in (0, 1)}
    print("case batch tiles", tiles, "rows", rows, flush=True)
    run_case(small_batch(seed=9, opts=kf.batch_opts(rows=rows, tiles=tiles)), 0, reps=2)


@pytest.mark.parametrize("opts", [dict(rows={0: RPS, 1: RPS}), dict(rows={0: [2048] * 6, 1: [2048] * 6}),
                                  dict(grid=1), dict(grid=3, rows={0: RPS, 1: RPS})],
                         ids=["all-split", "all-whole", "grid1", "grid3-split"])
def test_batch_shapes(opts):
    print("case batch opts", opts, flush=True)
    run_case(small_batch(opts=kf.batch_opts(**opts)), 0, reps=2)


def test_batch_deterministic_and_device_fill():
    bt = small_batch(seed=6)
    host_in = bt.host_arena(seed=31)
    bt.fill_device(seed=31)
    dev = bt.arena.cpu().numpy()
    for i in range(len(bt.ns)):
        n, kind = int(bt.ns[i]), int(bt.kinds[i])
        o, ld = bt.offset(i, "A")
        a_d = dev[o:o + n * ld].reshape(n, ld)[:, :n]
        a_h = host_in[o:o + n * ld].reshape(n, ld)[:, :n]
        assert np.array_equal(a_d, a_h), i
        for name in B.INPUTS[kind]:
            o, _ = bt.offset(i, name)
            assert np.array_equal(dev[o:o + n], host_in[o:o + n]), (i, name)
    outs = []
    for _ in range(2):
        bt.run(0)
        torch.cuda.synchronize()
        outs.append(bt.arena.cpu().numpy())
    assert bt.error() == 0
    for i in range(len(bt.ns)):
        for name, v in bt.outputs(outs[0], i).items():
            assert np.array_equal(v, bt.outputs(outs[1], i)[name], equal_nan=True), (i, name)
    check(bt, host_in, outs[0])


def test_batch_full_config_sampled():
    """4096 BiCGK + 4096 GEMVER, n log-uniform on [32, 2048], persistent launch
    with the tuned tile shapes; instances checked in full on a sample that
    holds the smallest and largest of each kind."""
    kinds, ns, al, be = B.make_instances(4096, 4096, seed=WL.BATCH_SEED)
    print("case batch full", len(ns), int(ns.sum()), flush=True)
    bt = B.Batch(kinds, ns, al, be, WL.batch_opts())
    bt.fill_device(seed=WL.BATCH_SEED)
    bt.run(0)
    torch.cuda.synchronize()
    assert bt.error() == 0
    pick = set(np.random.default_rng(0).choice(len(ns), 48, replace=False).tolist())
    for k in (B.BICGK, B.GEMVER):
        idx = np.where(kinds == k)[0]
        pick |= {int(idx[np.argmin(ns[idx])]), int(idx[np.argmax(ns[idx])])}
    host_out = bt.arena.cpu().numpy()
    for i in sorted(pick):
        n, kind = int(ns[i]), int(kinds[i])
        vals = B.instance_inputs(WL.BATCH_SEED, i, kind, n)
        if kind == B.BICGK:
            q, s = oracle.bicgk(vals["A"], vals["p"], vals["r"], cols=n)
            ref = {"q": q, "s": s}
        else:
            Bm, x, w = oracle.gemver(float(al[i]), float(be[i]), vals["A"], vals["u1"], vals["v1"], vals["u2"],
                                     vals["v2"], vals["y"], vals["z"], cols=n)
            ref = {"B": Bm, "x": x, "w": w}
        check(bt, None, host_out, idx=[i], refs={i: ref})


def test_wait_timeout_reported_and_cleared():
    """A spin limit of one lets the dependent items of split GEMVER instances
    give up their bounded wait (every workgroup still exits). kf_batch_error
    reports the bit and clears the counters and the error word; a batch of the
    same instances with the default limit, bound to the same arena and
    workspace, then runs correctly."""
    kinds = np.full(64, B.GEMVER, np.int32)
    ns = np.full(64, 2000)
    al, be = np.full(64, 1.25, np.float32), np.full(64, 0.75, np.float32)
    tiny = B.Batch(kinds, ns, al, be, kf.batch_opts(spin_limit=1))
    good = B.Batch(kinds, ns, al, be, None)
    assert tiny.elems == good.elems and tiny.ws_bytes == good.ws_bytes
    host_in = tiny.host_arena(seed=19)
    tiny.upload(host_in)
    st = tiny.stream()
    print("case timeout: tiny spin limit", flush=True)
    tiny.run(0)
    bits = kf.kf_batch_error(tiny.h, st)
    assert bits in (0, 1), bits
    assert kf.kf_batch_error(tiny.h, st) == 0     # cleared by the first call
    print("case timeout: bits %d, then the default limit" % bits, flush=True)
    kf.kf_batch_bind(good.h, tiny.arena.data_ptr(), tiny.ws.data_ptr(), st)
    good.arena = tiny.arena
    good.run(0)
    assert kf.kf_batch_error(good.h, st) == 0
    out = good.arena.cpu().numpy()
    check(good, host_in, out, idx=[0, 31, 63])


def test_split_batch_replays_bitwise_deterministic():
    """The all-split small batch (every instance above one step cut into
    blocks, cross-XCD arrivals and flags in every instance) replayed from a
    graph 100 times: every replay gives the bits of the first run."""
    bt = small_batch(opts=kf.batch_opts(rows={0: RPS, 1: RPS}))
    host_in = bt.host_arena(seed=23)
    bt.upload(host_in)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        kf.kf_batch_run(bt.h, 0, st.cuda_stream)
        st.synchronize()
        first = bt.arena.cpu().numpy()
        check(bt, host_in, first)
        kf.kf_batch_capture(bt.h, 0, st.cuda_stream)
        for r in range(100):
            kf.kf_batch_graph_launch(bt.h, 0, st.cuda_stream)
            st.synchronize()
            got = bt.arena.cpu().numpy()
            assert np.array_equal(got, first, equal_nan=True), "replay %d differs" % r
        assert kf.kf_batch_error(bt.h, st.cuda_stream) == 0
