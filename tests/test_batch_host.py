"""Host-side logic of the batched launch (no GPU): arena layout, work items,
queue order, byte accounting and argument checks."""
import numpy as np
import pytest

from paper_1305_1183_amd import batched as B
from paper_1305_1183_amd import kf

RPS = kf.BATCH_ROWS_PER_STEP


def bucket(n):
    return 0 if n <= 64 else 1 if n <= 128 else 2 if n <= 256 else 3 if n <= 512 else 4 if n <= 1024 else 5


def make(kinds, ns, **opts):
    o = kf.batch_opts(**opts) if opts else None
    return B.Batch(kinds, ns, np.full(len(ns), 1.5, np.float32), np.full(len(ns), 0.5, np.float32), o)


EDGE = [1, 2, 3, 4, 5, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2048]


@pytest.mark.parametrize("opts", [{}, {"rows": {0: RPS, 1: RPS}}, {"rows": {0: [2048] * 6, 1: [2048] * 6}}])
def test_layout_and_items(opts):
    kinds = np.array([0, 1] * len(EDGE), np.int32)
    ns = np.repeat(EDGE, 2)
    b = make(kinds, ns, **opts)
    rows = {k: (opts.get("rows", {}).get(k) or [None] * 6) for k in (0, 1)}
    spans = []
    for i, (k, n) in enumerate(zip(kinds, ns)):
        names = ["A"] + (["B"] if k == 1 else []) + B.SLOTS[k]
        for name in names:
            off, ld = b.offset(i, name)
            size = n * ld if name in ("A", "B") else n
            if name in ("A", "B"):
                assert ld == (n + 31) // 32 * 32
            assert off % 64 == 0                      # 256-byte aligned
            spans.append((off, off + size))
    spans.sort()
    assert spans[-1][1] <= b.elems
    assert all(a[1] <= c[0] for a, c in zip(spans, spans[1:])), "operands overlap"
    # every (instance, phase, block) exactly once, in both orders
    q = kf.kf_batch_items(b.h, 0)
    l = kf.kf_batch_items(b.h, 1)
    tq = sorted(zip(*[a.tolist() for a in q]))
    tl = sorted(zip(*[a.tolist() for a in l]))
    assert tq == tl and len(set(tq)) == len(tq)
    expect = []
    for i, (k, n) in enumerate(zip(kinds, ns)):
        r = rows[k][bucket(n)]
        r = {0: [64, 128, 256, 512, 256, 128], 1: [64, 128, 256, 128, 128, 64]}[k][bucket(n)] if r is None else r
        nblk = -(-n // r)
        expect += [(i, 0 if k == 0 else 1, j) for j in range(nblk)]
        if k == 1 and nblk > 1:
            expect += [(i, 2, j) for j in range(nblk)]
    assert tq == sorted(expect)
    # queue: all phase-1 items first, largest first; K2 blocks after them
    ph = q[1]
    first2 = np.argmax(ph == 2) if np.any(ph == 2) else len(ph)
    assert np.all(ph[:first2] != 2) and np.all(ph[first2:] == 2)
    # loop order: instance-major
    assert np.all(np.diff(l[0]) >= 0)


def test_bytes_match_fused_plan_counts():
    kinds = np.array([0, 1, 0, 1], np.int32)
    ns = np.array([100, 100, 2048, 33])
    b = make(kinds, ns)
    r, w = b.bytes()
    er = ew = 0
    for k, n in zip(kinds, ns):
        if k == 0:
            er += 4 * (n * n + 2 * n)
            ew += 4 * 2 * n
        else:
            er += 4 * (2 * n * n + 7 * n)
            ew += 4 * (n * n + 2 * n)
    assert (r, w) == (er, ew)


@pytest.mark.parametrize("kinds,ns,opts", [
    ([0], [0], None), ([0], [2049], None), ([2], [10], None),
    ([0], [100], {"rows": {0: [0, 0, 0, 0, 0, 3]}}),      # not a multiple of 4 rows per step
    ([0], [100], {"rows": {1: [17, 0, 0, 0, 0, 0]}}),
])
def test_create_rejects(kinds, ns, opts):
    with pytest.raises(kf.KFError):
        kf.kf_batch_create(np.array(kinds, np.int32), np.array(ns), None, None,
                           kf.batch_opts(**opts) if opts else None)


def test_instances_are_deterministic_and_in_range():
    k1, n1, a1, b1 = B.make_instances(50, 70, seed=9)
    k2, n2, a2, b2 = B.make_instances(50, 70, seed=9)
    assert np.array_equal(n1, n2) and np.array_equal(a1, a2) and np.array_equal(b1, b2)
    assert n1.min() >= 32 and n1.max() <= 2048 and (k1 == 0).sum() == 50
    assert np.all(a1[k1 == 1] >= 0.5) and np.all(a1[k1 == 1] <= 2.0)


def test_unbound_run_is_an_error():
    b = make(np.array([0], np.int32), np.array([10]))
    with pytest.raises(kf.KFError):
        kf.kf_batch_run(b.h, 0, 0)


def test_tile_menu_covers_each_bucket():
    """Every tile on a bucket's menu covers the bucket's widest rows (whole-row:
    2^ltpr lanes x k float4 >= n; wide: 256 lanes x k float4), reduces over at
    most its lanes, and entry 0 keeps the default rows per step."""
    top = [64, 128, 256, 512, 1024, 2048]
    for kind in (0, 1):
        for b in range(6):
            count, _ = kf.kf_batch_tile_info(kind, b, 0)
            assert count >= 1
            for t in range(count):
                _, x = kf.kf_batch_tile_info(kind, b, t)
                lanes = 256 if x["wide"] else 1 << x["ltpr"]
                assert lanes * x["k"] * 4 >= top[b], (kind, b, t, x)
                assert x["wide"] or x["lg"] <= x["ltpr"]
                assert not (x["wide"] and kind == 1), "GEMVER has no wide tile"
                step = (1 << x["lg"]) if x["wide"] else (256 >> x["ltpr"]) << x["lg"]
                assert x["rows_per_step"] == step
            assert kf.kf_batch_tile_info(kind, b, 0)[1]["rows_per_step"] == RPS[b]
            assert kf.kf_batch_tile_info(kind, b, count)[1] is None


def test_tile_choice_checks_and_describe():
    import json
    kinds, ns = np.array([0, 1, 0, 1], np.int32), np.array([40, 40, 1500, 700])
    # tile 2 of bucket 0 steps 128 rows: rows per block must be a multiple of 128
    with pytest.raises(kf.KFError) as e:
        make(kinds, ns, rows={0: [64, 0, 0, 0, 0, 0]}, tiles={0: [2, 0, 0, 0, 0, 0]})
    assert e.value.name == "KF_ERR_ARG"
    with pytest.raises(kf.KFError):
        make(kinds, ns, tiles={1: [0, 0, 0, 0, 0, 1]})          # GEMVER's bucket 5 has one tile
    with pytest.raises(kf.KFError):
        make(kinds, ns, tiles={0: [3, 0, 0, 0, 0, 0]})
    b = make(kinds, ns, tiles={0: [2, 0, 0, 0, 0, 2], 1: [1, 0, 0, 0, 2, 0]})
    d = json.loads(kf.kf_batch_describe(b.h))
    assert d["tiles"]["bicgk"][0] == "rows tpr8 k2 g4" and d["tiles"]["bicgk"][5] == "rows tpr64 k8 g1"
    assert d["tiles"]["gemver"][4] == "rows tpr32 k8 g1"
    assert d["rows"]["bicgk"][0] == 128                          # default 64 rounded up to the tile's step
