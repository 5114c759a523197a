"""Batched uneven-size BiCGK / GEMVER instances run as one persistent launch.

`make_instances` draws the instance list (kind, n log-uniform, scalars) from a
seed; `Batch` owns the library batch, the device arena holding every
operand, and the workspace; inputs are generated on the host per instance
from counter-based streams (so any instance can be regenerated alone) and
copied to the device in one transfer.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import inputs as I
from . import kf

BICGK, GEMVER = kf.KF_BATCH_BICGK, kf.KF_BATCH_GEMVER
INPUTS = {BICGK: ["p", "r"], GEMVER: ["u1", "v1", "u2", "v2", "y", "z"]}
OUTPUTS = {BICGK: ["q", "s"], GEMVER: ["x", "w"]}
SLOTS = {BICGK: ["p", "r", "q", "s"], GEMVER: ["u1", "v1", "u2", "v2", "y", "z", "x", "w"]}


def make_instances(n_bicgk: int, n_gemver: int, seed: int, lo: int = 32, hi: int = 2048):
    """Kinds (BiCGK first), sizes log-uniform on [lo, hi], GEMVER scalars
    uniform on [0.5, 2]; deterministic in seed."""
    kinds = np.array([BICGK] * n_bicgk + [GEMVER] * n_gemver, dtype=np.int32)
    ns = I.loguniform_int(seed, 0, len(kinds), lo, hi)
    alpha = np.array([I.scalar_uniform(seed, 1000 + 2 * i) for i in range(len(kinds))], dtype=np.float32)
    beta = np.array([I.scalar_uniform(seed, 1001 + 2 * i) for i in range(len(kinds))], dtype=np.float32)
    alpha[kinds == BICGK] = 1.0
    beta[kinds == BICGK] = 1.0
    return kinds, ns, alpha, beta


def instance_inputs(seed: int, i: int, kind: int, n: int, ld: int = 0):
    """Operands of instance i: A (n x ld, NaN padding; ld = round_up(n, 32)
    by default, the batch's row pitch) and the input vectors, from the streams
    (seed * 2^20 + i, tensor id); values do not depend on ld."""
    s = int(seed) * (1 << 20) + int(i)
    out = {"A": I.matrix(s, 0, n, n, ld=ld or I.padded_ld(n, 32))}
    for t, name in enumerate(INPUTS[kind]):
        out[name] = I.vector(s, 1 + t, n)
    return out


class Batch:
    def __init__(self, kinds, ns, alpha=None, beta=None, opts=None, device="cuda"):
        self.kinds = np.asarray(kinds, dtype=np.int32)
        self.ns = np.asarray(ns, dtype=np.int64)
        self.alpha = None if alpha is None else np.asarray(alpha, dtype=np.float32)
        self.beta = None if beta is None else np.asarray(beta, dtype=np.float32)
        self.h = kf.kf_batch_create(self.kinds, self.ns, self.alpha, self.beta, opts)
        self.elems = kf.kf_batch_arena_elems(self.h)
        self.ws_bytes = kf.kf_batch_workspace_bytes(self.h)
        self.device = device
        self.arena = None
        self.ws = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h and kf is not None:
            kf.kf_batch_destroy(h)
            self.h = None

    def offset(self, i: int, name: str):
        kind = int(self.kinds[i])
        op = 0 if name == "A" else 1 if name == "B" else 2 + SLOTS[kind].index(name)
        return kf.kf_batch_offset(self.h, i, op)

    def host_arena(self, seed: int, threads: int = 0) -> np.ndarray:
        """Host copy of the arena with every input filled (outputs NaN)."""
        host = np.full(self.elems, np.nan, dtype=np.float32)

        def fill(i):
            n = int(self.ns[i])
            off, ld = self.offset(i, "A")
            vals = instance_inputs(seed, i, int(self.kinds[i]), n, ld)
            host[off:off + n * ld] = vals["A"].ravel()
            for name in INPUTS[int(self.kinds[i])]:
                o, _ = self.offset(i, name)
                host[o:o + n] = vals[name]
        with ThreadPoolExecutor(threads or I._threads()) as ex:
            list(ex.map(fill, range(len(self.kinds))))
        return host

    def upload(self, host: np.ndarray) -> None:
        """Device arena from a host copy, then bind."""
        self.arena = torch.from_numpy(host).to(self.device)
        self._bind()

    def fill_device(self, seed: int) -> None:
        """Device arena with the same inputs as host_arena(seed), generated on
        the device (outputs are left unset), then bind."""
        self.arena = torch.empty(max(1, self.elems), dtype=torch.float32, device=self.device)
        st = self.stream()
        base = self.arena.data_ptr()
        for i in range(len(self.kinds)):
            n, kind = int(self.ns[i]), int(self.kinds[i])
            sd = int(seed) * (1 << 20) + i
            off, ld = self.offset(i, "A")
            kf.kf_util_fill_uniform(base + 4 * off, n, n, ld, I.stream_key(sd, 0), float("nan"), st)
            for t, name in enumerate(INPUTS[kind]):
                o, _ = self.offset(i, name)
                kf.kf_util_fill_uniform(base + 4 * o, 1, n, n, I.stream_key(sd, 1 + t), 0.0, st)
        self._bind()

    def _bind(self) -> None:
        self.ws = torch.empty(max(256, self.ws_bytes), dtype=torch.uint8, device=self.device)
        kf.kf_batch_bind(self.h, self.arena.data_ptr(), self.ws.data_ptr(), self.stream())

    def stream(self):
        return torch.cuda.current_stream().cuda_stream

    def run(self, which: int = 0) -> None:
        kf.kf_batch_run(self.h, which, self.stream())

    def error(self) -> int:
        return kf.kf_batch_error(self.h, self.stream())

    def outputs(self, host: np.ndarray, i: int) -> dict:
        """Outputs of instance i from a host copy of the arena."""
        n = int(self.ns[i])
        kind = int(self.kinds[i])
        out = {}
        for name in OUTPUTS[kind]:
            o, _ = self.offset(i, name)
            out[name] = host[o:o + n]
        if kind == GEMVER:
            o, ld = self.offset(i, "B")
            out["B"] = host[o:o + n * ld].reshape(n, ld)
        return out

    def bytes(self):
        return kf.kf_batch_bytes(self.h)

    def describe(self) -> str:
        return kf.kf_batch_describe(self.h)


BUCKET_RANGE = [(1, 64), (65, 128), (129, 256), (257, 512), (513, 1024), (1025, 2048)]


def bucket_median(bucket: int, lo: int = 32, hi: int = 2048) -> int:
    """Median size of a log-uniform draw on [lo, hi] that falls in the bucket."""
    a, b = BUCKET_RANGE[bucket]
    a, b = max(a, lo), min(b, hi)
    return int(round(np.sqrt(a * b)))


def row_candidates(step: int, n: int) -> list:
    """Rows per item: the tile's rows per step times powers of two, up to one
    item per instance."""
    r = step
    out = []
    while True:
        out.append(r)
        if r >= n:
            break
        r *= 2
    return out


def autotune(kind: int, bucket: int, count: int = 683, seed: int = 1, reps: int = 5, log=None):
    """Grid search over the bucket's tile menu crossed with the rows per item,
    on `count` instances of the bucket's median size; returns ((best tile,
    best rows), [(tile, rows, us, GB/s)])."""
    n = bucket_median(bucket)
    res = []
    ntile = kf.kf_batch_tile_info(kind, bucket, 0)[0]
    for t in range(ntile):
        step = kf.kf_batch_tile_info(kind, bucket, t)[1]["rows_per_step"]
        for rows in row_candidates(step, n):
            rt = {0: [0] * 6, 1: [0] * 6}
            tt = {0: [0] * 6, 1: [0] * 6}
            rt[kind][bucket] = rows
            tt[kind][bucket] = t
            bt = Batch(np.full(count, kind, np.int32), np.full(count, n), np.full(count, 1.25, np.float32),
                       np.full(count, 0.75, np.float32), kf.batch_opts(rows=rt, tiles=tt))
            bt.fill_device(seed)
            us = kf.kf_batch_time(bt.h, 0, False, bt.stream(), 2, reps)
            r, w = bt.bytes()
            res.append((t, rows, us, (r + w) / us / 1e3))
            if log:
                log("tune kind %d bucket %d n %d tile %d rows %d: %.1f us %.1f GB/s" % (kind, bucket, n, t, rows, us,
                                                                                     res[-1][3]))
            del bt
            torch.cuda.empty_cache()
    best = min(res, key=lambda x: x[2])
    return (best[0], best[1]), res


def tune_mix(kinds, ns, alpha, beta, seed: int, rows0: dict, tiles0: dict, reps: int = 5, tol: float = 0.003,
             log=None):
    """Coordinate search of (tile, rows per item) per kind and size bucket on
    the mixed batch itself: from (rows0, tiles0), each bucket in turn (largest
    first, GEMVER first) tries every tile of its menu with rows per item from
    the tile's step up to the whole instance, keeping a change only when the
    whole launch gets more than `tol` faster. The arena is filled once and
    shared by every configuration (its layout depends on the sizes only).
    Returns (rows, tiles, best_us, [(kind, bucket, tile, rows, us)])."""
    rows = {k: list(v) for k, v in rows0.items()}
    tiles = {k: list(v) for k, v in tiles0.items()}
    base = Batch(kinds, ns, alpha, beta, kf.batch_opts(rows=rows, tiles=tiles))
    base.fill_device(seed)
    arena = base.arena
    nmax = [int(max([n for n, k in zip(ns, kinds) if k == kind and bucket_of(n) == b] or [0]))
            for kind in (0, 1) for b in range(6)]

    def timed(r, t):
        bt = Batch(kinds, ns, alpha, beta, kf.batch_opts(rows=r, tiles=t))
        bt.arena = arena
        bt._bind()
        us = kf.kf_batch_time(bt.h, 0, False, bt.stream(), 2, reps)
        del bt
        return us

    best = timed(rows, tiles)
    hist = [(-1, -1, -1, -1, best)]
    if log:
        log("mix start: %.1f us" % best)
    for kind in (1, 0):
        for b in reversed(range(6)):
            top = nmax[kind * 6 + b]
            if top == 0:
                continue
            ntile = kf.kf_batch_tile_info(kind, b, 0)[0]
            for t in range(ntile):
                step = kf.kf_batch_tile_info(kind, b, t)[1]["rows_per_step"]
                for r in row_candidates(step, top):
                    if t == tiles[kind][b] and r == rows[kind][b]:
                        continue
                    rr = {k: list(v) for k, v in rows.items()}
                    tt = {k: list(v) for k, v in tiles.items()}
                    rr[kind][b], tt[kind][b] = r, t
                    us = timed(rr, tt)
                    hist.append((kind, b, t, r, us))
                    if log:
                        log("mix kind %d bucket %d tile %d rows %d: %.1f us (best %.1f)" % (kind, b, t, r, us, best))
                    if us < best * (1.0 - tol):
                        best, rows, tiles = us, rr, tt
    return rows, tiles, best, hist


def bucket_of(n: int) -> int:
    return next(i for i, (a, b) in enumerate(BUCKET_RANGE) if n <= b)


BUCKET_MAX = [b for _, b in BUCKET_RANGE]


class PlanLoop:
    """Baseline of the batched launch: the library's own single-instance fused
    plans launched once per instance. One runtime-shape plan per (kind, size
    bucket), declared at the bucket's largest n with the library's default
    parameters for that shape, runs every instance of the bucket at its own
    size n x n and row pitch (kf_plan_run_many), on the operands of a bound
    Batch's arena; GEMVER's alpha and beta are per-instance device scalars."""

    def __init__(self, bt: "Batch", params: dict = None):
        from . import sequences as S
        assert bt.arena is not None, "upload or fill the batch first"
        self.bt = bt
        n_inst = len(bt.kinds)
        al = bt.alpha if bt.alpha is not None else np.ones(n_inst, np.float32)
        be = bt.beta if bt.beta is not None else np.ones(n_inst, np.float32)
        self.scal = torch.from_numpy(np.stack([al, be], 1).astype(np.float32).ravel()).to(bt.device)
        base, sbase = bt.arena.data_ptr(), self.scal.data_ptr()
        self.groups = []
        buckets = np.searchsorted(BUCKET_MAX, bt.ns)
        for kind in (BICGK, GEMVER):
            for b in range(len(BUCKET_MAX)):
                idx = np.flatnonzero((bt.kinds == kind) & (buckets == b))
                if not len(idx):
                    continue
                nmax = BUCKET_MAX[b]
                q = S.bicgk(nmax, nmax) if kind == BICGK else S.gemver_dev(nmax, nmax)
                plan = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_RUNTIME_SHAPE, **(params or {}))
                need = kf.kf_plan_workspace_bytes(plan)
                ws = torch.empty(need // 4 + 64, dtype=torch.float32, device=bt.device)
                kf.kf_bind_workspace(plan, (ws.data_ptr() + 255) // 256 * 256, need)
                names = (["A", "p", "r", "q", "s"] if kind == BICGK else
                         ["A", "u1", "v1", "u2", "v2", "y", "z", "alpha", "beta", "B", "x", "w"])
                vals = [q.values[nm] for nm in names]
                ptrs = np.zeros((len(idx), len(names)), np.uint64)
                lds = np.zeros((len(idx), len(names)), np.int64)
                for r, i in enumerate(idx):
                    for j, nm in enumerate(names):
                        if nm in ("alpha", "beta"):
                            ptrs[r, j] = sbase + 4 * (2 * int(i) + (nm == "beta"))
                        else:
                            off, ld = bt.offset(int(i), nm)
                            ptrs[r, j] = base + 4 * off
                            lds[r, j] = ld if nm in ("A", "B") else 0
                shapes = np.stack([bt.ns[idx], bt.ns[idx]], 1).astype(np.int64)
                self.groups.append((q, plan, ws, shapes, vals, ptrs, lds))

    def __del__(self):
        for g in getattr(self, "groups", []):
            if kf is not None:
                kf.kf_plan_destroy(g[1])
        self.groups = []

    def run(self, stream: int) -> None:
        for q, plan, ws, shapes, vals, ptrs, lds in self.groups:
            kf.kf_plan_run_many(plan, shapes, vals, ptrs, lds, stream)

    def launches(self) -> int:
        """HIP launches of one run of the loop."""
        tot = 0
        for q, plan, ws, shapes, vals, ptrs, lds in self.groups:
            per = sum(kf.kf_plan_num_launches(plan, k) for k in range(kf.kf_plan_num_kernels(plan)))
            tot += per * len(shapes)
        return tot
