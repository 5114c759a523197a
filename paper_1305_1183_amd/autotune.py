"""Empirical choice of implementation parameters (Section 4.2, "fusion
implementations": block size and serial iterations per fusion).

For a compiled sequence and a fixed partition, every point of a parameter grid
is compiled and timed on the GPU (median of `reps` runs); the fastest wins.
Ties within 0.1% -- the paper's threshold for "same performance" -- go to the
point listed first.
"""
from __future__ import annotations

import itertools

from . import kf

MAT_GRID = [dict(mat_k=k, mat_waves=w, mat_group=g, mat_rows=r)
            for k in (1, 2)
            for (w, g) in ((4, 4), (4, 8), (8, 2), (8, 4), (2, 8))
            for r in (256, 512, 1024)] + \
           [dict(mat_k=k, mat_waves=w, mat_group=g, mat_rows=r)      # few waves, long row ranges:
            for k in (1, 2)                                          # fewer concurrent DRAM streams
            for (w, g, r) in ((4, 2, 1024), (4, 2, 2048), (2, 4, 2048), (8, 2, 2048), (4, 4, 2048), (4, 2, 4096))] + \
           [dict(mat_sched=1, mat_waves=w, mat_group=g, mat_rows=r)                # row-resident points
            for w in (8, 16) for g in (1, 2, 4) for r in (0, 16, 32, 64, 128)]
VEC_GRID = [dict(vec_unroll=u, vec_threads=t, vec_grid=g)
            for u in (2, 4, 8) for t in (256, 512) for g in (1024, 2048, 4096)] + \
           [dict(vec_unroll=u, vec_threads=256, vec_grid=g) for u in (4, 8) for g in (8192, 16384)]


def grid_for(seq) -> list:
    """Parameter grid for the iteration spaces present in the sequence."""
    kinds = set()
    for v in seq.inputs:
        kinds.add(len(seq.shapes[v]))
    has_mat = 2 in kinds
    has_vec = not has_mat
    out = []
    if has_mat:
        out += MAT_GRID
    if has_vec:
        out += VEC_GRID
    return out


def tune(seq, tensors: dict, mode="fused", partition=None, grid=None, warmup=2, reps=10,
         device="cuda"):
    """Return (best_params, [(params, median_us), ...]) for `seq` bound to `tensors`."""
    grid = grid if grid is not None else grid_for(seq)
    results = []
    for params in grid:
        kw = dict(params)
        if partition is not None:
            kw["partition"] = partition
        try:
            prog = seq.compile(mode=mode if partition is None else "partition", **kw)
        except kf.KFError:
            continue  # parameters outside the legal range for this shape
        prog.bind(device=device, **{k: tensors[k] for k in seq.inputs})
        us = prog.time(warmup, reps)
        results.append((params, us))
        del prog
    if not results:
        raise RuntimeError("no legal parameter point")
    best_us = min(t for _, t in results)
    for params, t in results:
        if t <= best_us * 1.001:
            return params, results
    return results[0][0], results


def tune_kernels(seq, tensors: dict, mode="fused", grid=None, warmup=2, reps=10, device="cuda"):
    """Per-kernel choice (Section 4.2: a plan combines one implementation per
    fused kernel). Every grid point is compiled with the plan's partition and
    timed kernel by kernel inside whole runs; each kernel keeps its fastest
    point (ties within 0.1% go to the point listed first).

    Returns (kernel_params, per_kernel) where kernel_params[k] is the chosen
    point of kernel k and per_kernel[k] the list of (params, median_us)."""
    grid = grid if grid is not None else grid_for(seq)
    per_kernel = None
    for params in grid:
        try:
            prog = seq.compile(mode=mode, **params)
        except kf.KFError:
            continue
        prog.bind(device=device, **{k: tensors[k] for k in seq.inputs})
        us = prog.time_kernels(warmup, reps)
        if per_kernel is None:
            per_kernel = [[] for _ in us]
        for k, t in enumerate(us):
            per_kernel[k].append((params, t))
        del prog
    if per_kernel is None:
        raise RuntimeError("no legal parameter point")
    chosen = []
    for res in per_kernel:
        best = min(t for _, t in res)
        chosen.append(next(p for p, t in res if t <= best * 1.001))
    return chosen, per_kernel
