"""Plan search (Section 4.2): candidates, the additive routine predictor, the
learned cost model, exhaustive timing, and the study that compares them.

Candidate plans of a script are the legal partitions crossed with implementation
parameter points (``kf.Candidates``). They are ranked by
* the paper's method: routine times measured in the same workgroup geometry,
  predicted per kernel as max(transfers, compute) and summed (``kf_predict_additive``);
* the learned cost model: an MLP over kernel features predicting log time, a
  plan being the sum of its kernels plus a per-launch term;
* exhaustive timing on the GPU, against which both are scored.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import kf

# BLAS-2 environments (k, waves, group, rows); k = 0 marks the row-resident
# schedule with its default geometry. BLAS-1 environments (unroll, threads, grid).
MAT_ENVS = [(1, 4, 4, 1024), (2, 8, 2, 1024), (1, 4, 4, 256), (2, 4, 4, 512), (0, 0, 0, 0)]
VEC_ENVS = [(4, 256, 2048), (4, 256, 4096), (2, 256, 1024)]


def mat_point(m):
    if m[0] == 0:
        return dict(mat_sched=1)
    return dict(mat_k=m[0], mat_waves=m[1], mat_group=m[2], mat_rows=m[3])


def grid_points():
    return [dict(mat_point(m), vec_unroll=v[0], vec_threads=v[1], vec_grid=v[2]) for m in MAT_ENVS for v in VEC_ENVS]


def sample_candidates(n: int, k: int, seed: int) -> list:
    """Deterministic subset of k candidate indices (always includes 0)."""
    if n <= k:
        return list(range(n))
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    rest = rng.choice(np.arange(1, n), size=k - 1, replace=False)
    return sorted([0] + [int(i) for i in rest])


# ---------------------------------------------------------------------------
# routine table (additive predictor)
# ---------------------------------------------------------------------------
# Extra LDS (KiB) of the probe environments: a fused kernel that holds more
# LDS than the probe itself fits fewer workgroups per CU.
LDS_AXIS = (0, 16, 32, 64)


def measure_routine_table(mat_shape=(8192, 8192), vec_n=1 << 24, reps=10, device="cuda", lds_axis=LDS_AXIS):
    """Routine table of the additive predictor: every BLAS-2 routine probed in
    each environment of MAT_ENVS (column strips, class 1; the row-resident
    schedule with its default geometry, class 2) at every extra-LDS amount of
    lds_axis, the FINISH launch of each environment, and the BLAS-1 routines.
    Entries are (cls, env, routine, us per unit, lds_kb)."""
    import torch
    from . import sequences as S
    rows, cols = mat_shape
    st = torch.cuda.current_stream().cuda_stream
    buf = torch.empty(max(rows * cols, vec_n) + (1 << 16), dtype=torch.float32, device=device)
    entries = []
    for env in MAT_ENVS:
        rowres = env[0] == 0
        p = mat_point(env)
        cls, tenv = (2, (0, 0, 0, 0)) if rowres else (1, tuple(env))
        for x in lds_axis:
            for r in range(5):
                us = kf.kf_routine_time(r, rows, cols, buf.data_ptr(), buf.numel() * 4, st, 2, reps,
                                        extra_lds_kb=x, **p)
                entries.append((cls, tenv, r, us / (rows * cols), x))
        # FINISH: the finishing launch of a column reduction in this environment
        # (the unfused gemtv for strips, single-pass ATAX's for row-resident)
        if rowres:
            q = S.atax(rows, cols)
            prog = q.compile(mode="fused", **p)
            prog.bind(A=buf[:rows * cols].view(rows, cols), x=buf[:cols].clone())
            entries.append((cls, tenv, 10, _launch_us(prog, 0, 1, reps), 0))
        else:
            q = S.bicgk(rows, cols)
            prog = q.compile(mode="unfused", **p)
            prog.bind(A=buf[:rows * cols].view(rows, cols), p=buf[:cols].clone(), r=buf[:rows].clone())
            entries.append((cls, tenv, 10, _launch_us(prog, 0, 1, reps), 0))
        del prog
    for env in VEC_ENVS:
        p = dict(vec_unroll=env[0], vec_threads=env[1], vec_grid=env[2])
        for r in range(5, 10):
            us = kf.kf_routine_time(r, vec_n, 0, buf.data_ptr(), buf.numel() * 4, st, 2, reps, **p)
            entries.append((0, tuple(env) + (0,), r, us / vec_n, 0))
        q = S.axpydot(vec_n, 1.5)
        prog = q.compile(mode="fused", **p)
        x = buf[:vec_n]
        prog.bind(w=x.clone(), v=x.clone(), u=x.clone())
        entries.append((0, tuple(env) + (0,), 10, _launch_us(prog, 0, 1, reps), 0))
    return entries


def _launch_us(prog, k, l, reps):
    import torch
    st = torch.cuda.current_stream()
    prog.run()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        kf.kf_run_kernel(prog.plan, k, st.cuda_stream)  # the launch's inputs are fresh
        a.record(st)
        kf.kf_run_launch(prog.plan, k, l, st.cuda_stream)
        b.record(st)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]) * 1e3)


def table_array(entries):
    return kf.routine_table(entries)


# ---------------------------------------------------------------------------
# data collection (exhaustive timing of sampled candidates)
# ---------------------------------------------------------------------------
def _grid(name: str):
    """The study's parameter grid ("study") or the library's default candidate
    grid ("default", None for kf_candidates)."""
    return grid_points() if name == "study" else None


def _precompile_job(args):
    seed, idx, cache_dir, grid = args
    os.environ["KF_CACHE_DIR"] = cache_dir
    from . import randscript as R
    rs = R.random_script(seed)
    c = kf.Candidates(rs.script, 64, _grid(grid))
    t0 = time.perf_counter()
    c.precompile(idx)
    dt = time.perf_counter() - t0
    names = set()
    for i in idx:
        p = c.compile(i, kf.KF_COMPILE_CODEGEN_ONLY)
        for kd in json.loads(kf.kf_plan_describe(p))["kernels"]:
            names.add(kd["name"])
        kf.kf_plan_destroy(p)
    return seed, dt, len(names)


def precompile(seeds, max_cands, cache_dir, workers, grid="study"):
    """Batch-compile the sampled candidates of each script in worker processes."""
    import multiprocessing as mp
    from . import randscript as R
    jobs = []
    for seed in seeds:
        rs = R.random_script(seed)
        c = kf.Candidates(rs.script, 64, _grid(grid))
        jobs.append((seed, sample_candidates(len(c), max_cands, seed), cache_dir, grid))
        del c, rs
    ctx = mp.get_context("spawn")
    out = {}
    with ctx.Pool(workers) as pool:
        for seed, dt, nk in pool.imap_unordered(_precompile_job, jobs):
            out[seed] = (dt, nk)
            print("precompiled script %d: %d kernels in %.1f s" % (seed, nk, dt), flush=True)
    return out, {j[0]: j[1] for j in jobs}


class Instance:
    """Device buffers of a random script: inputs (uniform [-1, 1)), outputs, workspace."""

    def __init__(self, rs, device="cuda"):
        import torch
        self.rs = rs
        self.t = {}
        g = torch.Generator(device=device)
        g.manual_seed(rs.seed)
        for v, shape in rs.inputs.items():
            self.t[v] = torch.empty(shape, dtype=torch.float32, device=device).uniform_(-1, 1, generator=g)
        for v, shape in rs.outputs.items():
            self.t[v] = torch.empty(shape, dtype=torch.float32, device=device)
        self.ws = None
        self.device = device

    def bind(self, plan):
        import torch
        for v, t in self.t.items():
            kf.kf_bind(plan, v, t.data_ptr())
        nb = kf.kf_plan_workspace_bytes(plan)
        if self.ws is None or self.ws.numel() * 4 < nb + 256:
            self.ws = None
            torch.cuda.empty_cache()
            self.ws = torch.empty(nb // 4 + 128, dtype=torch.float32, device=self.device)
        base = (self.ws.data_ptr() + 255) // 256 * 256
        kf.kf_bind_workspace(plan, base, nb)


def time_candidate(plan, reps=3, warmup=1):
    """(plan median us, per-kernel median us, wall seconds)."""
    import torch
    t0 = time.perf_counter()
    st = torch.cuda.current_stream()
    plan_us = kf.kf_time_plan(plan, st.cuda_stream, warmup, reps)
    nk = kf.kf_plan_num_kernels(plan)
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nk)]
           for _ in range(reps)]
    for r in range(reps):
        for k in range(nk):
            evs[r][k][0].record(st)
            kf.kf_run_kernel(plan, k, st.cuda_stream)
            evs[r][k][1].record(st)
    torch.cuda.synchronize()
    ku = [float(np.median([evs[r][k][0].elapsed_time(evs[r][k][1]) for r in range(reps)]) * 1e3)
          for k in range(nk)]
    return plan_us, ku, time.perf_counter() - t0


def _name_hash(name: str) -> int:
    return int(name.split("_")[-1][:15], 16) if "_" in name else 0


def collect(seeds, max_cands=512, cache_dir="/tmp/kf_cache", workers=14, reps=3, log=print, checkpoint=None,
            grid="study"):
    """Exhaustively time the candidates of each script (GPU). Kernels shared by
    several candidates are stored once (uk_*); kern_* rows are (candidate,
    kernel) timings."""
    import torch
    from . import randscript as R
    os.makedirs(cache_dir, exist_ok=True)
    os.environ["KF_CACHE_DIR"] = cache_dir
    comp, chosen = precompile(seeds, max_cands, cache_dir, workers, grid)
    rec = {k: [] for k in ("cand_seed", "cand_idx", "plan_us", "cand_nk", "cand_wall", "cand_launches")}
    krec = {k: [] for k in ("kern_cand", "kern_uk", "kern_us")}
    urec = {k: [] for k in ("uk_seed", "uk_hash", "uk_feat")}
    srec = {k: [] for k in ("script_seed", "script_compile_s", "script_nkernels", "script_codegen_s",
                            "script_load_s", "script_ncands")}
    for seed in seeds:
        rs = R.random_script(seed)
        c = kf.Candidates(rs.script, 64, _grid(grid))
        idx = chosen[seed]
        t0 = time.perf_counter()
        feats, ukmap = [], {}
        for i in idx:
            p = c.compile(i, kf.KF_COMPILE_CODEGEN_ONLY)
            d = json.loads(kf.kf_plan_describe(p))
            f = kf.kf_plan_features(p)
            ids = []
            for k, kd in enumerate(d["kernels"]):
                if kd["name"] not in ukmap:
                    ukmap[kd["name"]] = len(urec["uk_seed"])
                    urec["uk_seed"].append(seed)
                    urec["uk_hash"].append(_name_hash(kd["name"]))
                    urec["uk_feat"].append(f[k])
                ids.append(ukmap[kd["name"]])
            feats.append((ids, sum(len(k["launches"]) for k in d["kernels"])))
            kf.kf_plan_destroy(p)
        codegen_s = time.perf_counter() - t0
        inst = Instance(rs)
        load_s = 0.0
        for j, i in enumerate(idx):
            t1 = time.perf_counter()
            plan = c.compile(i)
            load_s += time.perf_counter() - t1
            inst.bind(plan)
            plan_us, ku, wall = time_candidate(plan, reps)
            kf.kf_plan_destroy(plan)
            ids, nl = feats[j]
            ci = len(rec["cand_seed"])
            rec["cand_seed"].append(seed)
            rec["cand_idx"].append(i)
            rec["plan_us"].append(plan_us)
            rec["cand_nk"].append(len(ku))
            rec["cand_wall"].append(wall)
            rec["cand_launches"].append(nl)
            for k, us in enumerate(ku):
                krec["kern_cand"].append(ci)
                krec["kern_uk"].append(ids[k])
                krec["kern_us"].append(us)
        srec["script_seed"].append(seed)
        srec["script_compile_s"].append(comp[seed][0])
        srec["script_nkernels"].append(comp[seed][1])
        srec["script_codegen_s"].append(codegen_s)
        srec["script_load_s"].append(load_s)
        srec["script_ncands"].append(len(idx))
        best = min(rec["plan_us"][-len(idx):])
        log("script %d (%s): %d candidates, %d kernels, best %.1f us, compile %.1f s" %
            (seed, rs.describe(), len(idx), len(ukmap), best, comp[seed][0]))
        del inst
        torch.cuda.empty_cache()
        kf.kf_jit_release()
        if checkpoint is not None and len(srec["script_seed"]) % 10 == 0:
            checkpoint(_pack(rec, srec, krec, urec))
    return _pack(rec, srec, krec, urec)


def _pack(rec, srec, krec, urec):
    out = {k: np.array(v) for k, v in {**rec, **srec}.items()}
    out["kern_cand"] = np.array(krec["kern_cand"], dtype=np.int64)
    out["kern_uk"] = np.array(krec["kern_uk"], dtype=np.int64)
    out["kern_us"] = np.array(krec["kern_us"])
    out["uk_seed"] = np.array(urec["uk_seed"], dtype=np.int64)
    out["uk_hash"] = np.array(urec["uk_hash"], dtype=np.int64)
    out["uk_feat"] = np.array(urec["uk_feat"], dtype=np.float32).reshape(-1, kf.FEATURE_DIM)
    return out


def merge(datasets):
    """Concatenate collected chunks (candidate and kernel indices re-based)."""
    out, coff, uoff = {}, 0, 0
    for d in datasets:
        d = dict(d)
        d["kern_cand"] = d["kern_cand"] + coff
        d["kern_uk"] = d["kern_uk"] + uoff
        coff += len(d["cand_seed"])
        uoff += len(d["uk_seed"])
        for k, v in d.items():
            out.setdefault(k, []).append(v)
    return {k: np.concatenate(v) for k, v in out.items()}


# ---------------------------------------------------------------------------
# training and evaluation
# ---------------------------------------------------------------------------
def kernel_training_set(data, seeds):
    """Unique (script, kernel) samples: features and log of the median time."""
    keep = np.isin(data["cand_seed"][data["kern_cand"]], list(seeds))
    times = {}
    for u, us in zip(data["kern_uk"][keep], data["kern_us"][keep]):
        times.setdefault(int(u), []).append(us)
    ids = np.array(sorted(times))
    X = data["uk_feat"][ids].astype(np.float32)
    y = np.log(np.array([max(np.median(times[u]), 0.1) for u in ids]))
    return X, y


def fit_launch_term(data, seeds, kern_pred_us=None):
    """Least-squares per-launch cost: plan - sum(kernels) ~ c * launches."""
    m = np.isin(data["cand_seed"], list(seeds))
    ksum = np.zeros(len(data["cand_seed"]))
    np.add.at(ksum, data["kern_cand"], data["kern_us"] if kern_pred_us is None else kern_pred_us)
    r = (data["plan_us"] - ksum)[m]
    L = data["cand_launches"][m].astype(np.float64)
    return float(max(0.0, np.dot(L, r) / max(np.dot(L, L), 1e-9)))


def rank_metrics(true_us, pred_us, tie=1e-3):
    """Table 4 analogues for one script."""
    order = np.argsort(pred_us, kind="stable")
    best = float(np.min(true_us))
    pos = next(i for i, j in enumerate(order) if true_us[j] <= best * (1 + tie))
    top1 = float(true_us[order[0]])
    return {"rank_of_best": int(pos) + 1, "first_pct_of_best": best / top1 * 100.0,
            "regret_top1": top1 / best - 1.0,
            "regret_top3": float(np.min(true_us[order[:3]])) / best - 1.0,
            "worst_pct_of_best": best / float(np.max(true_us)) * 100.0, "n": int(len(true_us))}


def combination_gain(data, seeds, c_launch, log=None):
    """Per script, the best measured candidate against the best per-kernel
    combination of the measured candidates (Section 4.2: one implementation
    per fused kernel), both estimated as the sum of measured kernel times plus
    c_launch per launch: candidates sharing a partition are grouped, and each
    kernel takes its fastest timing in the group (host only)."""
    from . import randscript as R
    out = []
    kern_of = {}
    for r, ci in enumerate(data["kern_cand"]):
        kern_of.setdefault(int(ci), []).append(r)
    for seed in seeds:
        m = np.where(data["cand_seed"] == seed)[0]
        if len(m) == 0:
            continue
        rs = R.random_script(seed)
        c = kf.Candidates(rs.script, 64, grid_points())
        groups = {}
        for ci in m:
            groups.setdefault(tuple(c.partition(int(data["cand_idx"][ci]))), []).append(int(ci))
        est = {ci: sum(data["kern_us"][r] for r in kern_of[ci]) + c_launch * data["cand_launches"][ci] for ci in m}
        uniform = min(est.values())
        comb = None
        for cis in groups.values():
            nk = len(kern_of[cis[0]])
            t = sum(min(data["kern_us"][kern_of[ci][k]] for ci in cis) for k in range(nk))
            t += c_launch * data["cand_launches"][cis[0]]
            comb = t if comb is None else min(comb, t)
        row = {"seed": int(seed), "candidates": int(len(m)), "partitions": len(groups),
               "best_measured_plan_us": float(data["plan_us"][m].min()),
               "uniform_est_us": float(uniform), "combination_est_us": float(comb),
               "gain": float(1.0 - comb / uniform)}
        out.append(row)
        if log:
            log("script %d: %d candidates in %d partitions, combination %.1f%% below the best candidate" %
                (seed, len(m), len(groups), row["gain"] * 100))
        del c, rs
    return out
