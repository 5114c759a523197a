#!/usr/bin/env python3
"""Benchmark: the single-instance FP32 suite of Table 1 sequences on one MI355X.

One step runs the fused plan of every sequence once -- AXPYDOT and WAXPBY on
2**26-entry vectors, BiCGK, ATAX, GESUMMV and GEMVER on 16384 x 16384 row-major
matrices -- over inputs already resident in HBM. `value` is the algorithmic
bytes of the six fused plans (each operand counted once per kernel that moves
it through HBM, as in the paper's bandwidth figures) divided by the time of a
step. Per-sequence fused and unfused times give the speedup of fusion.

Prints one JSON line. `--gpus` above 1 is refused: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "fused-sequence GB/s (% of HBM peak) & speedup vs unfused, FP32 GEMVER/BiCGK"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", default="", help="comma-separated subset of sequences (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-unfused", action="store_true")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="leave out the batched and reduced-precision results of the default line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB streaming copy (memory-counter calibration)")
    ap.add_argument("--tune", action="store_true",
                    help="grid-search the implementation parameters of every sequence and print them")
    ap.add_argument("--batched", action="store_true",
                    help="batched uneven sizes: 4096 BiCGK + 4096 GEMVER, n log-uniform on [32, 2048], "
                         "one persistent launch vs a loop of per-instance launches")
    ap.add_argument("--batched-no-loop", action="store_true",
                    help="with --batched: time only the persistent launch (for counter runs)")
    ap.add_argument("--tune-batch", action="store_true",
                    help="grid-search the lane tile and rows per work item of every size bucket of the batched "
                         "launch, bucket by bucket on instances of the bucket's median size")
    ap.add_argument("--tune-batch-mix", action="store_true",
                    help="coordinate search of the lane tile and rows per work item of every size bucket on the "
                         "mixed 4096 + 4096 batch itself")
    ap.add_argument("--layout", action="store_true",
                    help="row- vs column-major A: fused BiCGK, ATAX, SGEMVT, GEMVER at n = 16384")
    ap.add_argument("--precision", action="store_true",
                    help="reduced-precision suite: BiCGK and GEMVER at n = 32768 with A in FP32, BF16, FP8-E4M3")
    ap.add_argument("--wide-rows", action="store_true",
                    help="row-resident kernels at n = 32768: the geometry the library picks against the same "
                         "geometry requested explicitly (which the generator emits unadjusted)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads() -> int:
    """Threads for the all-core oracle run: the CPUs this process may run on,
    capped by OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS", "")
    return min(n, int(cap)) if cap.isdigit() and int(cap) > 0 else n


def cpu_baseline():
    """The FP64 oracle (plain C, unfused definitions) on the suite's full
    shapes, timed on this host: the all-core OpenMP build of the same source
    (one warm-up, then the median of three passes) and the one-thread build
    (one pass). GB/s over the FP32 algorithmic bytes of the unfused GPU plans
    of the same shapes."""
    import oracle
    from paper_1305_1183_amd import kf
    from paper_1305_1183_amd import sequences as S
    from paper_1305_1183_amd import workloads as WL
    from tests import seqcheck as SC  # the oracle: CPU-baseline leg only

    n, vec = WL.SUITE_N, WL.SUITE_VEC
    want = oracle_threads()
    total_bytes, t_one, t_all, used = 0, 0.0, 0.0, 1
    per = {}
    for name in WL.ORDER:
        m, nn = (vec, vec) if name in WL.BLAS1 else (n, n)
        arrays, scal = WL.make(name, m, nn, seed=WL.seed_for(2, name))
        q = S.by_name(name, m, nn, scal)
        p = kf.kf_compile(q.script, mode="unfused", flags=kf.KF_COMPILE_NO_LOAD)
        r, w = kf.kf_plan_bytes(p)
        kf.kf_plan_destroy(p)
        t0 = time.perf_counter()
        SC.oracle_outputs(name, arrays, scal, nn)
        one = time.perf_counter() - t0
        with oracle.all_cores(want) as used:
            times = []
            for rep in range(4):
                t0 = time.perf_counter()
                SC.oracle_outputs(name, arrays, scal, nn)
                if rep:
                    times.append(time.perf_counter() - t0)
        allc = float(np.median(times))
        del arrays
        total_bytes += r + w
        t_one += one
        t_all += allc
        per[name] = {"one_thread_s": round(one, 3), "all_cores_s": round(allc, 3), "unfused_bytes": r + w}
        log("cpu oracle %-8s one thread %.2f s, %d threads %.2f s" % (name, one, used, allc))
    return {"value": round(total_bytes / t_all / 1e9, 3), "unit": "GB/s", "cores": used,
            "kind": "oracle",
            "sample": "FP64 oracle (unfused definitions) on the full suite shapes: BiCGK/ATAX/GESUMMV/GEMVER "
                      "on %d x %d, AXPYDOT/WAXPBY on 2^26 entries; OpenMP build on %d threads, median of 3 "
                      "passes after one warm-up, %.1f s per pass; GB/s over the unfused GPU plans' FP32 "
                      "algorithmic bytes" % (n, n, used, t_all),
            "single_thread": {"value": round(total_bytes / t_one / 1e9, 3), "unit": "GB/s", "cores": 1,
                              "seconds": round(t_one, 2)},
            "cpu_model": cpu_model(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "bytes": total_bytes, "per_sequence": per}


def precision_suite(args, torch, kf, S, WL, dev):
    """GB/s of BiCGK and GEMVER at n = 32768 with A stored as FP32, BF16 and
    FP8-E4M3 (row scales), fused and unfused (one JSON line; not the headline)."""
    n = WL.PREC_N
    res = {}
    for name in WL.PREC_SEQ:
        t0 = time.time()
        stored, vecs, scal = WL.precision_inputs(name, n, WL.PREC_FORMATS, seed=4000 + WL.SEQ_INDEX[name])
        log("precision inputs %s: %.1f s" % (name, time.time() - t0))
        for fmt in WL.PREC_FORMATS:
            arrays = WL.precision_arrays(fmt, stored, vecs)
            q = S.bicgk_q(n, n, fmt) if name == "bicgk" else S.gemver_q(n, n, scal["alpha"], scal["beta"], fmt)
            devin = {}
            for k, v in arrays.items():
                if v.dtype == np.uint16:
                    v = v.view(np.int16)
                devin[k] = torch.from_numpy(np.ascontiguousarray(v)).to(dev)
            del arrays
            row = {}
            tp = WL.PREC_TUNED.get((name, fmt), {})
            variants = [("fused", "fused", tp), ("unfused", "unfused", {}),
                        ("unfused_same_params", "unfused", WL.plan_wide(tp))]
            if fmt != "f32":
                variants += [("fused_unit4", "fused", dict(tp, mat_unit=4)), ("fused_unit16", "fused", dict(tp, mat_unit=16))]
            # about 0.3 s of the fused plan first, so that the first timed variant
            # does not run on a device still ramping up after the input upload
            warm = q.compile(mode="fused", **tp).bind(device=dev, **devin)
            t_end = time.time() + 0.3
            while time.time() < t_end:
                warm.run()
                torch.cuda.synchronize()
            del warm
            for key, mode, extra in variants:
                try:
                    prog = q.compile(mode=mode, **extra).bind(device=dev, **devin)
                except kf.KFError as e:          # e.g. a load width these parameters cannot take
                    row[key] = {"illegal": str(e)}
                    continue
                r, w = prog.bytes()
                us = prog.time(3, 20)
                row[key] = {"us": round(us, 2), "bytes": r + w, "gbps": round((r + w) / us / 1e3, 1),
                            "pct_peak": round((r + w) / us / 1e3 / HBM_PEAK_GBPS * 100, 1)}
                del prog
            best_unfused = min(row["unfused"]["us"], row["unfused_same_params"]["us"])
            row["speedup"] = round(best_unfused / row["fused"]["us"], 3)
            res["%s/%s" % (name, fmt)] = row
            log("precision %s %s: fused %.1f us (%.1f GB/s), unfused %.1f us" %
                (name, fmt, row["fused"]["us"], row["fused"]["gbps"], row["unfused"]["us"]))
            del devin
            torch.cuda.empty_cache()
        del stored
    print(json.dumps({"metric": "reduced-precision A: GB/s and speedup vs unfused (not the headline)",
                      "n": n, "results": res, "unit": "GB/s", "peak": HBM_PEAK_GBPS}), flush=True)


def wide_rows_suite(args, torch, kf, S, WL, dev):
    """Row-resident kernels on rows of 32768 columns (eight float4 per lane per
    row): fused plans with the geometry the library picks (it halves the rows
    per group and moves column vectors out of the registers when they would
    not fit) against the same 16-wave, two-rows-per-group geometry requested
    explicitly (one JSON line; not the headline)."""
    n = 32768
    asked = dict(mat_sched=1, mat_waves=16, mat_group=2, mat_rows=128)
    cases = [("atax", kf.KF_ROW_MAJOR, {}), ("sgemvt", kf.KF_COL_MAJOR, {}), ("gemver", kf.KF_COL_MAJOR, {}),
             ("bicgk", kf.KF_ROW_MAJOR, dict(mat_sched=1)), ("gesummv", kf.KF_ROW_MAJOR, dict(mat_sched=1)),
             ("gemver", kf.KF_ROW_MAJOR, dict(mat_sched=1))]
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    res = {}
    for name, layout, params in cases:
        q = S.by_name(name, n, n, {"alpha": 1.5, "beta": 0.75}, layout=layout)
        devin = {k: torch.empty(q.shapes[k], dtype=torch.float32, device=dev).uniform_(-1, 1, generator=gen)
                 for k in q.inputs}
        row = {}
        for key, opts in (("library", params), ("requested", asked)):
            prog = q.compile(mode="fused", **opts).bind(device=dev, **devin)
            r, w = prog.bytes()
            us = prog.time(3, 20)
            d = json.loads(kf.kf_plan_describe(prog.plan))
            row[key] = {"us": round(us, 1), "gbps": round((r + w) / us / 1e3, 1),
                        "kernels": [k["name"] for k in d["kernels"]], "params": [k["params"] for k in d["kernels"]]}
            del prog
        key = "%s/%s%s" % (name, "col" if layout == kf.KF_COL_MAJOR else "row", "/sched1" if params else "")
        row["speedup"] = round(row["requested"]["us"] / row["library"]["us"], 3)
        res[key] = row
        log("wide rows %s: library %.1f us, requested %.1f us" % (key, row["library"]["us"], row["requested"]["us"]))
        del devin
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "row-resident kernels at n = 32768: library geometry vs requested (not the headline)",
                      "n": n, "requested": asked, "results": res, "unit": "us",
                      "config": {"workload": "fused ATAX, SGEMVT (column-major), GEMVER (both layouts), BiCGK and "
                                             "GESUMMV (row-resident schedule), A 32768 x 32768 FP32 uniform[-1, 1)"}}),
          flush=True)


def layout_suite(args, torch, kf, S, WL, dev):
    """Fused plans of BiCGK, ATAX, SGEMVT and GEMVER at n = 16384 with A
    row-major and column-major (one JSON line; not the headline). The layout
    moves the dependence that blocks fusion, so the kernel counts differ."""
    n = WL.SUITE_N
    scal = {"alpha": 1.5, "beta": 0.75}
    gen = torch.Generator(device=dev)
    gen.manual_seed(5150)
    res = {}
    for name in WL.LAYOUT_SEQ:
        row = {}
        for key, layout, params in (("row", kf.KF_ROW_MAJOR, WL.TUNED.get((name, "fused"), {})),
                                    ("col", kf.KF_COL_MAJOR, WL.LAYOUT_TUNED[name])):
            q = S.by_name(name, n, n, scal, layout=layout)
            devin = {k: torch.empty(q.shapes[k], dtype=torch.float32, device=dev).uniform_(-1, 1, generator=gen)
                     for k in q.inputs}
            prog = q.compile(mode="fused", **params).bind(device=dev, **devin)
            r, w = prog.bytes()
            us = prog.time(3, 20)
            row[key] = {"us": round(us, 2), "kernels": prog.num_kernels, "bytes": r + w,
                        "gbps": round((r + w) / us / 1e3, 1),
                        "pct_peak": round((r + w) / us / 1e3 / HBM_PEAK_GBPS * 100, 1)}
            del prog, devin
            torch.cuda.empty_cache()
        row["col_speedup"] = round(row["row"]["us"] / row["col"]["us"], 3)
        res[name] = row
        log("layout %s: row %.1f us (%d kernels), col %.1f us (%d kernels)" %
            (name, row["row"]["us"], row["row"]["kernels"], row["col"]["us"], row["col"]["kernels"]))
    print(json.dumps({"metric": "fused plans, row- vs column-major A: time, kernels, GB/s (not the headline)",
                      "n": n, "results": res, "unit": "GB/s", "peak": HBM_PEAK_GBPS,
                      "config": {"workload": "BiCGK/ATAX/SGEMVT/GEMVER, A 16384 x 16384 FP32 uniform[-1, 1)"}}),
          flush=True)


def batched_suite(args, torch, kf, WL, dev):
    """GB/s of the batched configuration: the persistent launch, the loop of
    per-instance launches, and graph replays of both (one JSON line; not the
    headline)."""
    from paper_1305_1183_amd import batched as B
    kinds, ns, al, be = B.make_instances(*WL.BATCH_COUNTS, seed=WL.BATCH_SEED)
    res = {}
    modes = ((0, "persistent"),) if args.batched_no_loop else ((0, "persistent"), (1, "loop"))
    for which, name in modes:
        t0 = time.time()
        bt = B.Batch(kinds, ns, al, be, WL.batch_opts(loop=which == 1))
        bt.fill_device(seed=WL.BATCH_SEED)
        torch.cuda.synchronize()
        log("batched inputs (%s items): %d instances, %.1f s" % (name, len(ns), time.time() - t0))
        r, w = bt.bytes()
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            us = kf.kf_batch_time(bt.h, which, False, st.cuda_stream, args.warmup, max(3, args.steps // 4))
            kf.kf_batch_capture(bt.h, which, st.cuda_stream)
            ug = kf.kf_batch_time(bt.h, which, True, st.cuda_stream, args.warmup, max(3, args.steps // 4))
            err = kf.kf_batch_error(bt.h, st.cuda_stream)
        if err:
            raise RuntimeError("batched launch reported error bits %d" % err)
        res[name] = {"us": round(us, 1), "gbps": round((r + w) / us / 1e3, 1),
                     "pct_peak": round((r + w) / us / 1e3 / HBM_PEAK_GBPS * 100, 1)}
        res[name + "_graph"] = {"us": round(ug, 1), "gbps": round((r + w) / ug / 1e3, 1),
                                "pct_peak": round((r + w) / ug / 1e3 / HBM_PEAK_GBPS * 100, 1)}
        res[name + "_batch"] = json.loads(bt.describe())
        log("batched %s: %.1f us, graph %.1f us" % (name, us, ug))
        del bt
        torch.cuda.empty_cache()
    loop = "loop" in res
    if loop:
        pl = plan_loop_times(torch, kf, WL, dev, kinds, ns, al, be, reps=max(3, args.steps // 4))
        r_, w_ = B.Batch(kinds, ns, al, be, WL.batch_opts()).bytes()
        for key in ("plan_loop", "plan_loop_graph"):
            res[key] = {"us": pl[key + "_us"], "gbps": round((r_ + w_) / pl[key + "_us"] / 1e3, 1)}
        res["plan_loop"]["launches"] = pl["plan_loop_launches"]
        log("batched plan loop: %.1f us, graph %.1f us" % (pl["plan_loop_us"], pl["plan_loop_graph_us"]))
    best_loop = min(res["loop"]["us"], res["loop_graph"]["us"], res["plan_loop"]["us"],
                    res["plan_loop_graph"]["us"]) if loop else None
    ach = res["persistent"]["gbps"]
    print(json.dumps({"metric": "batched uneven sizes: GB/s and speedup of one persistent launch vs per-instance "
                                "launches (not the headline)",
                      "value": res["persistent_graph"]["gbps"], "unit": "GB/s",
                      "speedup_vs_loop": round(res["loop"]["us"] / res["persistent"]["us"], 2) if loop else None,
                      "speedup_vs_best_loop": round(best_loop / res["persistent_graph"]["us"], 2) if loop else None,
                      "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                   "frac": round(ach / HBM_PEAK_GBPS, 4),
                                   "traffic": WL.traffic_from_profiles(os.path.join(ROOT, "profiles"),
                                                                       "kfb_kernel", batched=True),
                                   "kernel": "kfb_kernel (persistent launch, one dispatch)"},
                      "bytes": r + w, "results": res,
                      "config": {"workload": "%d BiCGK + %d GEMVER, n log-uniform on [32, 2048], FP32 uniform[-1,1)"
                                             % WL.BATCH_COUNTS}}), flush=True)


def batched_compact(args, torch, kf, WL, dev):
    """Batched uneven sizes (4096 BiCGK + 4096 GEMVER, n log-uniform on
    [32, 2048]) on the benchmark's clock: the persistent launch, its graph
    replay, and the loop of per-instance launches (graph-captured too)."""
    from paper_1305_1183_amd import batched as B
    kinds, ns, al, be = B.make_instances(*WL.BATCH_COUNTS, seed=WL.BATCH_SEED)
    out = {}
    for which, name in ((0, "persistent"), (1, "loop")):
        bt = B.Batch(kinds, ns, al, be, WL.batch_opts(loop=which == 1))
        bt.fill_device(seed=WL.BATCH_SEED)
        r, w = bt.bytes()
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            reps = 5 if which == 0 else 2
            us = kf.kf_batch_time(bt.h, which, False, st.cuda_stream, 1, reps)
            kf.kf_batch_capture(bt.h, which, st.cuda_stream)
            ug = kf.kf_batch_time(bt.h, which, True, st.cuda_stream, 1, reps)
            err = kf.kf_batch_error(bt.h, st.cuda_stream)
        if err:
            raise RuntimeError("batched launch reported error bits %d" % err)
        out[name + "_us"] = round(us, 1)
        out[name + "_graph_us"] = round(ug, 1)
        out["bytes"] = r + w
        del bt
        torch.cuda.empty_cache()
    out.update(plan_loop_times(torch, kf, WL, dev, kinds, ns, al, be, reps=2))
    best = min(out["persistent_us"], out["persistent_graph_us"])
    out["gbps"] = round(out["bytes"] / best / 1e3, 1)
    out["pct_peak"] = round(out["bytes"] / best / 1e3 / HBM_PEAK_GBPS * 100, 1)
    best_loop = min(out["loop_us"], out["loop_graph_us"], out["plan_loop_us"], out["plan_loop_graph_us"])
    out["speedup_vs_best_loop"] = round(best_loop / best, 2)
    out["what"] = ("%d BiCGK + %d GEMVER, n log-uniform on [32, 2048], one persistent launch vs per-instance "
                   "launches: the library's fused plans (one runtime-shape plan per kind and size bucket) and the "
                   "batch kernel, each plain and graph-captured" % WL.BATCH_COUNTS)
    log("batched: persistent %.1f us (graph %.1f), kernel loop %.1f us, plan loop %.1f us (graph %.1f)" %
        (out["persistent_us"], out["persistent_graph_us"], out["loop_us"], out["plan_loop_us"],
         out["plan_loop_graph_us"]))
    return out


def plan_loop_times(torch, kf, WL, dev, kinds, ns, al, be, reps=3):
    """The per-instance loop of the library's own fused plans over the batch's
    instances (B.PlanLoop), timed plain and as a graph replay."""
    from paper_1305_1183_amd import batched as B
    bt = B.Batch(kinds, ns, al, be, WL.batch_opts())
    bt.fill_device(seed=WL.BATCH_SEED)
    loop = B.PlanLoop(bt)
    st = torch.cuda.Stream()
    res = {"plan_loop_launches": loop.launches()}
    with torch.cuda.stream(st):
        loop.run(st.cuda_stream)          # warm-up (and module loads)
        st.synchronize()

        def timed(fn):
            ts = []
            for _ in range(reps):
                a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a_.record(st)
                fn()
                b_.record(st)
                st.synchronize()
                ts.append(a_.elapsed_time(b_) * 1e3)
            return float(np.median(ts))
        res["plan_loop_us"] = round(timed(lambda: loop.run(st.cuda_stream)), 1)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            loop.run(st.cuda_stream)
        g.replay()
        st.synchronize()
        res["plan_loop_graph_us"] = round(timed(g.replay), 1)
    del g, loop, bt
    torch.cuda.empty_cache()
    return res


def precision_compact(args, torch, kf, S, WL, dev):
    """Reduced-precision A at n = 32768 on the benchmark's clock: fused BiCGK
    and GEMVER per storage format (FP32, BF16, FP8-E4M3 with row scales),
    time, GB/s and the relative L2 error of sampled outputs against the FP64
    oracle on the float64 A and on the dequantised A."""
    import oracle
    from oracle import quant as OQ
    from paper_1305_1183_amd import inputs as I
    n = WL.PREC_N
    rows = np.unique(np.concatenate([[0, n - 1], I.small_ints(7, 0, 24, 0, n - 1).astype(np.int64)]))
    cols = np.unique(np.concatenate([[0, n - 1], I.small_ints(7, 1, 24, 0, n - 1).astype(np.int64)]))
    e4m3 = OQ.decode_e4m3(np.arange(256, dtype=np.uint8))
    res = {}
    for name in WL.PREC_SEQ:
        keep = {"rows": rows, "cols": cols}
        stored, vecs, scal = WL.precision_inputs(name, n, WL.PREC_FORMATS, seed=4000 + WL.SEQ_INDEX[name], keep=keep)
        f = {k: v.astype(np.float64) for k, v in vecs.items()}
        for fmt in WL.PREC_FORMATS:
            st_, sc_ = stored[fmt]
            dec = {"f32": lambda a: a.astype(np.float64), "bf16": OQ.decode_bf16, "fp8": lambda a: e4m3[a]}[fmt]
            Dr = dec(st_[rows, :n]) * sc_[rows].astype(np.float64)[:, None]
            Dc = dec(st_[:, cols]) * sc_.astype(np.float64)[:, None]
            devin = {}
            for k, v in WL.precision_arrays(fmt, stored, vecs).items():
                devin[k] = torch.from_numpy(np.ascontiguousarray(v.view(np.int16) if v.dtype == np.uint16 else v)).to(dev)
            if name == "bicgk":
                q = S.bicgk_q(n, n, fmt)
            else:
                q = S.gemver_q(n, n, scal["alpha"], scal["beta"], fmt)
            prog = q.compile(mode="fused", **WL.PREC_TUNED.get((name, fmt), {})).bind(device=dev, **devin)
            outs = prog.run()
            torch.cuda.synchronize()
            # about 0.3 s of the plan before timing, as in --precision: right after
            # the input upload the first timings run up to 8% slow
            t_end = time.time() + 0.3
            while time.time() < t_end:
                prog.run()
                torch.cuda.synchronize()
            r, w = prog.bytes()
            us = prog.time(3, 10)
            row = {"us": round(us, 1), "gbps": round((r + w) / us / 1e3, 1),
                   "pct_peak": round((r + w) / us / 1e3 / HBM_PEAK_GBPS * 100, 1)}
            if name == "bicgk":
                qg, sg = outs["q"].cpu().numpy(), outs["s"].cpu().numpy()
                for key, got, deq, a64 in (("q", qg[rows], oracle.gemv(1.0, Dr, f["p"]), oracle.gemv(1.0, keep["A64_rows"], f["p"])),
                                           ("s", sg[cols], oracle.gemtv(1.0, Dc, f["r"]), oracle.gemtv(1.0, keep["A64_cols"], f["r"]))):
                    row["err_" + key] = {"vs_dequantised": float("%.3g" % WL.rel_l2(got, deq)),
                                         "vs_fp64_A": float("%.3g" % WL.rel_l2(got, a64))}
            else:
                xg = outs["x"].cpu().numpy()[cols]
                a, b = scal["alpha"], scal["beta"]
                for key, A_ in (("vs_dequantised", Dc), ("vs_fp64_A", keep["A64_cols"])):
                    Bc = oracle.ger(1.0, oracle.ger(1.0, A_, f["u1"], f["v1"][cols]), f["u2"], f["v2"][cols])
                    row.setdefault("err_x", {})[key] = float("%.3g" % WL.rel_l2(xg, oracle.gemtv(b, Bc, f["y"], 1.0, f["z"][cols])))
            res["%s/%s" % (name, fmt)] = row
            log("precision %s %s: %.1f us, %.1f GB/s" % (name, fmt, us, row["gbps"]))
            del prog, devin, outs
            torch.cuda.empty_cache()
        del stored
    res["what"] = ("n = %d, A drawn N(0, 1) in float64 and stored per format with one FP32 scale per row; fused plans "
                   "with their tuned points; errors on %d sampled rows / %d columns (GEMVER: x on the columns)"
                   % (n, len(rows), len(cols)))
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1305_1183_amd import kf
    from paper_1305_1183_amd import sequences as S
    from paper_1305_1183_amd import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    kf.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    st = stream.cuda_stream

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).uniform_(-1, 1)
        dst = torch.empty_like(src)
        for _ in range(5):
            kf.kf_util_copy(dst.data_ptr(), src.data_ptr(), src.numel() * 4, st)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "launches": 5}))
        return

    names = [s for s in args.only.split(",") if s] or list(WL.ORDER)
    n, vec = WL.SUITE_N, WL.SUITE_VEC
    if args.precision:
        precision_suite(args, torch, kf, S, WL, dev)
        return
    if args.layout:
        layout_suite(args, torch, kf, S, WL, dev)
        return
    if args.wide_rows:
        wide_rows_suite(args, torch, kf, S, WL, dev)
        return
    if args.batched:
        batched_suite(args, torch, kf, WL, dev)
        return
    if args.tune_batch_mix:
        from paper_1305_1183_amd import batched as B
        kinds, ns, al, be = B.make_instances(*WL.BATCH_COUNTS, seed=WL.BATCH_SEED)
        rows, tiles, best, hist = B.tune_mix(kinds, ns, al, be, WL.BATCH_SEED, WL.BATCH_TUNED, WL.BATCH_TILES,
                                             log=log)
        for kind, b, t, r, us in hist:
            print(json.dumps({"kind": kind, "bucket": b, "tile": t, "rows": r, "us": round(us, 1)}), flush=True)
        print(json.dumps({"batch_tuned": rows, "batch_tiles": tiles, "best_us": round(best, 1)}), flush=True)
        return
    if args.tune_batch:
        from paper_1305_1183_amd import batched as B
        rows = {0: [0] * 6, 1: [0] * 6}
        tiles = {0: [0] * 6, 1: [0] * 6}
        for kind in (0, 1):
            for bucket in range(6):
                (bt_, br_), res = B.autotune(kind, bucket, log=log)
                tiles[kind][bucket], rows[kind][bucket] = bt_, br_
                print(json.dumps({"kind": kind, "bucket": bucket, "n": B.bucket_median(bucket), "best_tile": bt_,
                                  "best_rows": br_,
                                  "candidates": [[t_, r_, round(u, 1), round(g, 1)] for t_, r_, u, g in res]}),
                      flush=True)
        print(json.dumps({"batch_tuned": rows, "batch_tiles": tiles}), flush=True)
        return
    if args.tune:
        from paper_1305_1183_amd import autotune
        for name in names:
            m, nn = (vec, vec) if name in WL.BLAS1 else (n, n)
            arrays, scal = WL.make(name, m, nn, seed=WL.seed_for(2, name))
            q = S.by_name(name, m, nn, scal)
            devin = {k: torch.from_numpy(v).to(dev) for k, v in arrays.items()}
            for mode in ("fused", "unfused"):
                # every grid point timed kernel by kernel: the best single point
                # for the whole plan (least summed time) and the best point per kernel
                kbest, per = autotune.tune_kernels(q, devin, mode=mode)
                res = sorted(((per[0][i][0], sum(r[i][1] for r in per)) for i in range(len(per[0]))),
                             key=lambda r: r[1])
                uni = q.compile(mode=mode, **res[0][0]).bind(device=dev, **devin)
                prog = q.compile(mode=mode, kernel_params=kbest).bind(device=dev, **devin)
                print(json.dumps({"seq": name, "mode": mode, "best": res[0][0],
                                  "top": [[p, round(t, 2)] for p, t in res[:6]],
                                  "worst": [res[-1][0], round(res[-1][1], 2)],
                                  "best_plan_us": round(uni.time(3, 20), 2),
                                  "kernel_params": kbest,
                                  "kernel_us": [round(min(t for _, t in r), 2) for r in per],
                                  "per_kernel_plan_us": round(prog.time(3, 20), 2)}), flush=True)
                del prog, uni
            del devin
            torch.cuda.empty_cache()
        return
    def prepare(name):
        m, nn = (vec, vec) if name in WL.BLAS1 else (n, n)
        arrays, scal = WL.make(name, m, nn, seed=WL.seed_for(2, name))
        q = S.by_name(name, m, nn, scal)
        devin = {k: torch.from_numpy(v).to(dev) for k, v in arrays.items()}
        del arrays
        fused = q.compile(mode="fused", **WL.tuned_params(name, m, nn, "fused")).bind(device=dev, **devin)
        unfused = None if args.no_unfused else q.compile(
            mode="unfused", **WL.tuned_params(name, m, nn, "unfused")).bind(device=dev, **devin)
        return q, fused, unfused, devin

    def measure(prog_tuple):
        q, fused, unfused, _ = prog_tuple
        r, w = fused.bytes()
        tf = fused.time(3, 20)
        entry = {"fused_us": round(tf, 2), "fused_bytes": r + w,
                 "fused_gbps": round((r + w) / tf / 1e3, 1),
                 "fused_pct_peak": round((r + w) / tf / 1e3 / HBM_PEAK_GBPS * 100, 1),
                 "kernels": fused.num_kernels}
        if unfused is not None:
            ru, wu = unfused.bytes()
            tu = unfused.time(3, 20)
            entry.update({"unfused_us": round(tu, 2), "unfused_bytes": ru + wu,
                          "unfused_gbps": round((ru + wu) / tu / 1e3, 1),
                          "speedup": round(tu / tf, 3), "unfused_kernels": unfused.num_kernels})
        return entry

    progs = {}
    t0 = time.time()
    for name in names:
        progs[name] = prepare(name)
        log("prepared %s (%.1f s)" % (name, time.time() - t0))

    # launch table of the fused step: every HIP launch of every plan kernel
    kernels = []
    for name in names:
        d = progs[name][1].describe()
        for k, kd in enumerate(d["kernels"]):
            for l, ld in enumerate(kd["launches"]):
                kernels.append({"seq": name, "k": k, "l": l, "name": ld["name"],
                                "bytes": ld["bytes_read"] + ld["bytes_written"],
                                "calls": [c["op"] for c in kd["calls"]], "params": kd["params"]})
    plans = [progs[k["seq"]][1].plan for k in kernels]

    def step(events=None):
        for i, kd in enumerate(kernels):
            if events is not None:
                events[i][0].record(stream)
            kf.kf_run_launch(plans[i], kd["k"], kd["l"], st)
            if events is not None:
                events[i][1].record(stream)

    # warm-up steps; the first one also times every launch to find the dominant one
    probe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in kernels]
    for w in range(max(1, args.warmup)):
        step(probe if w == 0 else None)
    torch.cuda.synchronize()
    avg_k = np.array([a.elapsed_time(b) for a, b in probe]) * 1e3  # us, one warm-up step
    dom = int(np.argmax(avg_k))
    dk = kernels[dom]

    def timed_step(ev):
        # every launch of the step, with HIP events on the stream around the dominant one only
        for i, kd in enumerate(kernels):
            if i == dom:
                ev[0].record(stream)
            kf.kf_run_launch(plans[i], kd["k"], kd["l"], st)
            if i == dom:
                ev[1].record(stream)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        timed_step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    dom_us = float(np.mean([a.elapsed_time(b) for a, b in ev])) * 1e3
    step_bytes = sum(k["bytes"] for k in kernels)
    ms_per_step = wall * 1e3 / args.steps
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    achieved = dk["bytes"] / (dom_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": WL.traffic_from_profiles(os.path.join(ROOT, "profiles"), dk["name"]),
                "kernel": "%s kernel %d launch %d (%s) %s" % (dk["seq"], dk["k"], dk["l"], "+".join(dk["calls"]), dk["name"]),
                "avg_us": round(dom_us, 2), "bytes_per_launch": dk["bytes"],
                "timing": "HIP events on the launch stream around this launch, mean over the timed steps"}
    # the same kernel in the committed rocprofv3 --kernel-trace --stats summary
    # of this command (None when the summary does not cover this kernel text)
    prof = WL.kernel_stats_from_profiles(os.path.join(ROOT, "profiles"), WL.SUITE_STATS_FILE, dk["name"])
    if prof is not None:
        prof["frac"] = round(dk["bytes"] / (prof["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)
        prof["event_vs_profile"] = round(dom_us / prof["avg_us"], 4)
    roofline["profile"] = prof

    # attainable-bandwidth references on this device, 1 GiB each, measured
    # right after the timed steps (same device state): the library's streaming
    # read and its copy in the strip kernels' layout, and the runtime's own
    # device-to-device copy (torch copy_); the dominant launch reads one matrix
    # and writes one, like a copy
    stream_ref = None
    if not args.only:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).uniform_(-1, 1)
        dst = torch.empty_like(src)
        nbytes = src.numel() * 4

        def median_us(fn, reps=10):
            for _ in range(3):
                fn()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for a_, b_ in evs:
                a_.record(stream)
                fn()
                b_.record(stream)
            torch.cuda.synchronize()
            return float(np.median([a_.elapsed_time(b_) for a_, b_ in evs])) * 1e3

        read_gbps = nbytes / median_us(lambda: kf.kf_util_stream(0, dst.data_ptr(), src.data_ptr(), nbytes, st)) / 1e3
        copy_gbps = 2 * nbytes / median_us(lambda: kf.kf_util_stream(1, dst.data_ptr(), src.data_ptr(), nbytes, st)) / 1e3
        torch_gbps = 2 * nbytes / median_us(lambda: dst.copy_(src)) / 1e3
        stream_ref = {"read_gbps": round(read_gbps, 1), "copy_gbps": round(copy_gbps, 1),
                      "torch_copy_gbps": round(torch_gbps, 1),
                      "dominant_vs_copy": round(achieved / copy_gbps, 4),
                      "what": "1 GiB of uniform[-1, 1) floats on this device, median of 10, right after the timed "
                              "steps: the library's read (kf_util_stream kind 0) and strip-layout copy (kind 1), "
                              "and torch copy_; copies count read + write bytes"}
        del src, dst

    seqs = {name: measure(progs[name]) for name in names}
    extra = {}
    if not args.only:
        # further Table 1 sequences, measured alone (not part of the step)
        del progs, plans
        torch.cuda.empty_cache()
        for name in WL.EXTRA:
            pt = prepare(name)
            extra[name] = measure(pt)
            del pt
            torch.cuda.empty_cache()

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "single-instance FP32 suite: " + ", ".join(names) +
                      " (A %d x %d row-major, vectors 2^26, uniform[-1,1), fused plans)" % (n, n),
                      "n": n, "vector_length": vec, "sequences": names},
           "pct_peak": round(value / HBM_PEAK_GBPS * 100, 2),
           "roofline": roofline,
           "sequences": seqs,
           "sequences_extra": extra,
           "launches_us_warmup_probe": {"%s/%d/%d %s" % (k["seq"], k["k"], k["l"], k["name"]): round(float(a), 2)
                                        for k, a in zip(kernels, avg_k)}}
    if stream_ref is not None:
        out["stream_reference"] = stream_ref
    if not args.only and not args.no_extra_configs:
        # the batched and reduced-precision configurations, on the same clock
        out["batched"] = batched_compact(args, torch, kf, WL, dev)
        out["precision"] = precision_compact(args, torch, kf, S, WL, dev)
    if not args.no_cpu_baseline and not args.only:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
