"""Plan-search study on random scripts (command line).

    python -m paper_1305_1183_amd.plansearch table    --out T.json
    python -m paper_1305_1183_amd.plansearch collect  --seeds 0:50 --out D0.npz
    python -m paper_1305_1183_amd.plansearch evaluate --data D*.npz --table T.json \
        --train 0:150 --eval 150:200 --out report.json --model model.npz
    python -m paper_1305_1183_amd.plansearch modes --model M.kfcm --eval 150:160 --out modes.json
    python -m paper_1305_1183_amd.plansearch combination --data D*.npz --eval 150:200 --out comb.json

`modes` runs kf_compile's learned and exhaustive modes end to end on random
scripts and times the chosen plans. `combination` (host only) compares, on the collected timings, the best
candidate with the best per-kernel combination of the candidates.

`collect` times every sampled candidate plan of each script on the GPU
(exhaustive search); `evaluate` trains the cost model on the training scripts
with the library's GPU kernels, then ranks the candidates of the evaluation
scripts with the additive predictor and with the model, and reports the rank
of the true best plan, the regret of the chosen plan and the search time
against exhaustive timing.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import shutil
import sys
import tempfile
import time

import numpy as np


def _range(s):
    a, b = s.split(":")
    return list(range(int(a), int(b)))


def cmd_table(a):
    from . import search as SE
    entries = SE.measure_routine_table(reps=a.reps)
    json.dump({"entries": [[c, list(e), r, u, x] for c, e, r, u, x in entries],
               "note": "[class (0 BLAS-1, 1 BLAS-2 strips, 2 BLAS-2 row-resident), environment, routine, "
                       "us per matrix element / vector entry / launch (FINISH), extra LDS KiB]; probes on "
                       "8192x8192 and 2^24"},
              open(a.out, "w"), indent=0)
    print("routine table: %d entries -> %s" % (len(entries), a.out), flush=True)


def cmd_collect(a):
    from . import search as SE
    d = SE.collect(_range(a.seeds), max_cands=a.max_cands, cache_dir=a.cache, workers=a.workers, reps=a.reps,
                   log=lambda s: print(s, flush=True),
                   checkpoint=lambda part: np.savez_compressed(a.out, **part), grid=a.grid)
    np.savez_compressed(a.out, **d)
    print("saved %d candidate timings, %d kernel timings, %d unique kernels -> %s" %
          (len(d["plan_us"]), len(d["kern_us"]), len(d["uk_seed"]), a.out), flush=True)


def cmd_evaluate(a):
    import torch
    from . import kf
    from . import randscript as R
    from . import search as SE
    from .costmodel import CostModel

    files = sorted(sum([glob.glob(p) for p in a.data], []))
    data = SE.merge([dict(np.load(f, allow_pickle=False)) for f in files])
    train, evals = set(_range(a.train)), set(_range(a.eval))
    have = set(int(s) for s in data["script_seed"])
    train, evals = sorted(train & have), sorted(evals & have)
    if a.model_in:
        # a model trained earlier (its launch term stored with it); no training scripts needed
        cm = CostModel.load(a.model_in)
        X, y, hist, train_s = np.zeros((0, kf.FEATURE_DIM)), np.zeros(0), [float("nan")], 0.0
        c_launch = float(cm.state()[4])
        print("model %s (launch term %.3f us)" % (a.model_in, c_launch), flush=True)
    else:
        X, y = SE.kernel_training_set(data, train)
        print("training on %d kernel samples from %d scripts (%d plan timings in all)" %
              (len(y), len(train), len(data["plan_us"])), flush=True)
        t0 = time.perf_counter()
        cm = CostModel(seed=a.seed)
        hist = cm.fit(X, y, epochs=a.epochs, batch=256, lr=a.lr, seed=a.seed, verbose=True)
        train_s = time.perf_counter() - t0
        kpred = np.exp(cm.predict_log(data["uk_feat"]))[data["kern_uk"]]
        c_launch = SE.fit_launch_term(data, train, kpred)
        cm.set_launch_us(c_launch)            # the per-launch term travels with the model
    if a.model and not a.model_in:
        cm.save(a.model)
        if a.model.endswith(".npz"):
            cm.save(a.model[:-4] + ".kfcm")
    table = None
    if a.table:
        T = json.load(open(a.table))
        entries = T["entries"]
        if a.strip_table:
            # the additive predictor without the row-resident environment and the
            # extra-LDS axis: row-resident kernels are then priced with the first
            # strip environment's routines
            entries = [e for e in entries if e[0] != 2 and (len(e) < 5 or e[4] == 0)]
        table = kf.routine_table([(e[0], tuple(e[1])) + tuple(e[2:]) for e in entries])
    per, summary = [], {}
    for seed in evals:
        m = np.where(data["cand_seed"] == seed)[0]
        true = data["plan_us"][m]
        idx = data["cand_idx"][m]
        walls = data["cand_wall"][m]
        srow = int(np.where(data["script_seed"] == seed)[0][0])
        rs = R.random_script(seed)
        cands = kf.Candidates(rs.script, 64, SE.grid_points())
        # learned ranking: features + model (timed as the search would run it)
        t1 = time.perf_counter()
        feats = []
        for i in idx:
            p = cands.compile(int(i), kf.KF_COMPILE_CODEGEN_ONLY)
            f = kf.kf_plan_features(p)
            feats.append(f)
            kf.kf_plan_destroy(p)
        t_feat = time.perf_counter() - t1
        t1 = time.perf_counter()
        learned = cm.predict_plan_us(feats)    # the model's launch term included (set above)
        t_pred = time.perf_counter() - t1
        row = {"seed": seed, "script": rs.describe(), "candidates": int(len(m)),
               "best_us": float(true.min()), "learned": SE.rank_metrics(true, learned)}
        if table is not None:
            t1 = time.perf_counter()
            add_all = cands.predict_additive(table)
            t_add = time.perf_counter() - t1
            additive = add_all[idx]
            row["additive"] = SE.rank_metrics(true, additive)
            # the additive search: predict every candidate, compile and time the first
            j = int(np.argsort(additive, kind="stable")[0])
            tmp = tempfile.mkdtemp(prefix="kfeval")
            old = os.environ.get("KF_CACHE_DIR")
            os.environ["KF_CACHE_DIR"] = tmp
            t1 = time.perf_counter()
            cands.precompile([int(idx[j])])
            t_comp = time.perf_counter() - t1
            if old is None:
                del os.environ["KF_CACHE_DIR"]
            else:
                os.environ["KF_CACHE_DIR"] = old
            shutil.rmtree(tmp, ignore_errors=True)
            row["additive_search_s"] = t_add + t_comp + float(walls[j])
        # search time: exhaustive vs learned top-k (compile measured in a fresh cache)
        exh = float(data["script_codegen_s"][srow] + data["script_compile_s"][srow] + data["script_load_s"][srow]
                    + walls.sum())
        row["exhaustive_search_s"] = exh
        for k in a.topk:
            order = np.argsort(learned, kind="stable")[:k]
            tmp = tempfile.mkdtemp(prefix="kfeval")
            old = os.environ.get("KF_CACHE_DIR")
            os.environ["KF_CACHE_DIR"] = tmp
            t1 = time.perf_counter()
            cands.precompile([int(idx[j]) for j in order])
            t_comp = time.perf_counter() - t1
            if old is None:
                del os.environ["KF_CACHE_DIR"]
            else:
                os.environ["KF_CACHE_DIR"] = old
            shutil.rmtree(tmp, ignore_errors=True)
            tl = t_feat + t_pred + t_comp + float(walls[order].sum())
            row["learned_top%d_search_s" % k] = tl
            row["learned_top%d_regret" % k] = float(true[order].min() / true.min() - 1.0)
        per.append(row)
        print(json.dumps(row), flush=True)
        kf.kf_jit_release()

    def agg(key, sub):
        v = [r[key][sub] for r in per if key in r]
        return v

    for meth in ("learned", "additive"):
        if not per or meth not in per[0]:
            continue
        regret = np.array(agg(meth, "regret_top1"))
        summary[meth] = {
            "mean_regret_top1": float(regret.mean()), "median_regret_top1": float(np.median(regret)),
            "frac_within_5pct": float(np.mean(regret <= 0.05)),
            "mean_first_pct_of_best": float(np.mean(agg(meth, "first_pct_of_best"))),
            "median_rank_of_best": float(np.median(agg(meth, "rank_of_best"))),
            "mean_regret_top3": float(np.mean(agg(meth, "regret_top3")))}
    exh = np.array([r["exhaustive_search_s"] for r in per])
    if per and "additive_search_s" in per[0]:
        at = np.array([r["additive_search_s"] for r in per])
        summary["additive"].update({"total_search_s": float(at.sum()), "search_time_ratio": float(exh.sum() / at.sum())})
    for k in a.topk:
        lt = np.array([r["learned_top%d_search_s" % k] for r in per])
        rg = np.array([r["learned_top%d_regret" % k] for r in per])
        summary["learned_top%d" % k] = {"total_search_s": float(lt.sum()), "exhaustive_total_s": float(exh.sum()),
                                        "search_time_ratio": float(exh.sum() / lt.sum()),
                                        "mean_regret": float(rg.mean()), "frac_within_5pct": float(np.mean(rg <= 0.05)),
                                        "plan_time_total_ratio_vs_best": float(
                                            np.sum([r["best_us"] * (1 + g) for r, g in zip(per, rg)]) /
                                            np.sum([r["best_us"] for r in per]))}
    report = {"train_scripts": len(train), "eval_scripts": len(evals), "kernel_samples": int(len(y)),
              "plan_timings": int(len(data["plan_us"])), "train_seconds": train_s,
              "final_train_loss": hist[-1], "launch_term_us": c_launch, "summary": summary, "per_script": per}
    json.dump(report, open(a.out, "w"), indent=1)
    print(json.dumps(summary, indent=1), flush=True)


def cmd_modes(a):
    """kf_compile's ranking modes end to end on random scripts (GPU): the
    learned mode (top-1 and timed top-k) and, given a routine table, the
    additive mode against the exhaustive mode, all combining kernel
    implementations; plan time and search time of each."""
    import torch
    from . import kf
    from . import randscript as R
    from . import search as SE
    from .costmodel import CostModel

    cm = CostModel.load(a.model)
    cm.predict_log(np.zeros((1, kf.FEATURE_DIM), np.float32))   # device state of the model set up once
    table = None
    if a.table:
        T = json.load(open(a.table))
        table = kf.routine_table([(e[0], tuple(e[1])) + tuple(e[2:]) for e in T["entries"]])
    st = torch.cuda.current_stream().cuda_stream
    per = []
    ranked = ["learned_top1", "learned_top%d" % a.topk] + (["additive"] if table is not None else [])
    for seed in _range(a.eval):
        rs = R.random_script(seed)
        inst = SE.Instance(rs)
        bind = {v: t.data_ptr() for v, t in inst.t.items()}
        row = {"seed": seed, "script": rs.describe()}
        modes = [("learned_top1", dict(mode="learned", model=cm.handle, top_k=0)),
                 ("learned_top%d" % a.topk, dict(mode="learned", model=cm.handle, top_k=a.topk, bind=bind))]
        if table is not None:
            modes.append(("additive", dict(mode="additive", table=table)))
        modes.append(("exhaustive", dict(mode="exhaustive", bind=bind)))
        for key, kw in modes:
            # every mode compiles from scratch: its own empty disk cache, no loaded modules
            os.environ["KF_CACHE_DIR"] = os.path.join(a.cache, "s%d_%s" % (seed, key))
            os.makedirs(os.environ["KF_CACHE_DIR"], exist_ok=True)
            kf.kf_jit_release()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = kf.kf_compile(rs.script, stream=st, max_partitions=a.max_partitions, **kw)
            search_s = time.perf_counter() - t0
            inst.bind(plan)
            us = kf.kf_time_plan(plan, st, 3, 20)
            row[key] = {"plan_us": us, "search_s": search_s, "kernels": kf.kf_plan_num_kernels(plan)}
            kf.kf_plan_destroy(plan)
        for key in ranked:
            row[key]["regret"] = row[key]["plan_us"] / row["exhaustive"]["plan_us"] - 1.0
        per.append(row)
        print("script %d: learned %.1f us (%.2f s), top-%d %.1f us (%.2f s), exhaustive %.1f us (%.2f s)" %
              (seed, row["learned_top1"]["plan_us"], row["learned_top1"]["search_s"], a.topk,
               row["learned_top%d" % a.topk]["plan_us"], row["learned_top%d" % a.topk]["search_s"],
               row["exhaustive"]["plan_us"], row["exhaustive"]["search_s"]), flush=True)
        del inst
        torch.cuda.empty_cache()
        kf.kf_jit_release()
    summary = {}
    exh_s = sum(r["exhaustive"]["search_s"] for r in per)
    for key in ranked:
        rg = np.array([r[key]["regret"] for r in per])
        summary[key] = {"mean_regret": float(rg.mean()), "median_regret": float(np.median(rg)),
                        "frac_within_5pct": float(np.mean(rg <= 0.05)),
                        "search_time_ratio": exh_s / sum(r[key]["search_s"] for r in per),
                        "plan_time_total_ratio_vs_exhaustive": float(sum(r[key]["plan_us"] for r in per) /
                                                                      sum(r["exhaustive"]["plan_us"] for r in per))}
    json.dump({"what": "kf_compile modes on random scripts: plan time (median of 20 runs) and search time "
                       "(wall clock of kf_compile, compilation included)", "max_partitions": a.max_partitions,
               "summary": summary, "per_script": per}, open(a.out, "w"), indent=1)
    print(json.dumps(summary, indent=1), flush=True)


def cmd_combination(a):
    from . import search as SE
    files = sorted(sum([glob.glob(p) for p in a.data], []))
    data = SE.merge([dict(np.load(f, allow_pickle=False)) for f in files])
    c_launch = SE.fit_launch_term(data, _range(a.train))
    per = SE.combination_gain(data, _range(a.eval), c_launch, log=lambda s: print(s, flush=True))
    g = np.array([r["gain"] for r in per])
    summary = {"scripts": len(per), "launch_term_us": c_launch, "mean_gain": float(g.mean()),
               "median_gain": float(np.median(g)), "max_gain": float(g.max()),
               "frac_gain_above_2pct": float(np.mean(g > 0.02))}
    json.dump({"what": "best per-kernel combination of the measured candidates against the best candidate, "
                       "both as summed measured kernel times plus the fitted launch term",
               "summary": summary, "per_script": per}, open(a.out, "w"), indent=1)
    print(json.dumps(summary, indent=1), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("table")
    t.add_argument("--out", required=True)
    t.add_argument("--reps", type=int, default=10)
    c = sub.add_parser("collect")
    c.add_argument("--seeds", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--max-cands", type=int, default=512)
    c.add_argument("--workers", type=int, default=14)
    c.add_argument("--reps", type=int, default=3)
    c.add_argument("--cache", default="/tmp/kf_cache")
    c.add_argument("--grid", choices=("study", "default"), default="study",
                   help="parameter points: the study's grid or the library's default candidate grid")
    e = sub.add_parser("evaluate")
    e.add_argument("--data", nargs="+", required=True)
    e.add_argument("--table", default="")
    e.add_argument("--strip-table", action="store_true",
                   help="keep only the table's strip and BLAS-1 environments without extra LDS (ablation)")
    e.add_argument("--train", default="0:150")
    e.add_argument("--eval", default="150:200")
    e.add_argument("--out", required=True)
    e.add_argument("--model", default="")
    e.add_argument("--model-in", default="", help="use this trained model (.kfcm or .npz) instead of training one")
    e.add_argument("--epochs", type=int, default=150)
    e.add_argument("--lr", type=float, default=1e-3)
    e.add_argument("--seed", type=int, default=0)
    e.add_argument("--topk", type=lambda s: [int(x) for x in s.split(",")], default=[1, 3])
    md = sub.add_parser("modes")
    md.add_argument("--eval", default="150:160")
    md.add_argument("--model", required=True)
    md.add_argument("--table", default="", help="routine table: also run the additive mode")
    md.add_argument("--out", required=True)
    md.add_argument("--topk", type=int, default=3)
    md.add_argument("--max-partitions", type=int, default=16)
    md.add_argument("--cache", default="/tmp/kf_cache_modes", help="a fresh directory per script and mode")
    cb = sub.add_parser("combination")
    cb.add_argument("--data", nargs="+", required=True)
    cb.add_argument("--train", default="0:150")
    cb.add_argument("--eval", default="150:200")
    cb.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    {"table": cmd_table, "collect": cmd_collect, "evaluate": cmd_evaluate, "modes": cmd_modes,
     "combination": cmd_combination}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
