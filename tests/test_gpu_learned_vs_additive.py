"""What the learned cost model gains over the paper's additive predictor.

The MLP is trained on the GPU by the library's own kernels on measured
kernel times of 70 random scripts (a stored subset of the plan-search study),
then both predictors rank the measured candidate plans of 20 other scripts.
The regret of a predictor is how much slower its top-ranked plan ran than the
best measured plan; the learned ranking must be better in mean and median."""
import json
import os

import numpy as np
import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import randscript as R
from paper_1305_1183_amd import search as SE

pytestmark = pytest.mark.gpu
DATA = os.path.join(os.path.dirname(kf.__file__), "data")


def test_learned_model_beats_additive_predictor():
    from paper_1305_1183_amd.costmodel import CostModel
    d = np.load(os.path.join(DATA, "plansearch_subset.npz"), allow_pickle=False)
    cm = CostModel(seed=0)
    hist = cm.fit(d["X"], d["y"], epochs=150, batch=256, lr=1e-3, seed=0)
    cm.set_launch_us(float(d["launch_us"]))   # plan time = sum of kernels + launch term per launch
    assert hist[-1] < hist[0]
    T = json.load(open(os.path.join(DATA, "routine_table.json")))
    table = kf.routine_table([(e[0], tuple(e[1])) + tuple(e[2:]) for e in T["entries"]])
    reg_l, reg_a = [], []
    for seed in np.unique(d["cand_seed"]):
        m = d["cand_seed"] == seed
        idx, true = d["cand_idx"][m], d["plan_us"][m].astype(np.float64)
        rs = R.random_script(int(seed))
        cands = kf.Candidates(rs.script, 64, SE.grid_points())
        feats = []
        for i in idx:
            p = cands.compile(int(i), kf.KF_COMPILE_CODEGEN_ONLY)
            f = kf.kf_plan_features(p)
            feats.append(f)
            kf.kf_plan_destroy(p)
        learned = cm.predict_plan_us(feats)
        additive = cands.predict_additive(table)[idx]
        reg_l.append(SE.rank_metrics(true, learned)["regret_top1"])
        reg_a.append(SE.rank_metrics(true, additive)["regret_top1"])
        print("script %d: learned regret %.3f, additive regret %.3f" % (seed, reg_l[-1], reg_a[-1]), flush=True)
    print("mean regret: learned %.3f, additive %.3f; median: learned %.3f, additive %.3f" %
          (np.mean(reg_l), np.mean(reg_a), np.median(reg_l), np.median(reg_a)), flush=True)
    assert np.mean(reg_l) < np.mean(reg_a)
    assert np.median(reg_l) < np.median(reg_a)
    assert np.mean(reg_l) <= 0.06
