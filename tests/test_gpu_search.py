"""Plan search on the GPU: routine probes, a plan chosen by the additive
predictor computes the right result, and a small collect/train/rank round trip."""
import json

import numpy as np
import pytest
import torch

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import search as SE
from paper_1305_1183_amd import workloads as WL
from tests import seqcheck as SC

pytestmark = pytest.mark.gpu


LDS = (0, 64)


@pytest.fixture(scope="module")
def table():
    return SE.measure_routine_table(mat_shape=(2048, 2048), vec_n=1 << 20, reps=3, lds_axis=LDS)


def test_routine_table_is_positive_and_plausible(table):
    # every BLAS-2 environment (strips and the row-resident one) at each extra-LDS
    # amount, one FINISH per environment, and the BLAS-1 routines
    assert len(table) == len(SE.MAT_ENVS) * (5 * len(LDS) + 1) + len(SE.VEC_ENVS) * 6
    for cls, env, r, us, x in table:
        assert us > 0 and np.isfinite(us), (cls, env, r, x)
    assert sum(1 for e in table if e[0] == 2) == 5 * len(LDS) + 1
    # the matrix-load probe streams at more than 0.1 TB/s even at this small shape
    for cls in (1, 2):
        for c, e, r, us, x in table:
            if c == cls and r == 0:
                assert 4.0 / us / 1e6 > 0.1, (c, e, x)


@pytest.mark.parametrize("name", ["gemver", "bicgk", "gesummv", "axpydot"])
def test_additive_plan_is_correct(table, name):
    m, n = (1000, 1001) if name != "axpydot" else (100003, 100003)
    arrays, scal = WL.make(name, m, n, seed=21)
    q = SC.build_sequence(name, m, n, scal)
    T = kf.routine_table(table)
    plan = kf.kf_compile(q.script, mode="additive", table=T)
    from paper_1305_1183_amd.sequences import Program
    prog = Program(q, plan)
    prog.bind(**{k: torch.from_numpy(v).cuda() for k, v in arrays.items()})
    outs = prog.run()
    torch.cuda.synchronize()
    SC.check_against_oracle(name, m, n, {k: v.cpu().numpy() for k, v in outs.items()},
                            SC.oracle_outputs(name, arrays, scal, n))


def test_collect_train_rank_roundtrip(tmp_path):
    from paper_1305_1183_amd.costmodel import CostModel
    d = SE.collect([3, 11], max_cands=24, cache_dir=str(tmp_path / "cache"), workers=2, reps=2,
                   log=lambda s: print(s, flush=True))
    assert len(d["plan_us"]) >= 30 and np.all(d["plan_us"] > 0)
    X, y = SE.kernel_training_set(d, [3])
    cm = CostModel(seed=0)
    hist = cm.fit(X, y, epochs=40, batch=64, lr=2e-3)
    assert hist[-1] < hist[0]
    m = d["cand_seed"] == 11
    pred = np.exp(cm.predict_log(d["uk_feat"]))
    ksum = np.zeros(len(d["cand_seed"]))
    np.add.at(ksum, d["kern_cand"], pred[d["kern_uk"]])
    r = SE.rank_metrics(d["plan_us"][m], ksum[m])
    assert 1 <= r["rank_of_best"] <= int(m.sum())
    assert r["regret_top1"] >= 0
