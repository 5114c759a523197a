"""Host-side plan search: the additive predictor against a hand computation
(Section 4.2: max of summed transfer and compute routine times), candidate
sets, random scripts and the ranking metrics."""
import numpy as np
import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import randscript as R
from paper_1305_1183_amd import search as SE
from paper_1305_1183_amd import sequences as S

ENV = (1, 4, 4, 256)
PAR = dict(mat_k=1, mat_waves=4, mat_group=4, mat_rows=256)


def table(load=1e-6, store=2e-6, gemv=3e-7, gemtv=5e-7, ger=7e-7, fin=4.0, vec=(1e-5, 2e-5, 1e-7, 2e-7, 3e-7, 5.0)):
    e = [(1, ENV, 0, load), (1, ENV, 1, store), (1, ENV, 2, gemv), (1, ENV, 3, gemtv), (1, ENV, 4, ger),
         (1, ENV, 10, fin)]
    venv = (4, 256, 64, 0)
    for r, u in zip((5, 6, 7, 8, 9, 10), vec):
        e.append((0, venv, r, u))
    return kf.routine_table(e)


def test_additive_bicgk_by_hand():
    m, n = 3000, 1000
    q = S.bicgk(m, n)
    T = table()
    pf = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_CODEGEN_ONLY, **PAR)
    pu = kf.kf_compile(q.script, mode="unfused", flags=kf.KF_COMPILE_CODEGEN_ONLY, **PAR)
    # fused: loads A, p, r; the finishing pass stores q and s; compute gemv + gemtv
    tt = (m * n + n + m) * 1e-6 + (m + n) * 2e-6
    tc = m * n * (3e-7 + 5e-7)
    assert abs(kf.kf_predict_additive(pf, T) - (max(tt, tc) + 4.0)) < 1e-3
    # unfused: A is loaded twice
    t1 = max((m * n + n) * 1e-6 + m * 2e-6, m * n * 3e-7) + 4.0
    t2 = max((m * n + m) * 1e-6 + n * 2e-6, m * n * 5e-7) + 4.0
    assert abs(kf.kf_predict_additive(pu, T) - (t1 + t2)) < 1e-3
    # compute-bound table: max picks the compute sum
    T2 = table(gemv=1e-3, gemtv=2e-3)
    assert abs(kf.kf_predict_additive(pf, T2) - (m * n * 3e-3 + 4.0)) < 1.0


def test_additive_vec_and_missing_env():
    n = 1 << 16
    q = S.waxpby(n, 1.5, 0.5)
    T = table()
    p = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_CODEGEN_ONLY, vec_unroll=4, vec_threads=256,
                      vec_grid=64)
    # loads x, y; stores w; computes scal + axpy; one launch (no finish)
    want = max(2 * n * 1e-5 + n * 2e-5, n * (1e-7 + 2e-7))
    assert abs(kf.kf_predict_additive(p, T) - want) < 1e-3
    p2 = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_CODEGEN_ONLY, vec_unroll=2, vec_threads=256,
                       vec_grid=64)
    with pytest.raises(kf.KFError) as e:
        kf.kf_predict_additive(p2, T)
    assert e.value.name == "KF_ERR_UNSUPPORTED"


def test_additive_mode_prefers_fusion_when_transfers_dominate():
    q = S.gemver(2048, 2048, 1.5, 0.5)
    p = kf.kf_compile(q.script, mode="additive", table=table(), flags=kf.KF_COMPILE_CODEGEN_ONLY)
    assert kf.kf_plan_num_kernels(p) == 2          # ger+ger+gemtv, gemv


def test_candidates_dedupe_and_params():
    q = S.axpydot(1 << 12, 1.5)                     # tiny: every grid point gives the same grid
    c = kf.Candidates(q.script, 64, SE.grid_points())
    assert len(c) <= 2 * len(SE.VEC_ENVS)
    for i in range(len(c)):
        assert c.params(i)["mat_k"] == 0            # no BLAS-2 kernel: BLAS-2 parameters cleared
    q2 = S.gemver(4096, 4096, 1.5, 0.5)
    c2 = kf.Candidates(q2.script, 64, SE.grid_points())
    assert len(c2) == 4 * len(SE.MAT_ENVS)          # 4 partitions x BLAS-2 points
    parts = {tuple(c2.partition(i)) for i in range(len(c2))}
    assert parts == {tuple(p) for p in kf.kf_enumerate(q2.script)}


def test_random_scripts_deterministic_and_compilable():
    a = R.random_script(5)
    b = R.random_script(5)
    assert a.calls == b.calls and a.n_mat == b.n_mat and a.n_vec == b.n_vec
    assert 8 <= len(a.calls) <= 12
    c = kf.Candidates(a.script, 16, SE.grid_points())
    for i in range(0, len(c), max(1, len(c) // 8)):
        p = c.compile(i, kf.KF_COMPILE_CODEGEN_ONLY)
        f = kf.kf_plan_features(p)
        assert f.shape == (kf.kf_plan_num_kernels(p), kf.FEATURE_DIM) and np.all(np.isfinite(f))
        kf.kf_plan_destroy(p)
    assert SE.sample_candidates(500, 128, 3) == SE.sample_candidates(500, 128, 3)
    assert SE.sample_candidates(500, 128, 3)[0] == 0 and len(SE.sample_candidates(500, 128, 3)) == 128


def test_rank_metrics():
    true = np.array([10.0, 5.0, 7.0, 5.004])
    m = SE.rank_metrics(true, np.array([1.0, 3.0, 2.0, 4.0]))
    assert m["rank_of_best"] == 3 and abs(m["regret_top1"] - 1.0) < 1e-12
    assert abs(m["first_pct_of_best"] - 50.0) < 1e-9 and m["regret_top3"] == 0.0
    m2 = SE.rank_metrics(true, np.array([5.0, 4.0, 3.0, 1.0]))   # 5.004 is within 0.1% of 5
    assert m2["rank_of_best"] == 1


def test_features_distinguish_fusion():
    q = S.bicgk(4096, 4096)
    pf = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_CODEGEN_ONLY)
    pu = kf.kf_compile(q.script, mode="unfused", flags=kf.KF_COMPILE_CODEGEN_ONLY)
    ff, fu = kf.kf_plan_features(pf), kf.kf_plan_features(pu)
    assert ff.shape[0] == 1 and fu.shape[0] == 2
    assert ff[0, 5] > 20 and fu[0, 5] == 0      # bytes saved: log2(4 n^2) vs none
    assert ff[0, 9] == 1 and ff[0, 10] == 1      # one gemv and one gemtv


def test_combination_gain_by_hand():
    """Two measured candidates of one partition: every kernel takes its faster
    timing; a third candidate of another partition competes as a whole."""
    seed = 3
    rs = R.random_script(seed)
    c = kf.Candidates(rs.script, 64, SE.grid_points())
    by_part = {}
    for i in range(len(c)):
        by_part.setdefault(tuple(c.partition(i)), []).append(i)
    part, idx = next((p, v) for p, v in by_part.items() if len(v) >= 2 and max(p) >= 1)
    other = next(v[0] for p, v in by_part.items() if p != part)
    nk = max(part) + 1
    k_a = [10.0] * nk
    k_b = [10.0] * nk
    k_a[0], k_b[0] = 4.0, 9.0
    k_a[1], k_b[1] = 8.0, 3.0
    k_o = [1000.0]
    cand_idx = [idx[0], idx[1], other]
    kern_cand, kern_us = [], []
    for ci, ks in enumerate((k_a, k_b, k_o)):
        kern_cand += [ci] * len(ks)
        kern_us += ks
    data = {"cand_seed": np.array([seed] * 3), "cand_idx": np.array(cand_idx),
            "cand_launches": np.array([nk, nk, 1]), "plan_us": np.array([sum(k_a), sum(k_b), 1000.0]),
            "kern_cand": np.array(kern_cand), "kern_us": np.array(kern_us)}
    r = SE.combination_gain(data, [seed], c_launch=0.5)[0]
    uniform = min(sum(k_a), sum(k_b)) + 0.5 * nk
    comb = 4.0 + 3.0 + 10.0 * (nk - 2) + 0.5 * nk
    assert r["partitions"] == 2 and r["candidates"] == 3
    assert abs(r["uniform_est_us"] - uniform) < 1e-9 and abs(r["combination_est_us"] - comb) < 1e-9
    assert abs(r["gain"] - (1 - comb / uniform)) < 1e-12


def test_additive_prices_row_resident_kernels_in_their_own_environment():
    """A kernel on the row-resident schedule takes the class 2 (row-resident)
    entries, not a strip environment's, and the extra-LDS amount nearest to its
    own LDS use (single-pass ATAX at n = 16384 stages x in 64 KiB of LDS)."""
    import json
    n = 16384
    q = S.atax(n, n)
    p = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_CODEGEN_ONLY)
    lds = json.loads(kf.kf_plan_describe(p))["kernels"][0]["lds_bytes"]
    assert 64 * 1024 <= lds < 80 * 1024
    env = (0, 0, 0, 0)

    def rowres(load, x):
        return [(2, env, 0, load, x), (2, env, 1, 5e-6, x), (2, env, 2, 1e-9, x), (2, env, 3, 2e-9, x),
                (2, env, 4, 3e-9, x)]
    strip = [(1, ENV, r, 1.0, 0) for r in range(5)] + [(1, ENV, 10, 100.0, 0)]
    T = kf.routine_table(strip + rowres(1e-6, 0) + rowres(2e-6, 64) + [(2, env, 10, 3.0, 0)])
    tt = (n * n + n) * 2e-6 + n * 5e-6          # A and x at the 64 KiB entries; y stored by the finishing launch
    tc = n * n * (1e-9 + 2e-9)
    assert abs(kf.kf_predict_additive(p, T) - (max(tt, tc) + 3.0)) < 1e-2 * max(tt, tc)
    # a table without row-resident entries falls back to its first strip environment
    T1 = kf.routine_table(strip)
    assert kf.kf_predict_additive(p, T1) > 1e6
    kf.kf_plan_destroy(p)


def test_additive_mode_grid_takes_row_resident_environments():
    """KF_MODE_ADDITIVE without a grid crosses every environment of the table;
    a class 2 environment becomes the row-resident schedule."""
    q = S.gesummv(2048, 2048, 1.5, 0.5)
    env = (0, 0, 0, 0)
    strip = [(1, ENV, r, 1e-3, 0) for r in range(5)] + [(1, ENV, 10, 4.0, 0)]
    rowres = [(2, env, r, 1e-9, 0) for r in range(5)] + [(2, env, 10, 4.0, 0)]
    vec = [(0, (4, 256, 64, 0), r, 1e-7, 0) for r in range(5, 11)]
    p = kf.kf_compile(q.script, mode="additive", table=kf.routine_table(strip + rowres + vec),
                      flags=kf.KF_COMPILE_CODEGEN_ONLY)
    assert kf.kf_plan_kernel_params(p, 0).get("mat_sched") == 1
    kf.kf_plan_destroy(p)


def test_additive_ranks_implementations_over_the_register_budget_last():
    """Section 4.2 prunes implementations that need more on-chip memory than
    another implementation of the same fusion. A row-resident kernel the
    generator marks over its register budget (column-major GEMVER at 32768
    columns) gets 1e9 us added; the same fusion within budget (16384 columns)
    and single-pass ATAX at 32768 columns do not."""
    import json
    env = (0, 0, 0, 0)
    T = kf.routine_table([(2, env, r, 1e-9, 0) for r in range(5)] + [(2, env, 10, 3.0, 0)])

    def plan(name, m, n, layout):
        q = S.by_name(name, m, n, {"alpha": 1.5, "beta": 0.75}, layout=layout)   # keeps the script alive
        p = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_CODEGEN_ONLY)
        (k,) = json.loads(kf.kf_plan_describe(p))["kernels"]
        return p, k["params"]

    p, prm = plan("gemver", 32768, 256, kf.KF_COL_MAJOR)
    assert prm["over_register_budget"] and prm["register_estimate"] > 96
    assert kf.kf_predict_additive(p, T) >= 1e9
    kf.kf_plan_destroy(p)
    for args in (("gemver", 16384, 256, kf.KF_COL_MAJOR), ("atax", 256, 32768, kf.KF_ROW_MAJOR)):
        p, prm = plan(*args)
        assert not prm["over_register_budget"]
        assert kf.kf_predict_additive(p, T) < 1e6
        kf.kf_plan_destroy(p)


def test_additive_mode_avoids_a_kernel_over_the_register_budget():
    """KF_MODE_ADDITIVE with row-resident routines far cheaper than the strip
    ones: column-major GEMVER at 32768 columns still does not take its
    one-kernel plan (a row-resident kernel over the register budget) but a
    plan whose kernels are all within budget; at 16384 columns the one-kernel
    plan is within budget and is taken."""
    import json
    env = (0, 0, 0, 0)
    strip = [(1, ENV, r, 1e-3, 0) for r in range(5)] + [(1, ENV, 10, 4.0, 0)]
    rowres = [(2, env, r, 1e-9, 0) for r in range(5)] + [(2, env, 10, 4.0, 0)]
    vec = [(0, (4, 256, 64, 0), r, 1e-7, 0) for r in range(5, 11)]
    T = kf.routine_table(strip + rowres + vec)
    for m, one_kernel in ((32768, False), (16384, True)):
        q = S.by_name("gemver", m, 256, {"alpha": 1.5, "beta": 0.75}, layout=kf.KF_COL_MAJOR)
        p = kf.kf_compile(q.script, mode="additive", table=T, flags=kf.KF_COMPILE_CODEGEN_ONLY)
        ks = json.loads(kf.kf_plan_describe(p))["kernels"]
        assert all(not k["params"].get("over_register_budget", False) for k in ks), ks
        assert (len(ks) == 1) == one_kernel, [k["params"] for k in ks]
        kf.kf_plan_destroy(p)
