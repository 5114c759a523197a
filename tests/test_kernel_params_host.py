"""Per-kernel implementation parameters (Section 4.2: a plan is a combination
of fusion implementations, so each kernel may use its own block size and
serial iterations) and the additive mode's choice of the cheapest
combination, checked against brute force over every partition and every
assignment of parameter points to its kernels."""
import itertools
import json

import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S

CG = kf.KF_COMPILE_CODEGEN_ONLY
P1 = dict(mat_k=2, mat_waves=4, mat_group=2, mat_rows=2048)
P2 = dict(mat_k=1, mat_waves=4, mat_group=2, mat_rows=1024)


def test_each_kernel_takes_its_own_parameters():
    q = S.gemver(4096, 4096, 1.5, 0.5)
    p = kf.kf_compile(q.script, mode="fused", flags=CG, kernel_params=[P1, P2])
    assert kf.kf_plan_num_kernels(p) == 2
    got = [kf.kf_plan_kernel_params(p, k) for k in range(2)]
    assert got[0] == P1 and got[1] == P2
    d = json.loads(kf.kf_plan_describe(p))
    names = [k["launches"][0]["name"] for k in d["kernels"]]
    # the same kernels as the uniform plans with each point
    u1 = kf.kf_compile(q.script, mode="fused", flags=CG, **P1)
    u2 = kf.kf_compile(q.script, mode="fused", flags=CG, **P2)
    assert names[0] == json.loads(kf.kf_plan_describe(u1))["kernels"][0]["launches"][0]["name"]
    assert names[1] == json.loads(kf.kf_plan_describe(u2))["kernels"][1]["launches"][0]["name"]
    for h in (p, u1, u2):
        kf.kf_plan_destroy(h)


def test_missing_and_zero_entries_inherit_the_plan_wide_point():
    q = S.gemver(4096, 4096, 1.5, 0.5)
    p = kf.kf_compile(q.script, mode="fused", flags=CG, kernel_params=[dict(mat_rows=2048)], **P2)
    assert kf.kf_plan_kernel_params(p, 0) == dict(P2, mat_rows=2048)
    assert kf.kf_plan_kernel_params(p, 1) == P2
    kf.kf_plan_destroy(p)
    q2 = S.waxpby(1 << 20, 1.5, 0.5)
    p2 = kf.kf_compile(q2.script, mode="fused", flags=CG, kernel_params=[dict(vec_grid=512)], vec_unroll=2)
    assert kf.kf_plan_kernel_params(p2, 0) == dict(vec_unroll=2, vec_threads=256, vec_grid=512)
    kf.kf_plan_destroy(p2)


def test_kernel_params_are_checked():
    q = S.gemver(1024, 1024, 1.5, 0.5)
    with pytest.raises(kf.KFError) as e:
        kf.kf_compile(q.script, mode="fused", flags=CG, kernel_params=[P1, P2, P1])
    assert e.value.name == "KF_ERR_ARG"
    with pytest.raises(kf.KFError) as e:
        kf.kf_compile(q.script, mode="fused", flags=CG, kernel_params=[P1, dict(mat_k=3)])
    assert e.value.name == "KF_ERR_ARG"
    with pytest.raises(kf.KFError) as e:
        kf.kf_compile(q.script, mode="fused", flags=CG, kernel_params=[dict(mat_rows=1000, mat_waves=4, mat_group=4)])
    assert e.value.name == "KF_ERR_ARG"
    with pytest.raises(TypeError):
        kf.kf_compile(q.script, mode="fused", flags=CG, kernel_params=[dict(rows=5)])
    p = kf.kf_compile(q.script, mode="fused", flags=CG)
    with pytest.raises(kf.KFError):
        kf.kf_plan_kernel_params(p, 2)
    kf.kf_plan_destroy(p)


E1, E2 = (1, 4, 4, 256), (2, 4, 2, 512)


def two_env_table():
    """E1 prices ger cheaply and gemv dearly, E2 the other way round; both
    compute-bound, so the best GEMVER plan mixes the two environments."""
    e = []
    for env, ger, gemv in ((E1, 1e-6, 4e-6), (E2, 4e-6, 1e-6)):
        e += [(1, env, 0, 1e-8), (1, env, 1, 1e-8), (1, env, 2, gemv), (1, env, 3, 2e-6), (1, env, 4, ger),
              (1, env, 10, 3.0)]
    return kf.routine_table(e)


def _env_params(env):
    return dict(mat_k=env[0], mat_waves=env[1], mat_group=env[2], mat_rows=env[3])


def test_additive_mode_picks_the_cheapest_combination():
    q = S.gemver(2048, 2048, 1.5, 0.5)
    T = two_env_table()
    best, best_at = None, None
    for part in kf.kf_enumerate(q.script):
        nk = max(part) + 1
        for envs in itertools.product((E1, E2), repeat=nk):
            p = kf.kf_compile(q.script, mode="partition", partition=part, flags=CG,
                              kernel_params=[_env_params(e) for e in envs])
            t = kf.kf_predict_additive(p, T)
            kf.kf_plan_destroy(p)
            if best is None or t < best * 0.999:
                best, best_at = t, (part, envs)
    p = kf.kf_compile(q.script, mode="additive", table=T, flags=CG)
    got = kf.kf_predict_additive(p, T)
    assert abs(got - best) <= 1e-6 * best
    part, envs = best_at
    assert kf.kf_plan_num_kernels(p) == max(part) + 1
    assert [kf.kf_plan_kernel_params(p, k) for k in range(len(envs))] == [_env_params(e) for e in envs]
    # the fused partition mixes the environments: ger kernel on E1, gemv kernel on E2
    assert envs == (E1, E2)
    # and beats every uniform candidate
    for env in (E1, E2):
        u = kf.kf_compile(q.script, mode="fused", flags=CG, **_env_params(env))
        assert got < kf.kf_predict_additive(u, T)
        kf.kf_plan_destroy(u)
    kf.kf_plan_destroy(p)


def test_mixed_classes_take_their_own_fields():
    """In a plan with BLAS-1 and BLAS-2 kernels, each kernel reads only the
    fields of its class from its entry."""
    import paper_1305_1183_amd.randscript as R
    rs = next(r for r in (R.random_script(s) for s in range(40))
              if {"dot", "gemv"} <= set(r.calls) or {"axpy", "gemv"} <= set(r.calls))
    p = kf.kf_compile(rs.script, mode="unfused", flags=CG)
    nk = kf.kf_plan_num_kernels(p)
    d = json.loads(kf.kf_plan_describe(p))
    kf.kf_plan_destroy(p)
    entry = dict(mat_k=2, mat_waves=8, mat_group=2, mat_rows=1024, vec_unroll=2, vec_threads=512, vec_grid=64)
    p = kf.kf_compile(rs.script, mode="unfused", flags=CG, kernel_params=[entry] * nk)
    for k, kd in enumerate(d["kernels"]):
        got = kf.kf_plan_kernel_params(p, k)
        if kd["class"] == "blas2":
            assert got == dict(mat_k=2, mat_waves=8, mat_group=2, mat_rows=1024), got
        else:
            assert got["vec_unroll"] == 2 and got["vec_threads"] == 512 and "mat_k" not in got, got
    kf.kf_plan_destroy(p)
