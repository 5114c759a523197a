"""Runtime-shape plans on the host: which scripts qualify, the checks of
kf_plan_set_shape and kf_bind_matrix, and that the generated kernels take
the shape as arguments (no GPU needed)."""
import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S

RS = kf.KF_COMPILE_RUNTIME_SHAPE
CG = kf.KF_COMPILE_CODEGEN_ONLY


def _plan(q, mode="fused", **kw):
    return kf.kf_compile(q.script, mode=mode, flags=RS | CG, **kw)


def test_kernels_take_the_shape_as_arguments():
    q = S.gemver(2048, 2048, 1.5, 0.5)
    p = _plan(q)
    try:
        for k in range(kf.kf_plan_num_kernels(p)):
            src = kf.kf_plan_source(p, k)
            assert "long M_" in src and "long N_" in src and "constexpr long M =" not in src
        # a plan compiled without the flag bakes the shape in
        p2 = kf.kf_compile(q.script, mode="fused", flags=CG)
        assert "constexpr long M = 2048L" in kf.kf_plan_source(p2, 0)
        kf.kf_plan_destroy(p2)
    finally:
        kf.kf_plan_destroy(p)


@pytest.mark.parametrize("make,why", [
    (lambda: S.atax(1024, 1024), "whole rows"),            # the fused ATAX kernel needs the row-resident schedule
    (lambda: S.axpydot(1 << 16, 1.5), "BLAS-2"),
])
def test_unsupported_scripts(make, why):
    with pytest.raises(kf.KFError) as e:
        _plan(make())
    assert "KF_ERR_UNSUPPORTED" in str(e.value) and why in str(e.value)


def test_row_resident_request_refused():
    with pytest.raises(kf.KFError) as e:
        _plan(S.bicgk(1024, 1024), mat_sched=1)
    assert "KF_ERR_UNSUPPORTED" in str(e.value)


def test_set_shape_and_bind_matrix_checks():
    q = S.bicgk(1024, 1024)
    p = _plan(q)
    L = kf.lib()
    A = q.values["A"]
    try:
        assert L.kf_plan_set_shape(p, 0, 0) == kf.KF_ERR_SHAPE
        assert L.kf_plan_set_shape(p, 1025, 1025) == kf.KF_ERR_SHAPE
        assert L.kf_plan_set_shape(p, 100, 200) == kf.KF_ERR_SHAPE      # declared square
        assert L.kf_plan_set_shape(p, 100, 100) == kf.KF_OK
        assert L.kf_bind_matrix(p, A, kf._vp(4096), 96) == kf.KF_ERR_ALIGN      # ld < cols
        assert L.kf_bind_matrix(p, A, kf._vp(4096), 102) == kf.KF_ERR_ALIGN     # rows not 16 bytes
        assert L.kf_bind_matrix(p, A, kf._vp(4096), 104) == kf.KF_OK
        assert L.kf_bind_matrix(p, q.values["p"], kf._vp(4096), 104) == kf.KF_ERR_DTYPE
        # an output overlapping the matrix at the runtime shape: 100 rows x 104 floats
        assert L.kf_bind(p, q.values["q"], kf._vp(4096 + 4 * 100 * 104 - 16)) == kf.KF_ERR_ALIAS
        assert L.kf_bind(p, q.values["q"], kf._vp(4096 + 4 * 100 * 104)) == kf.KF_OK
    finally:
        kf.kf_plan_destroy(p)
    # a plan without the flag has no runtime shape
    p = kf.kf_compile(q.script, mode="fused", flags=CG)
    try:
        assert L.kf_plan_set_shape(p, 10, 10) == kf.KF_ERR_STATE
        assert L.kf_bind_matrix(p, A, kf._vp(4096), 1024) == kf.KF_ERR_STATE
    finally:
        kf.kf_plan_destroy(p)


def test_non_square_declared_plan_takes_any_smaller_shape():
    q = S.bicgk(700, 1500)
    p = _plan(q)
    try:
        assert kf.lib().kf_plan_set_shape(p, 333, 1029) == kf.KF_OK
        assert kf.lib().kf_plan_set_shape(p, 701, 10) == kf.KF_ERR_SHAPE
    finally:
        kf.kf_plan_destroy(p)
