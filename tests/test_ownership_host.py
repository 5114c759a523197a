"""The caller owns all device memory (CPU checks).

The built library imports no device (or pinned host) allocation routine of
the HIP runtime, so no entry point can allocate behind the caller's back; the
cost model works on the host until caller memory is bound and refuses device
work before that; the timed compile modes and the batch size their caller
workspaces with entry points that need no GPU."""
import ctypes
import subprocess

import numpy as np
import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import randscript as R
from paper_1305_1183_amd import sequences as S

ALLOCATORS = ("hipMalloc", "hipMallocAsync", "hipMallocManaged", "hipMallocPitch", "hipMalloc3D",
              "hipExtMallocWithFlags", "hipHostMalloc", "hipMallocHost", "hipFree", "hipFreeAsync",
              "hipHostFree", "hipFreeHost", "hipMallocFromPoolAsync", "hipMemCreate")


def test_library_imports_no_allocator():
    out = subprocess.run(["nm", "-D", "--undefined-only", kf.LIB_PATH], capture_output=True, text=True, check=True)
    imported = {line.split()[-1].split("@")[0] for line in out.stdout.splitlines() if line.strip()}
    assert "hipLaunchKernel" in imported or "hipModuleLaunchKernel" in imported   # the check sees HIP imports
    assert not imported & set(ALLOCATORS), sorted(imported & set(ALLOCATORS))


def _cm():
    h = ctypes.c_void_p()
    kf._chk(kf.lib().kf_costmodel_create(32, 2, 5, ctypes.byref(h)))
    return h


def test_costmodel_is_host_only_until_bound(tmp_path):
    L = kf.lib()
    h = _cm()
    try:
        n = ctypes.c_int64()
        kf._chk(L.kf_costmodel_dims(h, None, None, ctypes.byref(n)))
        p = np.empty(n.value, np.float32)
        mu, sd = np.empty(kf.FEATURE_DIM, np.float32), np.empty(kf.FEATURE_DIM, np.float32)
        y = np.empty(2, np.float64)
        fp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        kf._chk(L.kf_costmodel_get(h, fp(p), fp(mu), fp(sd), y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None))
        assert np.any(p != 0) and np.all(sd == 1)
        p2 = p * 0.5
        kf._chk(L.kf_costmodel_set(h, fp(p2), fp(mu), fp(sd), y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.25))
        path = str(tmp_path / "m.kfcm")
        kf._chk(L.kf_costmodel_save(h, path.encode()))
        h2 = ctypes.c_void_p()
        kf._chk(L.kf_costmodel_load(path.encode(), ctypes.byref(h2)))
        q = np.empty_like(p)
        kf._chk(L.kf_costmodel_get(h2, fp(q), None, None, None, None))
        assert np.array_equal(q, p2)
        L.kf_costmodel_destroy(h2)
        # device work before any memory is bound is refused (no GPU call is made)
        assert L.kf_costmodel_predict(h, 0, 0, 0, None) == kf.KF_ERR_UNBOUND
        assert L.kf_costmodel_train(h, 8, 8, 10, 1, 4, ctypes.c_float(1e-3), 0, None, None) == kf.KF_ERR_UNBOUND
        st = np.array([0, 0], np.int64)
        out = np.empty(1, np.float64)
        assert L.kf_costmodel_plan_us(h, None, 0, st.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None) == kf.KF_ERR_UNBOUND
        # sizing and the checks of bind need no GPU either
        b1, b2 = ctypes.c_size_t(), ctypes.c_size_t()
        kf._chk(L.kf_costmodel_workspace_bytes(h, 256, ctypes.byref(b1)))
        kf._chk(L.kf_costmodel_workspace_bytes(h, 8192, ctypes.byref(b2)))
        assert b1.value % 256 == 0 and b2.value > b1.value >= 4 * 4 * n.value
        assert L.kf_costmodel_bind(h, 4096 + 4, b1.value, 256, None) == kf.KF_ERR_ALIGN
        assert L.kf_costmodel_bind(h, 4096, b1.value - 1, 256, None) == kf.KF_ERR_WORKSPACE
    finally:
        L.kf_costmodel_destroy(h)


def test_learned_mode_needs_bound_model():
    q = S.bicgk(512, 512)
    h = _cm()
    try:
        with pytest.raises(kf.KFError) as e:
            kf.kf_compile(q.script, mode="learned", model=h, flags=kf.KF_COMPILE_CODEGEN_ONLY)
        assert "KF_ERR_UNBOUND" in str(e.value)
    finally:
        kf.lib().kf_costmodel_destroy(h)


@pytest.mark.parametrize("seed", [3, 11])
def test_timed_mode_workspace_covers_every_candidate(seed):
    rs = R.random_script(seed)
    need = kf.kf_compile_workspace_bytes(rs.script, mode="exhaustive", max_partitions=16)
    cands = kf.Candidates(rs.script, 16, None)
    most = 0
    for i in range(len(cands)):
        p = cands.compile(i, kf.KF_COMPILE_CODEGEN_ONLY)
        most = max(most, kf.kf_plan_workspace_bytes(p))
        kf.kf_plan_destroy(p)
    assert need == most


def test_gemver_timed_workspace_holds_the_unfused_intermediate():
    n = 1024
    q = S.gemver(n, n, 1.5, 0.5)
    need = kf.kf_compile_workspace_bytes(q.script, mode="exhaustive")
    assert need >= n * n * 4      # the unfused plan keeps B1 = A + u1 v1^T in the workspace


def test_batch_workspace_holds_the_tables():
    kinds = np.array([0, 1] * 500, np.int32)
    ns = np.array([100, 2000] * 500)
    small = kf.kf_batch_create(kinds[:2], ns[:2])
    big = kf.kf_batch_create(kinds, ns)
    try:
        ws_s, ws_b = kf.kf_batch_workspace_bytes(small), kf.kf_batch_workspace_bytes(big)
        items = kf.kf_batch_items(big, 0)[0]
        assert ws_b % 256 == 0
        # instance table (112 bytes per instance) and two item tables (8 bytes per item)
        assert ws_b - ws_s >= 998 * 112 + 2 * (len(items) - 4) * 8
    finally:
        kf.kf_batch_destroy(small)
        kf.kf_batch_destroy(big)
