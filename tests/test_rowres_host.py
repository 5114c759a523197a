"""Register budget of the row-resident generator (no GPU).

Rows of 32768 columns give each lane eight float4 per row and per vector; with
the library's own geometry the generator then halves the rows per group and
moves column vectors to LDS or to loads from global memory. These tests check
where it does so and where it must not (requested parameters, rows of 16384
columns), and compile the generated kernels for gfx950 to check that the
forced single-pass kernels no longer spill."""
import json
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _plan(name, m, n, layout=kf.KF_ROW_MAJOR, **opts):
    q = S.by_name(name, m, n, {"alpha": 1.5, "beta": 0.75}, layout=layout)
    return kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD, **opts)


def _row_kernels(p):
    d = json.loads(kf.kf_plan_describe(p))
    return [(kk["params"], kf.kf_plan_source(p, k)) for k, kk in enumerate(d["kernels"])
            if kk["name"].startswith("kf_row")]


def test_wide_atax_halves_the_group():
    p = _plan("atax", 64, 32768)
    (params, src), = _row_kernels(p)
    assert params["group"] == 1 and params["kp"] == 8
    assert "__shared__ kf_f4 xs" in src and "cbg" not in src
    kf.kf_plan_destroy(p)


def test_wide_colmajor_gemver_moves_vectors_out_of_registers():
    p = _plan("gemver", 32768, 64, kf.KF_COL_MAJOR)
    (params, src), = _row_kernels(p)
    main = src.split("_fin")[0]
    assert params["group"] == 1
    assert len(re.findall(r"__shared__ kf_f4 xs\d+", main)) == 1        # one 128 KiB vector fits LDS
    assert len(set(re.findall(r"kf_ld4_tail\(V(\d+), \(long\)\(cbg", main))) == 2
    assert not re.findall(r"kf_f4 cv\d+\[KP\]", main)
    kf.kf_plan_destroy(p)


@pytest.mark.parametrize("name", ["atax", "gesummv", "gemver", "bicgk"])
def test_requested_and_narrower_geometries_are_untouched(name):
    """The same kernel text as with the geometry requested explicitly: at
    16384 columns (four float4 per lane) nothing is over the budget, and
    requested parameters are never adjusted."""
    narrow = _plan(name, 256, 16384, mat_sched=1)
    asked = _plan(name, 256, 16384, mat_sched=1, mat_waves=16, mat_group=2)
    assert [s for _, s in _row_kernels(narrow)] == [s for _, s in _row_kernels(asked)]
    wide = _plan(name, 256, 32768, mat_sched=1, mat_waves=16, mat_group=2, mat_rows=16)
    for params, src in _row_kernels(wide):
        assert params["group"] == 2 and "cbg" not in src
    for p in (narrow, asked, wide):
        kf.kf_plan_destroy(p)


def _scratch_bytes(src):
    """Per-lane scratch of a generated kernel compiled for gfx950 (hipcc's
    resource-usage remarks; the library compiles the same text with hipRTC)."""
    blocks = open(os.path.join(ROOT, "paper_1305_1183_amd", "csrc", "device", "kf_blocks.h")).read()
    d = tempfile.mkdtemp(prefix="kfres")
    try:
        f = os.path.join(d, "k.hip")
        open(f, "w").write("#include <hip/hip_runtime.h>\n" + blocks + "\n" + src)
        r = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "--cuda-device-only", "-O3", "-std=c++17",
                            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                            "-Rpass-analysis=kernel-resource-usage", "-c", f, "-o", os.path.join(d, "k.o")],
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    finally:
        shutil.rmtree(d, ignore_errors=True)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("case", [("atax", 64, 32768, kf.KF_ROW_MAJOR), ("sgemvt", 32768, 64, kf.KF_COL_MAJOR)])
def test_forced_single_pass_kernels_do_not_spill(case):
    """ATAX and column-major SGEMVT must be row-resident (a gemv result feeds
    a gemtv of the same pass); with the geometry the library picks, their
    kernels at 32768 columns compile without scratch. (Column-major GEMVER,
    which holds B, its three column vectors' loads and the accumulator, still
    spills a little at that width.)"""
    name, m, n, layout = case
    p = _plan(name, m, n, layout)
    (params, src), = _row_kernels(p)
    assert all(s == 0 for s in _scratch_bytes(src))
    kf.kf_plan_destroy(p)
