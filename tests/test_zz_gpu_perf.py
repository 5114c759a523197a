"""Performance floors of the fused suite at the benchmark's sizes (A 16384 x
16384, vectors 2**26, tuned parameters): the suite as a whole moves at least
70% of the 8 TB/s HBM peak in algorithmic bytes, every fused sequence at
least 60%, and fusion pays where it removes traffic (Table 2's speedups,
with margins for run-to-run noise). Inputs are filled on the device: the
values do not change the timing of these kernels.

Collected last, so that a slow device cannot stop the parity tests."""
import pytest
import torch

from paper_1305_1183_amd import sequences as S
from paper_1305_1183_amd import workloads as WL

pytestmark = pytest.mark.gpu

PEAK_GBPS = 8000.0
MIN_SPEEDUP = {"axpydot": 1.05, "waxpby": 1.4, "bicgk": 1.6, "atax": 1.6, "gesummv": 0.95, "gemver": 1.6}


def _time(q, mode, dev):
    m, n = (WL.SUITE_VEC,) * 2 if q.name in WL.BLAS1 else (WL.SUITE_N,) * 2
    prog = q.compile(mode=mode, **WL.tuned_params(q.name, m, n, mode)).bind(**dev)
    r, w = prog.bytes()
    us = prog.time(5, 20)
    return us, (r + w) / us / 1e3


def test_fused_suite_bandwidth_and_speedups():
    total_bytes, total_us, rows = 0.0, 0.0, {}
    for name in ("axpydot", "waxpby", "bicgk", "atax", "gesummv", "gemver"):
        m, n = (WL.SUITE_VEC,) * 2 if name in WL.BLAS1 else (WL.SUITE_N,) * 2
        q = S.by_name(name, m, n, {"alpha": 1.5, "beta": 0.75})
        dev = {}
        for k in q.inputs:
            shape = q.shapes[k]
            dev[k] = torch.empty(shape, dtype=torch.float32, device="cuda").uniform_(-1, 1)
        fu, fg = _time(q, "fused", dev)
        uu, _ = _time(q, "unfused", dev)
        rows[name] = (fg, uu / fu)
        total_bytes += fg * fu
        total_us += fu
        del dev
        torch.cuda.empty_cache()
    summary = {k: "%.0f GB/s, %.2fx" % v for k, v in rows.items()}
    assert total_bytes / total_us >= 0.70 * PEAK_GBPS, summary
    for name, (gbps, speedup) in rows.items():
        assert gbps >= 0.60 * PEAK_GBPS, (name, summary)
        assert speedup >= MIN_SPEEDUP[name], (name, summary)


def test_wide_row_single_pass_atax_keeps_its_registers():
    """Single-pass ATAX on rows of 32768 columns: the geometry the library
    picks (rows per group halved to fit the registers) at least 10% faster
    than the same 16-wave geometry with two rows per group requested, which
    spills (measured 632 against 789 us), and at least 65% of peak."""
    n = 32768
    q = S.atax(n, n)
    dev = {k: torch.empty(q.shapes[k], dtype=torch.float32, device="cuda").uniform_(-1, 1) for k in q.inputs}
    times = {}
    for key, opts in (("library", {}), ("requested", dict(mat_sched=1, mat_waves=16, mat_group=2, mat_rows=128))):
        prog = q.compile(mode="fused", **opts).bind(**dev)
        r, w = prog.bytes()
        times[key] = (prog.time(5, 20), (r + w))
        del prog
    (lib_us, nbytes), (req_us, _) = times["library"], times["requested"]
    assert req_us >= 1.10 * lib_us, times
    assert nbytes / lib_us / 1e3 >= 0.65 * PEAK_GBPS, times
