"""The library's measurement helpers on the GPU: the calibration copy, the
streaming read and copy references, and the seeded input fill."""
import numpy as np
import pytest
import torch

from paper_1305_1183_amd import inputs as I
from paper_1305_1183_amd import kf

pytestmark = pytest.mark.gpu


def _stream():
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("rows", [1, 3000, 4096])   # one row block, a ragged second one, exactly two
def test_strip_copy_reference_is_a_copy(rows):
    n = rows * 16384                                   # rows of 64 KiB
    src = torch.empty(n, dtype=torch.float32, device="cuda").uniform_(-1, 1)
    dst = torch.full((n + 16384,), 7.0, dtype=torch.float32, device="cuda")
    kf.kf_util_stream(1, dst.data_ptr(), src.data_ptr(), n * 4, _stream())
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src)
    assert torch.all(dst[n:] == 7.0)                  # nothing past the end is written


@pytest.mark.parametrize("n", [4, 1 << 20, (1 << 22) + 36])
def test_read_reference_sums_the_buffer(n):
    src = torch.empty(n, dtype=torch.float32, device="cuda").uniform_(-1, 1)
    sink = torch.zeros(2048, dtype=torch.float32, device="cuda")
    kf.kf_util_stream(0, sink.data_ptr(), src.data_ptr(), n * 4, _stream())
    torch.cuda.synchronize()
    got = float(sink.double().sum())
    want = float(src.double().sum())
    bound = 1e-6 * float(src.abs().double().sum()) + 1e-6
    assert abs(got - want) <= bound, (got, want)


def test_calibration_copy_and_fill():
    n = (1 << 20) + 4
    src = torch.empty(n, dtype=torch.float32, device="cuda").uniform_(-1, 1)
    dst = torch.zeros_like(src)
    kf.kf_util_copy(dst.data_ptr(), src.data_ptr(), n * 4, _stream())
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    rows, cols, ld, seed, tid = 37, 45, 48, 12345, 3
    out = torch.empty(rows * ld, dtype=torch.float32, device="cuda")
    kf.kf_util_fill_uniform(out.data_ptr(), rows, cols, ld, I.stream_key(seed, tid), float("nan"), _stream())
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(rows, ld)
    host = I.matrix(seed, tid, rows, cols, ld)        # the host generator, same stream
    assert np.all(np.isnan(got[:, cols:]))
    assert np.array_equal(got[:, :cols], host[:, :cols])


def test_plan_kernels_compile_together(monkeypatch):
    """A plan's new kernels are compiled in one invocation into one module
    (no disk cache) and still compute the right results."""
    from paper_1305_1183_amd import workloads as WL
    from tests import seqcheck as SC
    monkeypatch.delenv("KF_CACHE_DIR", raising=False)
    m, n = 999, 1234                                  # shapes no other test compiles
    arrays, scal = WL.make("gemver", m, n, seed=21)
    mods0, comp0 = kf.kf_jit_stats()
    q, prog, host = SC.run_gpu("gemver", m, n, arrays, scal, mode="unfused", mat_rows=64, mat_waves=2, mat_group=4)
    mods1, comp1 = kf.kf_jit_stats()
    assert prog.num_kernels == 4
    assert comp1 - comp0 == 4 and mods1 - mods0 == 1
    SC.check_against_oracle("gemver", m, n, host, SC.oracle_outputs("gemver", arrays, scal, n))
