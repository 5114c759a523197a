"""Failure paths that the host can force (no GPU): an injected hipRTC error
surfaces as KF_ERR_COMPILE with the compiler log, a damaged code-object cache
entry is rebuilt instead of loaded, and a damaged cost-model file is refused
before any device work."""
import glob
import os
import struct
import subprocess
import sys

import pytest

from paper_1305_1183_amd import kf
from paper_1305_1183_amd import sequences as S


def test_injected_compile_error_reports_log(monkeypatch):
    monkeypatch.delenv("KF_CACHE_DIR", raising=False)
    monkeypatch.setenv("KF_JIT_EXTRA_SOURCE", "#error injected-for-test")
    q = S.bicgk(100, 100)
    with pytest.raises(kf.KFError) as e:
        kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD)
    assert "KF_ERR_COMPILE" in str(e.value) and "injected-for-test" in str(e.value)


def _fnv(b):
    h = 1469598103934665603
    for c in b:
        h = ((h ^ c) * 1099511628211) & ((1 << 64) - 1)
    return h


def test_damaged_cache_entry_is_rebuilt(monkeypatch, tmp_path):
    monkeypatch.setenv("KF_CACHE_DIR", str(tmp_path))
    monkeypatch.delenv("KF_JIT_EXTRA_SOURCE", raising=False)
    q = S.waxpby(12347, 1.25, 0.75)
    kf.kf_plan_destroy(kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD))
    files = glob.glob(os.path.join(str(tmp_path), "kf_*.co"))
    assert files
    for f in files:
        d = open(f, "rb").read()
        assert d[:4] == b"KFCO" and struct.unpack("<Q", d[4:12])[0] == _fnv(d[12:])
        with open(f, "r+b") as fh:                     # damage the code object
            fh.seek(len(d) // 2)
            fh.write(b"\x00garbage\x00")
    # a fresh process (this one remembers what it compiled) finds the damaged entry
    code = ("import sys; sys.path.insert(0, %r); from paper_1305_1183_amd import kf, sequences as S; "
            "q = S.waxpby(12347, 1.25, 0.75); "
            "kf.kf_plan_destroy(kf.kf_compile(q.script, mode='fused', flags=kf.KF_COMPILE_NO_LOAD))"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    env = dict(os.environ, KF_CACHE_DIR=str(tmp_path))
    subprocess.run([sys.executable, "-c", code], check=True, env=env, timeout=300)
    for f in files:
        d = open(f, "rb").read()
        assert d[:4] == b"KFCO" and struct.unpack("<Q", d[4:12])[0] == _fnv(d[12:]), "entry not rebuilt"


@pytest.mark.parametrize("content", [b"", b"KFCM", b"not a model at all" * 10,
                                     b"KFCM" + struct.pack("<4iq", 2, 32, 128, 3, 37377) + b"\x00" * 64])
def test_damaged_costmodel_file_refused(tmp_path, content):
    p = tmp_path / "m.kfcm"
    p.write_bytes(content)
    h = kf._vp()
    with pytest.raises(kf.KFError, match="KF_ERR_ARG"):
        kf._chk(kf.lib().kf_costmodel_load(str(p).encode(), kf.ctypes.byref(h)))


def test_shipped_costmodel_files_agree():
    """The library-format model shipped beside the numpy one holds the same
    numbers, under a valid header and checksum (decoded here field by field)."""
    import numpy as np
    data = os.path.join(os.path.dirname(kf.__file__), "data")
    d = open(os.path.join(data, "plan_cost_model.kfcm"), "rb").read()
    assert d[:4] == b"KFCM"
    assert struct.unpack("<Q", d[-8:])[0] == _fnv(d[4:-8])
    ver, dim, hid, layers, npar = struct.unpack("<4iq", d[4:28])
    assert ver == 2 and dim == kf.FEATURE_DIM
    off = 28
    mu = np.frombuffer(d, np.float32, dim, off); off += 4 * dim
    sd = np.frombuffer(d, np.float32, dim, off); off += 4 * dim
    y = np.frombuffer(d, np.float64, 2, off); off += 16
    lu = np.frombuffer(d, np.float32, 1, off)[0]; off += 4
    p = np.frombuffer(d, np.float32, npar, off); off += 4 * npar
    assert off == len(d) - 8
    z = np.load(os.path.join(data, "plan_cost_model.npz"), allow_pickle=False)
    assert [int(v) for v in z["dims"][:3]] == [dim, hid, layers]
    assert np.array_equal(p, z["params"]) and np.array_equal(mu, z["mu"]) and np.array_equal(sd, z["sd"])
    assert np.array_equal(y, z["y"])
    assert lu >= 0 and ('launch_us' not in z.files or np.float32(z['launch_us']) == lu)


def test_cache_dir_set_through_the_api(tmp_path, monkeypatch):
    """kf_jit_set_cache_dir overrides KF_CACHE_DIR: a compile (no device needed)
    writes its code object there; "" turns the disk cache off; None goes back to
    the environment. A path that is not a directory is refused."""
    monkeypatch.delenv("KF_CACHE_DIR", raising=False)
    d = tmp_path / "cache"
    d.mkdir()
    q = S.waxpby(12349, 1.25, 0.75)
    try:
        kf.kf_jit_set_cache_dir(str(d))
        p = kf.kf_compile(q.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD)
        kf.kf_plan_destroy(p)
        files = glob.glob(str(d / "kf_*.co"))
        assert len(files) == 1
        with pytest.raises(kf.KFError) as e:
            kf.kf_jit_set_cache_dir(str(d / "missing"))
        assert e.value.name == "KF_ERR_ARG"
        kf.kf_jit_set_cache_dir("")
        q2 = S.waxpby(12351, 1.25, 0.75)
        p = kf.kf_compile(q2.script, mode="fused", flags=kf.KF_COMPILE_NO_LOAD)
        kf.kf_plan_destroy(p)
        assert len(glob.glob(str(d / "kf_*.co"))) == 1   # nothing written with the cache off
    finally:
        kf.kf_jit_set_cache_dir(None)
