"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer.

The C++ host sources (script recording, partition enumeration, code generation,
plan search, cost-model files, batch layout) are compiled with
``-fsanitize=address,undefined`` by the host compiler; the ahead-of-time device
sources are compiled by hipcc without any sanitizer, as the library build does.
``host_sanitize_driver.cpp`` then walks the C ABI in code-generation-only mode,
so no device is needed. A sanitizer report or a wrong status fails the test.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1305_1183_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(B.ROOT, "_build", "sanitize")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:]))


def _host_obj(src):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = [B.CLANG, "-x", "c++"] + B.COMMON + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                                                    "-c", os.path.join(B.CSRC, src), "-o", obj]
    _run(cmd)
    return obj


def _device_obj(src):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    _run([B.HIPCC, "-x", "hip"] + B.DEVICE + B.COMMON + ["-c", os.path.join(B.CSRC, src), "-o", obj])
    return obj


@pytest.fixture(scope="module")
def driver():
    if not os.path.exists(B.CLANG) or not os.path.exists(B.HIPCC):
        pytest.skip("ROCm compilers not found")
    os.makedirs(OUT, exist_ok=True)
    B._embed_blocks()
    with ThreadPoolExecutor(max_workers=8) as ex:
        host = list(ex.map(_host_obj, B.HOST_SOURCES))
        dev = list(ex.map(_device_obj, B.DEVICE_SOURCES))
        drv = ex.submit(_host_obj_driver).result()
    exe = os.path.join(OUT, "host_sanitize_driver")
    _run([B.CLANG] + SAN + ["-o", exe, drv] + host + dev +
         ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lhiprtc", "-lpthread"])
    return exe


def _host_obj_driver():
    obj = os.path.join(OUT, "host_sanitize_driver.o")
    _run([B.CLANG, "-x", "c++", "-std=c++17", "-I" + os.path.join(B.ROOT, "include")] + SAN +
         ["-c", os.path.join(HERE, "host_sanitize_driver.cpp"), "-o", obj])
    return obj


def test_host_code_clean_under_sanitizers(driver, tmp_path):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["KF_CACHE_DIR"] = str(tmp_path / "cache")
    r = subprocess.run([driver], capture_output=True, text=True, cwd=str(tmp_path), env=env, timeout=600)
    log = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in log, log[-6000:]
    assert "runtime error:" not in log, log[-6000:]
    assert r.returncode == 0, log[-6000:]
    assert "host sanitize driver: ok" in r.stdout
    shutil.rmtree(str(tmp_path / "cache"), ignore_errors=True)
