"""Build the gfx950 library ``libkf.so`` in-tree with hipcc.

The host runtime (script recording, plan enumeration, code generation, hipRTC
compilation, launch) and the ahead-of-time HIP kernels are compiled into one
shared library next to this file. The device building-block header is
embedded into the library as a string so that run-time compiled kernels need
no files on disk.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkf.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
ARCH = "gfx950"
COMMON = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

HOST_SOURCES = ["api.cpp", "plan.cpp", "codegen.cpp", "jit.cpp", "search.cpp", "costmodel.cpp", "batch.cpp"]
DEVICE_SOURCES = ["device/kf_util.hip", "device/kf_mlp.hip", "device/kf_batch.hip", "device/kf_noalloc.hip", "device/kf_quant.hip"]


def _embed_blocks() -> None:
    src = os.path.join(CSRC, "device", "kf_blocks.h")
    dst = os.path.join(CSRC, "kf_blocks_embed.inc")
    text = open(src).read()
    if ")KFBLOCKS\"" in text:
        raise RuntimeError("building-block header contains the raw-string delimiter")
    out = 'R"KFBLOCKS(' + text + ')KFBLOCKS"\n'
    if not os.path.exists(dst) or open(dst).read() != out:
        with open(dst, "w") as f:
            f.write(out)


def _compile(src: str) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + DEVICE + COMMON + ["-c", path, "-o", obj]
    else:
        cmd = [CLANG, "-x", "c++"] + COMMON + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                                           "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libkf.so (always rebuilds)."""
    _embed_blocks()
    sources = [s for s in HOST_SOURCES + DEVICE_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(sources))) as ex:
        objs = list(ex.map(_compile, sources))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC"] + DEVICE + ["-o", tmp] + objs + ["-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
