"""Build libstencil.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2306_13002_amd.build [--jobs N]

Every translation unit is compiled with -ffp-contract=off: the plain forms
rely on it to keep the written rounding order, and the saturated forms state
every fused multiply-add explicitly with fma().  Packed FP32 instructions are
disabled (-packed-fp32-ops).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libstencil.so")
SOURCES = ["abi.cpp", "tune.cpp", "batch.cpp", "support.hip", "heat.hip", "poisson19.hip", "wave25.hip", "generic.hip", "stream.hip", "costmodel.hip", "costmodel_host.cpp", "rtc.cpp", "saturator.cpp", "program.cpp"]
ARCH = os.environ.get("STENCIL_OFFLOAD_ARCH", "gfx950")

CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "_build"),
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str) -> None:
    cmd = [hipcc(), *CXXFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")


def embed_headers(objdir: str) -> None:
    """Write rtc_headers.inc: the headers that generated kernels include, as
    C string literals (hipRTC compiles from memory)."""
    out = []
    for var, name in (("kCommonHppText", "common.hpp"), ("kGenericBodyHppText", "generic_body.hpp")):
        text = open(os.path.join(CSRC, name)).read()
        assert ")__HDR__" not in text
        out.append(f'static const char {var}[] = R"__HDR__({text})__HDR__";\n')
    path = os.path.join(objdir, "rtc_headers.inc")
    new = "".join(out)
    if not os.path.exists(path) or open(path).read() != new:
        with open(path, "w") as f:
            f.write(new)


def build(jobs: int = 8, verbose: bool = False) -> str:
    """Compile every source and link libstencil.so; always rebuilds."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    embed_headers(objdir)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(lambda so: _compile(*so), zip(SOURCES, objs)))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-ldl", "-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libstencil.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
