"""Builds the native library (HIP for gfx950 + host C++) in-tree.

    python paper_2507_04786_amd/build.py           # (run by path, not as a module)
    python paper_2507_04786_amd/build.py --jitter  # the race-detection build

Produces paper_2507_04786_amd/lib/libvccl.so (with --jitter:
lib/libvccl_jitter.so, compiled with -DVCCL_JITTER: random pauses before every
publish and poisoned consumed FIFO slots; the binding loads it when VCCL_LIB
names it).  Every source is compiled by hipcc for gfx950 only; objects are
cached per source and variant under paper_2507_04786_amd/_build/ and rebuilt
when the source or a header changes.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libvccl.so")

SOURCES = ["device.hip", "host_comm.cpp", "host_plan.cpp", "host_api.cpp", "host_serve.cpp", "host_noalloc.cpp"]
HEADERS = ["vccl_dev.h", "host_internal.h", "tune_table.inc"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]
# no fused multiply-add contraction in the reduction code; no packed fp32 ops
DEVICE_FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-ffp-contract=off",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


VARIANTS = {"": [], "jitter": ["-DVCCL_JITTER=1"]}


def _digest(src: str, extra: list) -> str:
    h = hashlib.sha256()
    for name in [src] + HEADERS + [os.path.join("..", "..", "include", "vccl.h")]:
        path = os.path.join(CSRC, name)
        with open(path, "rb") as f:
            h.update(f.read())
    h.update(" ".join(COMMON + DEVICE_FLAGS + extra).encode())
    return h.hexdigest()[:16]


def _compile(src: str, force: bool, extra: list) -> str:
    obj = os.path.join(BUILD, src + "." + _digest(src, extra) + ".o")
    if os.path.exists(obj) and not force:
        return obj
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(force: bool = False, verbose: bool = True, variant: str = "") -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    extra = VARIANTS[variant]
    lib = LIB if not variant else os.path.join(LIBDIR, f"libvccl_{variant}.so")
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, extra), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(force="--force" in sys.argv, variant="jitter" if "--jitter" in sys.argv else "")
