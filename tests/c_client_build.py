"""Compile tests/c_client.c, a plain C program using the library through
include/vccl.h, with gcc against the built libvccl.so and the HIP runtime."""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCE = os.path.join(ROOT, "tests", "c_client.c")
LIBDIR = os.path.join(ROOT, "paper_2507_04786_amd", "lib")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def available() -> str:
    """Empty when the client can be built here, else the reason it cannot."""
    if shutil.which("gcc") is None:
        return "gcc not found"
    if not os.path.exists(os.path.join(LIBDIR, "libvccl.so")):
        return "libvccl.so is not built"
    if not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h")):
        return "HIP headers not found"
    return ""


def build(out_path: str) -> None:
    """Strict C11 with every warning an error; raises on failure."""
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           SOURCE, "-o", out_path,
           "-L", LIBDIR, "-lvccl", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + LIBDIR, "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("c_client build failed:\n" + res.stdout + res.stderr)
