"""Compile librecsplit.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/build.hip", "csrc/api.hip", "csrc/tables.cpp", "csrc/server.cpp", "csrc/schedule.cpp"]
HEADERS = ["csrc/rs_internal.h", "csrc/rs_host.h", "csrc/launch.h", "../include/recsplit.h"]
LIB = os.path.join(HERE, "librecsplit.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17", "-Wall", "-pthread",
    # no packed fp32 instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


TORCH_ALLOC = os.path.join(HERE, "libtorchalloc.so")


def _run(cmd, out, verbose):
    tmp = out + ".tmp"
    res = subprocess.run([*cmd, "-o", tmp], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, out)
    return out


def build_library(verbose: bool = False) -> str:
    _run([HIPCC, *FLAGS, *[os.path.join(HERE, s) for s in SOURCES]], LIB, verbose)
    build_torch_allocator(verbose)
    return LIB


def build_torch_allocator(verbose: bool = False) -> str:
    """The shim that hands PyTorch's caching allocator to rs_set_allocator
    (host code only; links the installed torch's c10 libraries)."""
    import torch

    tdir = os.path.dirname(torch.__file__)
    abi = int(torch._C._GLIBCXX_USE_CXX11_ABI)
    cmd = [HIPCC, "-O2", "-fPIC", "-shared", "-std=c++17", "-Wall", "-D__HIP_PLATFORM_AMD__=1", "-DUSE_ROCM=1",
           f"-D_GLIBCXX_USE_CXX11_ABI={abi}", "-I" + os.path.join(tdir, "include"),
           os.path.join(HERE, "csrc/torch_alloc.cpp"), "-L" + os.path.join(tdir, "lib"), "-lc10_hip", "-lc10",
           "-Wl,-rpath," + os.path.join(tdir, "lib")]
    return _run(cmd, TORCH_ALLOC, verbose)


if __name__ == "__main__":
    print(build_library(verbose=True))
