"""Build libcutcell.so (host C++ + HIP kernels for gfx950) in-tree.

    python -m paper_2410_05865_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcutcell.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["api.cpp", "kernels.hip", "net.hip", "quadrature.cpp", "level.cpp", "mf_lu.cpp", "fitted.cpp"]
ARCH = os.environ.get("CUTCELL_ARCH", "gfx950")

# packed FP32 instructions stay off (the compiler must not form v_pk_*_f32)
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# hardware FP64 atomic add on device memory (coarse-grained allocations only)
COMMON = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-munsafe-fp-atomics", "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *COMMON, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), "-shared", "-fopenmp", *DEVICE_FLAGS, *objs, "-o", tmp,
           f"-Wl,-rpath,{rocm}/llvm/lib", f"-Wl,-rpath,{rocm}/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed\n{res.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
