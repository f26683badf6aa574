"""Build libdcg.so (the C-ABI library) from the HIP sources with hipcc.

Usage:  python -m paper_1706_00241_amd.build   (or build() from Python)

Every source is compiled for gfx950 only.  Packed FP32 instructions are
disabled for device code (-packed-fp32-ops); hipcc's host pass warns that it
does not know that target feature, which is harmless.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdcg.so")
SOURCES = ["matvec.hip", "exact.hip", "blas.hip", "eig.hip", "operator.hip", "solver.hip",
           "block.hip", "grad.hip", "batch.hip", "gpc.hip",
           "stored.hip", "slq.hip", "implicit.hip", "wide.hip"]
# host-only C++ (no kernels): built by the host compiler alone
HOST_SOURCES = ["host.cpp"]
ARCH = "gfx950"


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the HIP toolchain is required")
    return p


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def host_cxx():
    p = shutil.which("g++")
    if p is None:
        raise RuntimeError("g++ not found: the host compiler is required")
    return p


def host_flags():
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    return ["-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__",
            "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
            "-Wall", "-Wno-unused-function"]


def _compile_host(src, objdir):
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = [host_cxx()] + host_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed for {src}:\n{r.stderr}")
    return obj


def _compile(src, objdir):
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stderr or "").splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
    return obj


def build(verbose=False):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir), SOURCES))
        objs += list(ex.map(lambda s: _compile_host(s, objdir), HOST_SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
