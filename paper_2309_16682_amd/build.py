"""Build libvmt.so (HIP kernels for gfx950 + the C ABI) in the package directory.

    python -m paper_2309_16682_amd.build

Host sources are compiled with g++ (PCLMULQDQ for the GF(2) arithmetic),
the kernels with hipcc for gfx950, and everything is linked by hipcc.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libvmt.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HOST_SOURCES = ["gf2poly.cpp", "vmt_capi.cpp", "vmt_serve.cpp", "vmt_tune.cpp"]
HIP_SOURCES = ["vmt_kernels.hip", "vmt_check.hip"]
HIP_FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    # keep hipcc from forming packed FP32 instructions
    "-Xclang",
    "-target-feature",
    "-Xclang",
    "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-mpclmul", "-msse4.1", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(
        line for line in r.stdout.splitlines() if "packed-fp32-ops' is not a recognized feature" not in line
    )
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    gxx = shutil.which("g++") or "g++"
    inc = [f"-I{INCLUDE}", f"-I{CSRC}", f"-I{ROCM}/include"]
    with tempfile.TemporaryDirectory(prefix="vmt_build_") as tmp:
        objs = []
        for src in HOST_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            _run([gxx, *HOST_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
            objs.append(obj)
        for src in HIP_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            _run([hipcc, *HIP_FLAGS, *[f"-D{d}" for d in defines], *inc, "-c", os.path.join(CSRC, src), "-o", obj],
                 verbose)
            objs.append(obj)
        out_tmp = out + f".tmp{os.getpid()}"
        _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp, *objs], verbose)
        os.replace(out_tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
