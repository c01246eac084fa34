"""Build libgoat.so (HIP kernels for gfx950 + host C ABI) in-tree with hipcc.

    python -m paper_2111_05366_amd.build          # build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgoat.so")
ARCH = os.environ.get("GOAT_OFFLOAD_ARCH", "gfx950")
OMP_LIBDIR = "/opt/rocm/lib/llvm/lib"   # host OpenMP runtime of the ROCm clang

HIP_SOURCES = ["pack.hip", "gemm.hip", "sinkhorn.hip", "fw.hip", "mlp.hip", "batch.hip", "assign.hip", "noalloc.hip"]
CPP_SOURCES = ["api.cpp", "solve.cpp", "profile.cpp", "lap.cpp", "batch.cpp"]

# packed-fp32 instructions stay disabled for all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False, out: str = LIB, extra=None) -> str:
    """Compile every source and link libgoat.so at `out`. `extra`: additional
    compiler flags (e.g. ["-DGOAT_SK_NT"] for experiment builds)."""
    extra = list(extra or [])
    cc = hipcc()
    objs = []
    with tempfile.TemporaryDirectory(prefix="goat_build_") as tmp:
        for src in HIP_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc, *COMMON, *extra, "--offload-arch=" + ARCH, *DEVICE_FLAGS, "-x", "hip",
                   "-c", os.path.join(CSRC, src), "-o", obj]
            msg = _run(cmd)
            if verbose and msg.strip():
                print(msg)
            objs.append(obj)
        for src in CPP_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc, *COMMON, "-fopenmp", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-x", "c++", "-c",
                   os.path.join(CSRC, src), "-o", obj]
            _run(cmd)
            objs.append(obj)
        tmp_lib = os.path.join(tmp, "libgoat.so")
        _run([cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-fopenmp",
              "-Wl,-rpath," + OMP_LIBDIR, "-o", tmp_lib])
        shutil.copyfile(tmp_lib, out + ".tmp")
        os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
