"""Build libitergp.so (HIP for gfx950) in-tree.

    python -m paper_2310_20285_amd.build

Compiles every source under csrc/ with hipcc for gfx950 and links one shared
library next to this file.  Always rebuilds (the object files of the previous
build are reused only when their source and headers are older).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libitergp.so")
# issue-rate microbenchmarks (bench.py --workload peaks), a library of their own
PEAKS_SRC = "peaks.hip"
PEAKS_LIB = os.path.join(HERE, "libitergp_peaks.so")

SOURCES = ["kv.hip", "kv_mfma.hip", "kv_bf16.hip", "hessian.hip", "diaglik.hip", "linalg.hip", "batched_ops.hip", "blocklik.hip", "noalloc.hip", "itergp.cpp", "abi.cpp",
           "eigh.cpp"]
ARCH = "gfx950"
COMMON = [*os.environ.get("IGP_EXTRA_FLAGS", "").split(), "-O3", "-fPIC", "-std=c++17", f"-I{INCLUDE}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-parameter"]
# Packed FP32 instructions stay disabled on this target.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


# per-source device flags: the FP32 matrix-core kernels keep their MFMA
# accumulators in ordinary VGPRs (no accumulator-register copies before the
# kernel transform reads the distances)
SOURCE_FLAGS = {"kv_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
                # accumulators in VGPRs: loop-carried AGPR accumulators get rotated
                # through extra moves, which would be timed with the matrix unit
                "peaks.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}

# host-only sources (no HIP kernels), built with the host C++ compiler against
# the HIP host headers
HOST_ONLY = {"eigh.cpp"}
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def host_cxx() -> str:
    for c in (os.environ.get("CXX"), shutil.which("g++"), shutil.which("c++")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("no host C++ compiler found")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _headers_mtime() -> float:
    m = os.path.getmtime(os.path.join(INCLUDE, "itergp.h"))
    for f in os.listdir(CSRC):
        if f.endswith((".hpp", ".h")):
            m = max(m, os.path.getmtime(os.path.join(CSRC, f)))
    return m


def _compile(src: str, force: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJDIR, src + ".o")
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) > max(os.path.getmtime(path), _headers_mtime())):
        return obj
    if src in HOST_ONLY:
        cmd = [host_cxx(), *COMMON, "-mavx2", "-mfma", f"-I{ROCM}/include",
               "-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
    else:
        cmd = [hipcc(), "-x", "hip", *COMMON, *DEVICE, *SOURCE_FLAGS.get(src, []), "-c", path,
               "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(force: bool = True, verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    pobj = _compile(PEAKS_SRC, force)
    ptmp = PEAKS_LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", pobj, "-o", ptmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(ptmp, PEAKS_LIB)
    if verbose:
        print(f"built {LIB} and {PEAKS_LIB}")
    return LIB


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv, verbose=True)
