"""Builds libxf.so (HIP kernels for gfx950 + host plan code) in-tree.

Every kernel translation unit (csrc/k_*.hip) is compiled separately, in
parallel, then linked with the host object."""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libxf.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# The host plan (sampling table, FP64 precompute) is compiled without FMA
# contraction on the baseline x86-64 ISA.
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall",
              "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def kernel_sources():
    return sorted(glob.glob(os.path.join(CSRC, "k_*.hip")))


def _stale(obj: str, src: str, headers) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src, *headers])


def build(verbose: bool = False, jobs: int = 0, incremental: bool = False) -> str:
    """Compiles every unit (or, with ``incremental``, those older than their
    source or any header) and links libxf.so."""
    os.makedirs(BUILD, exist_ok=True)
    headers = glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(HERE, "..", "include", "xf.h")]
    host_src = os.path.join(CSRC, "xf_host.cpp")
    host_o = os.path.join(BUILD, "xf_host.o")
    cmds = []
    if not incremental or _stale(host_o, host_src, headers):
        cmds.append(["g++", *HOST_FLAGS, "-c", host_src, "-o", host_o])
    objs = [host_o]
    for src in kernel_sources():
        o = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
        if not incremental or _stale(o, src, headers):
            cmds.append([HIPCC, *DEVICE_FLAGS, "-c", src, "-o", o])
        objs.append(o)
    jobs = jobs or min(max(len(cmds), 1), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    import sys
    build(verbose=True, incremental="--incremental" in sys.argv)
