"""Builds the HIP library libhmc.so in-tree for gfx950 with hipcc: each source compiled to an
object (in parallel, in a temporary directory), then linked."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhmc.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 (v_pk_*_f32) code generation stays off on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
# Per-source code-generation options.  The zone solve's step loop is pure FP32 arithmetic at
# two wavefronts per SIMD: the scheduler's instruction-level-parallelism strategy orders it
# 2 % faster per solve (the same registers, no spills); on the colour pass the same strategy
# costs occupancy, so it stays with the default there.  For the 5^3 zone (h = 2, its own
# source) the AMDGPU register-pressure trackers in that scheduler give a further 7 % (128^3
# workload: 5.62 -> 5.24 ms per colour launch, 254 of 256 registers, no spills); the same
# option makes h = 1 and h = 3 slower (0.365 -> 0.386 and 37.4 -> 38.1 ms) and the colour
# pass, explicit step and adjoint step too, so it is given to that source alone.
_MAX_ILP = ["-mllvm", "--amdgpu-sched-strategy=max-ilp"]
SOURCE_FLAGS = {
    "hmc_zone.hip": _MAX_ILP,
    "hmc_zone_h2.hip": _MAX_ILP + ["-mllvm", "--amdgpu-use-amdgpu-trackers"],
    # the 7^3 zone (its step loop spills a few registers at two wavefronts per SIMD): the
    # iterative maximum-occupancy strategy, 37.4 -> 35.6 ms per 128^3 colour launch
    "hmc_zone_h3.hip": ["-mllvm", "--amdgpu-sched-strategy=iterative-maxocc"],
}
LINK = [
    "--offload-arch=gfx950", "-shared", "-fPIC",
    # roctx ranges around sweeps, colour passes, refreshes and adjoint passes
    "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    inc = ["-I", os.path.join(HERE, "..", "include")]
    with tempfile.TemporaryDirectory(prefix="hmc_build_") as tmpdir:
        def compile_one(src):
            obj = os.path.join(tmpdir, os.path.basename(src)[:-4] + ".o")
            cmd = ["hipcc", *FLAGS, *SOURCE_FLAGS.get(os.path.basename(src), []), *inc, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
            return obj

        with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(compile_one, sources()))
        tmp = LIB + ".tmp"
        cmd = ["hipcc", *LINK, *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
