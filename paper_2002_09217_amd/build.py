"""Build libpond.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2002_09217_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpond.so")
SOURCES = ["pond_kernels.hip", "pond_step.hip", "pond_kernels3.hip", "pond_api.hip", "pond_batch.hip", "pond_noalloc.hip"]
# compilation units: (source, extra flags).  LLVM's max-ilp scheduling is faster for the
# D3Q27 kernels and for the FP64-window fused-step kernels, slower for the FP32-window ones:
# pond_step.hip is compiled a second time for its FP64 windows, with that strategy.
MAX_ILP = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
UNITS = [(s, MAX_ILP if s == "pond_kernels3.hip" else []) for s in SOURCES] + [
    ("pond_step.hip", ["-DPOND_STEP_DOUBLE_WINDOWS", *MAX_ILP])]
HEADERS = ["pond_device.h", "pond_internal.h", "pond_collide.h", "pond_stream.h", "pond_eos.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd))


def build(verbose: bool = False) -> str:
    """Compile every HIP compilation unit for gfx950 and link paper_2002_09217_amd/libpond.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="pond_build_") as d:
        objs = [os.path.join(d, f"u{i}.o") for i in range(len(UNITS))]
        cmds = [[hipcc, *HIPCC_FLAGS, *extra, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
                for (src, extra), obj in zip(UNITS, objs)]
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as pool:
            for f in [pool.submit(_run, c, verbose) for c in cmds]:
                f.result()
        _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
