"""Build libbp.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2402_14821_amd.build

Every HIP translation unit is compiled with the packed-fp32 feature off.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbp.so")
ARCH = os.environ.get("BP_OFFLOAD_ARCH", "gfx950")

SOURCES = ["bp_kernels.hip", "bp_api.cpp", "bp_queue.cpp", "bp_solve.cpp"]
# VALU issue-rate microbenchmark (bench.py --valu-rates), a library of its own
UBENCH_SOURCES = ["bp_ubench.hip"]
UBENCH_LIB = os.path.join(HERE, "libbp_ubench.so")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          f"--offload-arch={ARCH}", "-I", os.path.join(HERE, "..", "include")]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


# Kernels that must not use per-lane scratch memory: register spills there
# cost issue slots in the hot loops and HBM traffic (the compiler reports
# each kernel's scratch size; the build fails when one of these has any).
NO_SCRATCH = ("_ZN3bpi7k_sweepILi1E", "_ZN3bpi7k_sweepILi2E", "_ZN3bpi7k_sweepILi4E", "_ZN3bpi9k_combineILi",
              "_ZN3bpi13k_small_check",
              "_ZN3bpi6k_prep", "_ZN3bpi9k_vt_", "_ZN3bpi10k_finalize")


def _scratch_kernels(remarks: str):
    """Kernels (mangled names) with a nonzero scratch size in the compiler's
    kernel-resource-usage remarks."""
    bad, name = [], None
    for line in remarks.splitlines():
        if "Function Name:" in line:
            name = line.split("Function Name:")[1].split("[")[0].strip()
        elif "ScratchSize [bytes/lane]:" in line and name:
            size = int(line.split("ScratchSize [bytes/lane]:")[1].split("[")[0].strip())
            if size > 0 and name.startswith(NO_SCRATCH):
                bad.append((name, size))
    return bad


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile {src} failed:\n{res.stdout}\n{res.stderr}")
    bad = _scratch_kernels(res.stderr)
    if bad:
        raise RuntimeError(f"compile {src}: kernels that must not spill use scratch memory: {bad}")
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile every source, link libbp.so and the microbenchmark library
    libbp_ubench.so; returns the path of libbp.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES + UBENCH_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    _link([objs[s] for s in SOURCES], LIB)
    _link([objs[s] for s in UBENCH_SOURCES], UBENCH_LIB)
    if verbose:
        print(f"built {LIB} and {UBENCH_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
