"""Build libspx.so (all HIP kernels plus the C ABI) for gfx950 with hipcc.

Every translation unit is compiled to an object in parallel, then linked
into ``paper_2311_15439_amd/libspx.so`` in place.  Run
``python -m paper_2311_15439_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libspx.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("SPX_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.hip", "mlp.hip", "optim.hip", "field_query.hip", "composite.hip", "measure.hip"]
# encode_unit.hip is compiled once per (cell, dimension, features): (object name, defines)
UNITS = [(f"encode_{'grid' if g else 'simplex'}_d{d}_f{f}",
          [f"-DSPX_UNIT_GRID={g}", f"-DSPX_UNIT_DIM={d}", f"-DSPX_UNIT_F={f}"])
         for g in (1, 0) for d in (6, 5, 4, 3, 2, 1) for f in (2, 8, 4, 1)]

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    # no packed binary32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]
# The encoding's index path must follow the IEEE operation order exactly.
PER_FILE = {
    "encode_unit.hip": ["-ffp-contract=off"],
    # the fused adjoint + Adam (in the encode units) and the standalone Adam
    # perform the same binary32 operation sequence
    "optim.hip": ["-ffp-contract=off"],
    "field_query.hip": ["-ffp-contract=off"],
    # the network backward's products feed vector code: their results go to
    # ordinary registers instead of accumulation registers (which took one
    # copy instruction per result value)
    "mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _compile(job) -> str:
    src, name, defines = job
    obj = os.path.join(BUILD, name + ".o")
    cmd = ["hipcc", *COMMON, *PER_FILE.get(src, []), *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    # the slowest units (grid, high dimensions) first
    jobs = [("encode_unit.hip", name, d) for name, d in UNITS] + [(s, s.replace(".hip", ""), []) for s in SOURCES]
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
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
