"""Build libdl.so (the C-ABI library of include/dl.h) for gfx950 with hipcc.

Every HIP source is compiled with packed-fp32 instructions disabled and
linked into one shared library next to this file.  Sources are compiled in
parallel; the build always runs (no staleness check), as the package loader
never builds by itself.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdl.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["bool_kernels.hip", "eps_solve.hip", "prog_kernels.hip", "peak.hip", "peak_agpr.hip", "dl_api.cpp",
           "serve.cpp", "program.cpp", "noalloc.cpp"]

# fp64 MFMA accumulators in architectural VGPRs rather than AGPRs: measured
# on MI355X, v_mfma_f64_16x16x4f64 chains sustain 77 TFLOP/s with VGPR
# accumulators and 48 TFLOP/s with AGPR ones (the compiler's default here)
PER_FILE = {
    "eps_solve.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
    "peak.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
}

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _compile(src: str, objdir: str) -> str:
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC, *COMMON, *PER_FILE.get(src, []), *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(6, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libdl.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
