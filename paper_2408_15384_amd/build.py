"""Builds libmm.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_2408_15384_amd.build

Every source under csrc/ is compiled by hipcc to an object in _build/ (in
parallel), then linked into paper_2408_15384_amd/libmm.so.  The MFMA-only
measurement aid peak/mfma_peak.hip becomes libmm_peak.so."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build", "libmm")
LIB = os.path.join(HERE, "libmm.so")
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# Packed FP32 instructions are disabled for every device compile.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, *DEVICE_FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


PEAK_SRC = os.path.join(HERE, "peak", "mfma_peak.hip")
PEAK_LIB = os.path.join(HERE, "libmm_peak.so")


def build_peak(verbose: bool = True) -> str:
    """The MFMA-only measurement aid (include/mm_peak.h) as its own library."""
    tmp = PEAK_LIB + ".tmp"
    # accumulators in VGPRs: otherwise the binary64 chains are copied between
    # accumulation and vector registers on every iteration and the probe
    # measures the copies
    cmd = [hipcc(), *COMMON, *DEVICE_FLAGS, "-mllvm", "-amdgpu-mfma-vgpr-form=1", "-shared", "-o", tmp, PEAK_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {PEAK_SRC}:\n{r.stderr}")
    os.replace(tmp, PEAK_LIB)
    if verbose:
        print(f"built {PEAK_LIB}", file=sys.stderr)
    return PEAK_LIB


def build(verbose: bool = True) -> str:
    """Build libmm.so (and the measurement aid libmm_peak.so)."""
    build_peak(verbose)
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
