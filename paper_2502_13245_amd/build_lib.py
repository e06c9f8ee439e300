"""Build the HIP library (librr.so) for gfx950 with hipcc.

Usage: python -m paper_2502_13245_amd.build_lib   (or build() from Python)
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
OUT = os.path.join(HERE, "librr.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["rr_api.cpp", "rr_build.cpp", "rr_tune.cpp", "rr_server.cpp", "rr_kernels.hip", "rr_scan.hip", "rr_probe.hip"]
# rr_inst.hip holds the search kernels of one kernel data type (element type
# u8 0, i8 1, f32 2, bf16 pass 3, 8-bit pass 4; + 8 for the inner product);
# it is compiled once per type so the instantiations build in parallel.
INST_TYPES = {"u8": 0, "i8": 1, "f32": 2, "bf16": 3, "sq8": 4,
              "u8ip": 8, "i8ip": 9, "f32ip": 10, "bf16ip": 11, "sq8ip": 12}

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable", "-Xarch_host", "-march=x86-64-v3"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
# The MFMA scan keeps its accumulators in ordinary VGPRs, so that the
# per-element epilogue reads them without accumulator-register moves.
PER_SOURCE = {"rr_scan.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str) -> str:
    defs = []
    if ":" in src:  # rr_inst.hip:<type>
        src, tname = src.split(":")
        defs = [f"-DRR_INST={INST_TYPES[tname]}"]
        obj = os.path.join(BUILD, f"rr_inst_{tname}.o")
    else:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + DEVICE + defs + PER_SOURCE.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + COMMON + ["-x", "hip"] + DEVICE + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile {src} failed:\n{r.stderr[-8000:]}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [f"rr_inst.hip:{t}" for t in INST_TYPES] + [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-8000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
