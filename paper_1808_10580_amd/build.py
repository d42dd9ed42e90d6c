"""Build libpm.so (gfx950) in-tree with hipcc.

    python -m paper_1808_10580_amd.build          # compile every source, link
    python -m paper_1808_10580_amd.build --asm    # also dump the device ISA
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpm.so")
SOURCES = ["pm_kernels.hip", "pm_abi.hip", "pm_mlp.hip", "pm_hk.hip", "pm_mx.hip"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 VALU ops are disabled for every HIP translation unit.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-Wno-unused-but-set-variable", "-munsafe-fp-atomics"]


# The small-K matrix-core kernel keeps its MFMA accumulators in ordinary
# VGPRs (no AGPR copies between the contraction and the y form).
EXTRA = {"pm_mx.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC, *COMMON, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def sources():
    return [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(asm: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if asm:
        for s in srcs:
            out = os.path.join(BUILD, s.replace(".hip", ".s"))
            cmd = [HIPCC, *COMMON, *EXTRA.get(s, []), "--cuda-device-only", "-S", os.path.join(CSRC, s), "-o", out]
            subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--asm", action="store_true")
    ap.add_argument("-j", type=int, default=4)
    a = ap.parse_args()
    print(build(asm=a.asm, jobs=a.j))
    sys.exit(0)
