"""Build libmbbp.so (HIP kernels for gfx950 + host library) in-tree with hipcc.

Every HIP translation unit is compiled with -ffp-contract=off (no fused
multiply-add is formed behind the source's back, so single-precision results
follow the written operation order) and without packed FP32 instructions.
"""

from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmbbp.so")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-result"]
# Packed FP32 instructions are disabled in every translation unit.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Kernels only: IEEE mode off, so min/max need no NaN-quieting canonicalisation (BP
# messages are never NaN, no result changes).  Not for the host file, whose argument
# checks must still see NaN.
KERNEL_ONLY = ["-mno-amdgpu-ieee", "-fno-honor-nans"]
# The flooding BP kernels: branches on wave-uniform values (a pass's largest degree)
# are left as scalar branches rather than rewritten into structured flow with flag
# registers, which cost the variable phase a dozen scalar instructions per pass.
UNIFORM_BRANCHES = ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]
PER_SOURCE = {"mbbp_bp_dual.hip": UNIFORM_BRANCHES, "mbbp_bp.hip": UNIFORM_BRANCHES}
SOURCES = ["mbbp_bp.hip", "mbbp_bp_dual.hip", "mbbp_bp_serial.hip", "mbbp_bp_serial_slots.hip", "mbbp_wbp.hip",
           "mbbp_kernels.hip", "mbbp_host.cpp"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE, *KERNEL_ONLY, *PER_SOURCE.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, "-x", "hip", *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    warn = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build() -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
