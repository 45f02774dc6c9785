"""Build the HIP library ``liblbm_hip.so`` for gfx950 (in-tree).

    python -m paper_2309_02825_amd.build

Every HIP source is compiled with packed-FP32 instructions disabled (the
kernels are FP64; this keeps the compiler from emitting packed FP32 forms in
any float code).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblbm_hip.so")
SOURCES = [os.path.join(CSRC, "lbm_kernels.hip"), os.path.join(CSRC, "lbm_api.hip")]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    # no floating-point contraction: every kernel that runs the same
    # collision performs the same roundings (fused multi-step passes and the
    # batched form are bitwise equal to single steps)
    return ["-O3", "-ffp-contract=off", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
            "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + hipcc_flags() + ["-shared", "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
