"""Builds the HIP library ``liblbm.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lbm.hip", "lbm_api.hip", "lbm_batch.hip", "lbm_adjoint.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

HIPFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP64 fused multiply-adds as three-address v_fma_f64: the two-address
    # v_fmac_f64 ties the addend to the destination, which costs a register
    # copy per polynomial coefficient held in a vector register
    "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst",
    "-Wno-unused-command-line-argument",
    # only the functions of include/lbm.h are exported (LBM_API)
    "-fvisibility=hidden",
]


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES
            if os.path.exists(os.path.join(CSRC, s))]


def build(extra: list[str] | None = None, out: str = LIB) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPFLAGS, *(extra or []), *sources(), "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1:]))
