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
    """Compiles every source to an object (in parallel: the translation units
    share no device code) and links them into ``out``."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(os.path.dirname(HERE), "_build")
    os.makedirs(objdir, exist_ok=True)
    cflags = [f for f in HIPFLAGS if f != "-shared"] + list(extra or [])

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        subprocess.run([hipcc, *cflags, "-c", src, "-o", obj], check=True)
        return obj

    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = out + ".tmp"
    subprocess.run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC",
                    *objs, "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1:]))
