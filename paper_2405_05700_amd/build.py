"""Builds libpp.so (the C-ABI library and its gfx950 kernels) in place with
hipcc. Run as ``python -m paper_2405_05700_amd.build``."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpp.so")
SOURCES = [os.path.join(CSRC, f) for f in ("pp_api.cpp", "pp_kernels.hip", "sur_api.cpp",
                                            "sur_kernels.hip", "srv_api.cpp", "pp_static.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("pp_device.h", "pp_internal.h", "sur_device.h", "gelu_cdf_table.h")] + \
          [os.path.join(ROOT, "include", f) for f in ("pp.h", "pp_surrogate.h", "pp_server.h")]
ARCH = "gfx950"

# Packed-FP32 instructions are disabled: hipcc -O3 would otherwise form
# v_pk_* FP32 ops from scalar code.
HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result", "-pthread"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-shared", *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
