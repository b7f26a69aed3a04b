"""Build ``liblbm_axi.so`` (HIP, gfx950) in place next to this file.

    python -m paper_1409_5929_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
SOURCES = [os.path.join(_HERE, "csrc", "lbm_axi.hip")]
HEADERS = [os.path.join(_HERE, "csrc", h) for h in ("lbm_axi_dev.h", "lbm_axi_desc.h")] + [
    os.path.join(_ROOT, "include", "lbm_axi.h")]
TARGET = os.path.join(_HERE, "liblbm_axi.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = TARGET + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I" + os.path.join(_ROOT, "include"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + " ".join(SOURCES))
    os.replace(tmp, TARGET)
    return TARGET


if __name__ == "__main__":
    print(build(verbose=True))
