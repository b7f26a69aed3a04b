"""Build the HIP libraries (gfx950) in place next to this file:
``liblbm_axi.so`` (the lattice Boltzmann step) and ``liblbm_no.so`` (the
warm-start network).

    python -m paper_1409_5929_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIBS = {  # target -> sources
    os.path.join(_HERE, "liblbm_axi.so"): [os.path.join(_HERE, "csrc", "lbm_axi.hip"),
                                           os.path.join(_HERE, "csrc", "lbm_axi_s16.hip")],
    os.path.join(_HERE, "liblbm_no.so"): [os.path.join(_HERE, "csrc", "lbm_no.hip")],
}
TARGET = os.path.join(_HERE, "liblbm_axi.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    for target, sources in LIBS.items():
        tmp = target + ".tmp"
        cmd = [hipcc, *HIPCC_FLAGS, "-I" + os.path.join(_ROOT, "include"), "-o", tmp, *sources]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed for " + " ".join(sources))
        os.replace(tmp, target)
    return TARGET


if __name__ == "__main__":
    print(build(verbose=True))
