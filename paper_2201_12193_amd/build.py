"""Build the gfx950 shared library libmrhweno.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmrhweno.so")
SOURCES = ["mr_kernels.hip", "mr_stage2d.hip", "mr_mlp.hip", "mr_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # packed FP32 instructions stay off (they are not needed for FP64 code)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def regenerate_coefficients() -> None:
    """Regenerate recon_gen.h from gen_recon.py (exact rational derivation)."""
    out = subprocess.check_output([sys.executable, os.path.join(CSRC, "gen_recon.py")])
    path = os.path.join(CSRC, "recon_gen.h")
    old = open(path, "rb").read() if os.path.exists(path) else b""
    if old != out:
        with open(path, "wb") as f:
            f.write(out)


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-I", CSRC, "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--regen" in sys.argv:
        regenerate_coefficients()
    print(build(verbose=True))
