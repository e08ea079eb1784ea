"""Build the gfx950 shared library libmrhweno.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmrhweno.so")
SOURCES = ["mr_kernels.hip", "mr_stage2d.hip", "mr_kxrcf2d.hip", "mr_mlp.hip", "mr_api.hip"]
# per-file code generation options: the 2D stage kernel runs at a fixed two
# waves per SIMD (LDS-bound), so its instructions are scheduled for
# instruction-level parallelism rather than for occupancy (measured ~2%
# faster; the indicator kernel is faster with the default)
FILE_FLAGS = {"mr_stage2d.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}
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
    """Compile every translation unit (in parallel) and link the library."""
    import concurrent.futures
    import tempfile
    cflags = [f for f in FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory() as tmpdir:
        objs, cmds = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src.replace(".hip", ".o"))
            objs.append(obj)
            cmds.append([HIPCC] + cflags + FILE_FLAGS.get(src, []) + ["-I", CSRC, "-c",
                                                                     os.path.join(CSRC, src), "-o", obj])
        with concurrent.futures.ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            for cmd in cmds:
                if verbose:
                    print(" ".join(cmd), flush=True)
            list(ex.map(subprocess.check_call, cmds))
        tmp = LIB + ".tmp"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--regen" in sys.argv:
        regenerate_coefficients()
    print(build(verbose=True))
