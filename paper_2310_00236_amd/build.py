"""Build libhalfwave.so (HIP for gfx950) in place, next to this file.

    python -m paper_2310_00236_amd.build

Every source is compiled without floating-point contraction (so a*b+c is two
rounded operations, as the method's op-by-op definition requires), without
fast-math, with fp32 denormals kept, and with packed-fp32 instructions
disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhalfwave.so")
SOURCES = ["acoustic2d.hip", "acoustic2d_var.hip", "acoustic2d_tb.hip", "acoustic2d_tb_var.hip",
           "elastic3d.hip", "elastic2d.hip", "runtime.hip", "convert.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-mcode-object-version=5", "-O3", "-std=c++17",
    "-fPIC",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _obj(src: str, outdir: str) -> str:
    return os.path.join(outdir, os.path.splitext(src)[0] + ".o")


def build(verbose: bool = False, jobs: int = 7) -> str:
    """Compile every HIP source for gfx950 and link libhalfwave.so."""
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)

    def compile_one(src):
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", _obj(src, outdir)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return r.stderr

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for warn in ex.map(compile_one, SOURCES):
            if verbose and warn.strip():
                print(warn, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-mcode-object-version=5",
           "-shared", "-fPIC", "-o", tmp,
           *[_obj(s, outdir) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
