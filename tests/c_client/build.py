"""Build the plain C client of the C ABI (halfwave_run, next to this file)
with the host C compiler, against include/halfwave.h, the in-tree
libhalfwave.so and the HIP runtime.

    python tests/c_client/build.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
EXE = os.path.join(HERE, "halfwave_run")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror",
           "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{ROCM}/include",
           os.path.join(HERE, "halfwave_run.c"), "-o", EXE,
           f"-L{os.path.join(ROOT, 'paper_2310_00236_amd')}", "-lhalfwave",
           f"-L{ROCM}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2310_00236_amd", f"-Wl,-rpath,{ROCM}/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
