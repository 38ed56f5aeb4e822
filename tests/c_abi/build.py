"""Build the C-only roundtrip program against the in-tree libshtx.so (gcc,
host code only; the library carries the GPU code)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "_build", "roundtrip")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__", os.path.join(HERE, "roundtrip.c"),
           "-L", os.path.join(ROOT, "paper_1908_06097_amd"), "-lshtx", "-L", os.path.join(ROCM, "lib"),
           "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN/../../../paper_1908_06097_amd",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", EXE]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))
