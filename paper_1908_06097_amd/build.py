"""Build libshtx.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed-FP32 instructions
disabled, then linked into one shared library next to this file.
"""
import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libshtx.so")
SOURCES = ["plan.cpp", "capi.cpp", "autotune.cpp", "k_tables.hip", "k_gemm.hip", "k_fft.hip", "k_wind.hip",
           "k_probe.hip"]
BUILD = os.path.join(HERE, "_build")

FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-I", INCLUDE,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]
# The peak probes' MFMA loops keep their accumulators in vector registers
# (with the accumulation-register form the compiler copies every accumulator
# out and back around each iteration's MFMAs).
EXTRA_FLAGS = {"k_probe.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def build_id():
    """Hash of every library source: keys the autotuner's cache to the kernels."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _compile(src, verbose, bid):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    cmd = ["hipcc", *lang, *FLAGS, *EXTRA_FLAGS.get(src, []), f'-DSHTX_BUILD_ID="{bid}"', "-c",
           os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    bid = build_id()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, bid), SOURCES))
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
