"""Build tests/asan/_build/plan_checks: the library's sources with their host
code instrumented by AddressSanitizer (each -fsanitize flag on a hipcc line
follows -Xarch_host, so the GPU code is built as usual and not instrumented),
linked with the host-only driver plan_checks.cpp.  It exercises the plan,
ring-blocking and work-list logic through the host dry runs of the C ABI;
no kernel is launched."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from paper_1908_06097_amd import build as lib_build  # noqa: E402

OUT = os.path.join(HERE, "_build")
EXE = os.path.join(OUT, "plan_checks")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src):
    obj = os.path.join(OUT, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = ["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-I",
           os.path.join(ROOT, "include"), "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *ASAN,
           '-DSHTX_BUILD_ID="asan"', "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(lib_build.CSRC, s) for s in lib_build.SOURCES] + [os.path.join(HERE, "plan_checks.cpp")]
    with cf.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(_compile, srcs))
    link = ["hipcc", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", *objs, "-L",
            os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", EXE]
    subprocess.run(link, check=True)
    return EXE


if __name__ == "__main__":
    print(build())
