"""Host-side AddressSanitizer check of the gpfvm C++ library.

Builds a variant of libgpfvm.so whose host code is instrumented with
AddressSanitizer (the device code is compiled as usual: the sanitizer flags go
to the host pass only), then runs the host-only C-ABI tests against it in a
child process with the sanitizer runtime preloaded.  Those tests reach the
IBVP validation, the option checks of every entry point and the null-handle
paths, all of which run on the host before any HIP call, so the check needs
no GPU.  Any invalid host memory access ends the child with the sanitizer's
report and a non-zero status.

    python paper_2406_05020_amd/asan_check.py
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
import build as B  # noqa: E402  (the library's own compile flags and source list)

OUT = os.path.join(HERE, "_build", "asan")
LIB = os.path.join(OUT, "libgpfvm_asan.so")
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    r = subprocess.run(["hipcc", *B.CFLAGS, "-g", *HOST_ASAN, "-c", src, "-o", obj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def asan_runtime() -> str:
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("the AddressSanitizer runtime of the ROCm clang was not found")
    return hits[-1]


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = B.sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    cmd = ["hipcc", f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-shared-libasan", *HOST_ASAN, "-o", LIB, *objs,
           "-lrocblas"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    return LIB


def run() -> int:
    lib = build()
    env = dict(os.environ)
    env["GPFVM_LIB"] = lib
    env["LD_PRELOAD"] = asan_runtime()
    # the interpreter and the uninstrumented libraries it loads are not what is checked here
    env["ASAN_OPTIONS"] = "detect_leaks=0:alloc_dealloc_mismatch=0:halt_on_error=1"
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q", "-p", "no:cacheprovider"]
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(run())
