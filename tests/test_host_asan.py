"""The host code of the C-ABI library under AddressSanitizer: the library is
rebuilt with the sanitizer on its host pass and the host-only boundary tests
(validation, option checks, null handles) run against it in a child process
(see paper_2406_05020_amd/asan_check.py).  No GPU is needed."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None or
                    not glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"),
                    reason="hipcc or the AddressSanitizer runtime is not installed")
def test_host_code_is_clean_under_address_sanitizer():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "paper_2406_05020_amd", "asan_check.py")],
                       capture_output=True, text=True, timeout=900, cwd=ROOT)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
