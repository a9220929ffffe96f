"""The library's host runtime under AddressSanitizer: runtime.hip and
batch.hip rebuilt with the sanitizer on their host code only (device code
unchanged), linked with the other objects of the in-tree build, and the
CPU-side ABI tests (descriptions, validation, required sizes, errors, null
handles) run against that copy in a child process with the sanitizer
runtime preloaded."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

pytestmark = pytest.mark.slow


def test_host_runtime_under_address_sanitizer(tmp_path):
    from paper_2010_11751_amd import build as B
    runtime = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not runtime or not os.path.exists(B.HIPCC):
        pytest.skip("no hipcc or no clang AddressSanitizer runtime")
    objs = []
    for src in B.SOURCES:
        obj = os.path.join(B.OBJDIR, os.path.splitext(src)[0] + ".o")
        if src in ("runtime.hip", "batch.hip"):
            obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
            subprocess.check_call([B.HIPCC, *B.CFLAGS, "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                                   "-fno-omit-frame-pointer", "-c", os.path.join(B.CSRC, src), "-o", obj],
                                  stderr=subprocess.DEVNULL)
        elif not os.path.exists(obj):
            pytest.skip("the in-tree build's objects are missing (build first)")
        objs.append(obj)
    lib = str(tmp_path / "liblbm_asan.so")
    subprocess.check_call([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-Xarch_host",
                           "-fsanitize=address", *objs, "-o", lib])
    env = dict(os.environ, LD_PRELOAD=runtime[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", LBM_LIBRARY=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
