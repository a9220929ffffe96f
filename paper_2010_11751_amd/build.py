"""Build ``liblbm.so`` (HIP, gfx950) in-tree.

Each kernel translation unit (one per lattice x storage type) and the host
runtime compile in parallel with hipcc; the objects link into
``paper_2010_11751_amd/liblbm.so`` next to this file.
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
LIB = os.path.join(HERE, "liblbm.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = [
    "runtime.hip", "batch.hip",
    "k_q19_f64.hip", "k_q19_f32.hip", "k_q19_f16.hip",
    "k_q27_f64.hip", "k_q27_f32.hip", "k_q27_f16.hip",
    "k_q19_f64_mrt.hip", "k_q19_f32_mrt.hip", "k_q19_f16_mrt.hip",
    "k_q27_f64_mrt.hip", "k_q27_f32_mrt.hip", "k_q27_f16_mrt.hip",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
    # Fused multiply-adds only where one source expression has a*b + c, so
    # every kernel that inlines the collision computes it bit-identically.
    "-ffp-contract=on",
    # Packed FP32 instructions stay off (hipcc would otherwise form them from
    # float code).
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-variable", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _stale(src: str, obj: str) -> bool:
    """True if obj is older than its source or any header it may include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(d, f) for d in (CSRC, INCLUDE)
                                        for f in os.listdir(d) if f.endswith((".hpp", ".h"))]
    return any(os.path.getmtime(p) > t for p in deps)


def _compile(src: str, objdir: str = OBJDIR, defines=(), incremental: bool = False) -> str:
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    if incremental and not _stale(src, obj):
        return obj
    cmd = [HIPCC, *CFLAGS, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, defines=(), out: str | None = None,
          incremental: bool = False) -> str:
    """Compile every translation unit and link liblbm.so; returns its path.

    `defines` are extra preprocessor definitions (NAME=VALUE) and `out` an
    alternative library path, for building tuning variants side by side.
    `incremental` skips translation units whose object is newer than every
    source and header (development rebuilds; the default compiles all)."""
    out = out or LIB
    objdir = OBJDIR if out == LIB else out + ".objs"
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, objdir, defines, incremental), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
