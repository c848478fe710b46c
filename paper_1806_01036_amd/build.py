"""Build libborth.so (HIP kernels + C ABI) for gfx950 with hipcc.

Each translation unit is compiled in parallel into ``_build/`` and linked
into ``paper_1806_01036_amd/libborth.so``.  Device code is built with
floating-point contraction off (the double-double kernels rely on it; every
FMA in the library is explicit) and with packed fp32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
INCLUDE = PKG.parent / "include"
OUT = PKG / "libborth.so"
BUILD = PKG / "_build"
ARCH = os.environ.get("BORTH_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    "gram.hip",
    "split.hip",
    "factor.hip",
    "update.hip",
    "update_k4.hip",
    "update_k8.hip",
    "update_k16.hip",
    "update_k32.hip",
    "update_k64.hip",
    "update_narrow.hip",
    "update_narrow_gram.hip",
    "update_dd.hip",
    "noalloc.hip",
    "probe.hip",
    "batch_persistent.hip",
    "batch.cpp",
    "borth.cpp",
]

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    "-Wno-unused-value",
    "-Wno-pass-failed",
    f"-I{INCLUDE}",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _compile(src: str, force: bool) -> Path:
    s = CSRC / src
    o = BUILD / (s.stem + ".o")
    deps = [s] + list(CSRC.glob("*.hpp")) + [INCLUDE / "borth.h"]
    if not force and o.exists() and all(o.stat().st_mtime >= d.stat().st_mtime for d in deps):
        return o
    tmp = o.with_suffix(".o.tmp")
    cmd = [_hipcc(), *CFLAGS, "-c", str(s), "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    os.replace(tmp, o)
    return o


def build(force: bool = True, jobs: int | None = None, verbose: bool = False) -> Path:
    """Compile every source (all of them when ``force``) and link libborth.so."""
    BUILD.mkdir(exist_ok=True)
    srcs = [s for s in SOURCES if (CSRC / s).exists()]
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    tmp = OUT.with_suffix(".so.tmp")
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp),
           *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}", file=sys.stderr)
    return OUT


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
