"""Builds librflbm.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2507_08820_amd.build   (or __graft_entry__.build()).
Every call recompiles all sources.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librflbm.so")
SOURCES = ["step.hip", "aux.hip", "sk.hip", "noalloc.hip", "api.cpp", "batch.cpp"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-munsafe-fp-atomics",
    # multiply-adds only where the source writes them (fmaf, or a * b + c in one
    # expression): every kernel that expands the node body then rounds alike, so
    # the row-aligned, tiled and batched steps store the same bits
    "-ffp-contract=on",
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip():
        print(err, file=sys.stderr)
    return obj


# AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (the C
# interface, batch and run-time logic); device code is built as usual.  The
# library is then loaded with clang's ASan runtime preloaded.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-g"]


def build(verbose: bool = False, extra_flags=(), out: str = LIB, build_dir: str = BUILD,
          sanitize_host: bool = False) -> str:
    """Compiles every source and links `out`; extra_flags go to every hipcc call."""
    if sanitize_host:
        extra_flags = (*extra_flags, *HOST_SANITIZE)
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, tuple(extra_flags)), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}", file=sys.stderr)
    return out


if __name__ == "__main__":
    build(verbose=True)
