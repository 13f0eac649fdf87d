"""Builds libgacelle.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled with packed-FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``): the library relies on
ordinary FP32 VALU code only.  The host pass of hipcc warns that it does not
know that feature; the warning is expected.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libgacelle.so")
SOURCES = ["gc_pack.hip", "gc_mh.hip", "gc_ens.hip", "gc_fit.hip", "gc_sense.hip", "gc_capi.cpp", "gc_variants.cpp", "gc_noalloc.cpp",
           "gc_timing.cpp", "gc_server.cpp"]
ARCH = os.environ.get("GACELLE_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Wno-unused-function", "-Wno-pass-failed", "-Wno-cuda-compat", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(os.path.dirname(HERE), "include")]


def source_files():
    """Every file the library is compiled from (sorted, repository-relative)."""
    root = os.path.dirname(HERE)
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".hpp", ".h")))
    files = [os.path.join("paper_2511_22094_amd", "csrc", f) for f in names]
    files.append(os.path.join("include", "gacelle.h"))
    files.append(os.path.join("paper_2511_22094_amd", "build.py"))
    return root, files


def source_hash() -> str:
    """sha256 (first 16 hex digits) over the library's sources and its build
    script; embedded in the library and returned by gc_version(), so a run can
    tell whether the library it loaded was built from the sources beside it."""
    root, files = source_files()
    h = hashlib.sha256()
    for f in files:
        h.update(f.encode() + b"\0")
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()[:16]


def _compile(src: str, extra=()) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *COMMON, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    tag = [f'-DGC_SOURCE_HASH="{source_hash()}"']
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, tag if f == "gc_capi.cpp" else ()), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
