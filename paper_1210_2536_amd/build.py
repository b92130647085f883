"""Build the HIP library ``libsmat_spmv.so`` for gfx950 (in-tree).

Usage: ``python -m paper_1210_2536_amd.build`` (always recompiles).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsmat_spmv.so")
ARCH = os.environ.get("SMAT_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.hip", "k_features.hip", "k_convert.hip", "k_spmv.hip", "k_mlp.hip", "batch.hip",
           "noalloc.hip"]

# Packed-fp32 instructions are disabled for every device compile.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


# The sources that decide what the SpMV kernels cost: the kernels, their
# launch parameters and plan set-up, the formats they read, the interface.
TIMING_SOURCES = ["csrc/k_spmv.hip", "csrc/spmv_device.hpp", "csrc/api.hip", "csrc/k_convert.hip",
                  "csrc/internal.hpp", "csrc/plan.hpp", "../include/spmv.h"]


def _strip_comments(text: str) -> str:
    """C/C++ source without comments and with whitespace runs collapsed
    (string and character literals kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def sources_digest(rel_paths) -> str:
    """SHA-256 of the given sources (relative to the package) with comments
    and layout removed."""
    import hashlib
    h = hashlib.sha256()
    for rel in rel_paths:
        with open(os.path.join(HERE, rel)) as fh:
            h.update(os.path.basename(rel).encode())
            h.update(_strip_comments(fh.read()).encode())
    return h.hexdigest()


def timing_sources_digest() -> str:
    """Digest of TIMING_SOURCES: timing tables and the models fitted to them
    describe the kernels these sources build, and no others."""
    return sources_digest(TIMING_SOURCES)


def all_sources_digest() -> str:
    """Digest of every HIP source and header of the library and the C
    interface: a counter record describes the kernels these build."""
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".h")))
    return sources_digest([os.path.join("csrc", f) for f in names] + ["../include/spmv.h"])


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if warn.strip():
        print(warn, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
