"""Build the HIP library libsr.so for gfx950 in-tree (no JIT cache).

    python -m paper_2003_12693_amd.build        # or build() from Python

Compiles csrc/*.hip with hipcc into paper_2003_12693_amd/_build/*.o and
links paper_2003_12693_amd/libsr.so.  Packed-FP32 instruction selection is
disabled for device code (-packed-fp32-ops) on purpose.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsr.so")
ARCH = os.environ.get("SR_OFFLOAD_ARCH", "gfx950")

SOURCES = ["sr_kernels.hip", "sr_fused.hip", "sr_fused_small.hip", "sr_fused_512.hip", "sr_fused_1024.hip",
           "sr_dct.hip", "sr_aos.hip", "sr_api.hip", "sr_noalloc.hip", "sr3d.hip", "cnn.hip"]
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only within one source expression, so a kernel's
    # rounding does not depend on how a template instance happens to be
    # unrolled (results stay bitwise independent of tile shapes)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]


def source_id():
    """Hex digest (16 digits) of every HIP source and header the library is
    built from, the C headers and the compiler flags.  Compiled into the
    library (sr_build_id), so a loaded libsr.so can be matched to a tree."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp"))
                   + glob.glob(os.path.join(ROOT, "include", "*.h")))
    for fn in files:
        h.update(os.path.basename(fn).encode())
        with open(fn, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(FLAGS[:-2] + [ARCH]).encode())
    return h.hexdigest()[:16]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm required to build libsr.so)")


def _compile(src, hipcc, sid):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc, *FLAGS, f'-DSR_BUILD_ID="{sid}"', "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def build(verbose=False):
    """Compile every HIP source for gfx950 and link libsr.so (always rebuilds)."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    sid = source_id()
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        results = list(ex.map(lambda s: _compile(s, hipcc, sid), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, w in results:
            if w:
                print(w, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
