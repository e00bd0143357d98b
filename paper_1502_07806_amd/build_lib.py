"""Compile libpfsm.so (HIP, gfx950) in-tree.

    python -m paper_1502_07806_amd.build_lib

Every translation unit under csrc/ is compiled with hipcc for gfx950 and
linked into paper_1502_07806_amd/libpfsm.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpfsm.so")
HOOKS_LIB = os.path.join(HERE, "libpfsm_testhooks.so")
ARCH = "gfx950"

CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
    # packed FP32 instructions are excluded from code generation on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: libpfsm needs the ROCm HIP compiler")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [hipcc()] + CFLAGS + ["-I", os.path.join(HERE, "..", "include"), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-4000:]))
    return obj


def _link(objs, out):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, out)


def build(verbose: bool = True) -> str:
    """Build libpfsm.so (the product) and libpfsm_testhooks.so (same objects plus
    C entry points to internal kernels, used only by kernel-level tests)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    hooks = sorted(glob.glob(os.path.join(CSRC, "testhooks", "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs) + len(hooks))) as ex:
        objs = list(ex.map(_compile, srcs + hooks))
    _link(objs[:len(srcs)], LIB)
    _link(objs, HOOKS_LIB)
    if verbose:
        print("built", LIB, "and", HOOKS_LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
