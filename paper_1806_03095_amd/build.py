"""Builds the HIP library libdgns.so for gfx950 in-tree.

    python -m paper_1806_03095_amd.build [--jobs N]

Every translation unit is compiled with hipcc for gfx950 only; packed-FP32
instructions are disabled for all device code.  Object files go to
paper_1806_03095_amd/_build/, the library to paper_1806_03095_amd/libdgns.so.
The compiler's per-kernel resource report (registers, spills, LDS) of each unit is
kept beside its object file as <unit>.resources.txt.
"""

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libdgns.so")

SOURCES = ["dgns_api.cpp", "setup.cpp", "aux_kernels.hip"] + ["op_k%d.hip" % k for k in range(1, 8)] + \
    ["op_hd0.hip", "op_hd1.hip", "op_hd2.hip"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC,
         "-Wno-unused-command-line-argument", "-Rpass-analysis=kernel-resource-usage"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    with open(os.path.splitext(obj)[0] + ".resources.txt", "w") as f:
        f.write(r.stderr)
    return obj


def build(jobs=None, verbose=False):
    """Compiles every source and links libdgns.so; always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-6000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    args = ap.parse_args()
    build(args.jobs, verbose=True)
    sys.exit(0)
