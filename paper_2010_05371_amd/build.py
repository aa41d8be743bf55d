"""Builds libeapdtw.so (gfx950) from csrc/ with hipcc, compiling translation
units in parallel.  Usage: python -m paper_2010_05371_amd.build [-j N]."""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libeapdtw.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# -ffp-contract=off: every multiply-add the kernels want is an explicit fma,
# so all code paths round identically.  Packed FP32 is disabled.
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + CSRC, "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]

# window ranges of the band-kernel instantiations (one object each)
BAND_RANGES = [(0, 7), (8, 13), (14, 18), (19, 23), (24, 27), (28, 31), (32, 35), (36, 39),
               (40, 43), (44, 47), (48, 51), (52, 55), (56, 58), (59, 61), (62, 64)]


# translation units that compile longest, started first so that the pool of
# compilers does not end waiting on one of them
SLOW_FIRST = ("wide_inst.hip", "wf.hip", "batch.hip", "lanes.hip")


def _units():
    others = [src for src in sorted(os.listdir(CSRC))
              if src != "band_inst.hip" and (src.endswith(".hip") or src.endswith(".cpp"))]
    others.sort(key=lambda src: (src not in SLOW_FIRST,
                                 SLOW_FIRST.index(src) if src in SLOW_FIRST else 0))
    units = [(src, os.path.splitext(src)[0] + ".o", []) for src in others
             if src in SLOW_FIRST]
    for lo, hi in BAND_RANGES[::-1]:  # the widest windows compile longest
        units.append(("band_inst.hip", f"band_r{lo:02d}_{hi:02d}.o",
                      [f"-DEAPDTW_R_LO={lo}", f"-DEAPDTW_R_HI={hi}"]))
    units += [(src, os.path.splitext(src)[0] + ".o", []) for src in others
              if src not in SLOW_FIRST]
    return units


def _compile(unit):
    src, obj, extra = unit
    out = os.path.join(BUILD, obj)
    cmd = [HIPCC, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    p = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (p.stdout + p.stderr).splitlines()
            if "is not a recognized feature for this target" not in ln]
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
    return out, "\n".join(msgs)


def build(jobs: int | None = None, verbose: bool = False) -> str:
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found")
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or max(1, min(16, len(os.sched_getaffinity(0))))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out, msgs in ex.map(_compile, _units()):
            objs.append(out)
            if verbose and msgs.strip():
                print(msgs, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    args = ap.parse_args()
    print(build(args.j, args.v))
