"""Compile the gfx950 solver library (libcbs.so) in-tree with hipcc.

The FFT pass kernels are compiled once per plan group (the axis lengths are
spread over several objects so the builds run in parallel).  Every
translation unit is built for gfx950 only, with packed-FP32 ALU
instructions disabled, then linked into one shared library that exports the C
ABI of include/cbs.h.  ``python -m paper_2507_16087_amd.build`` or
``paper_2507_16087_amd.build.build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcbs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["cbs_kernels.hip", "cbs_host.cpp", "cbs_noalloc.hip"]
# the FFT pass kernels, one object per plan group (see csrc/cbs_plans.h)
PLAN_GROUPS = 11
GROUP_SRC = "cbs_pass_group.hip"
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument",
          "-I", INCLUDE, "-I", CSRC]


def _compile(job, verbose: bool) -> str:
    src, group = job
    tag = src if group is None else f"{src}.g{group}"
    obj = os.path.join(OBJDIR, tag + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    defs = [] if group is None else [f"-DCBS_GROUP={group}"]
    cmd = [HIPCC] + COMMON + defs + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if verbose:
        print(f"{tag}: {time.time() - t0:.1f} s", flush=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    warn = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if verbose and warn:
        print("\n".join(warn[:40]))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = [(GROUP_SRC, g) for g in range(PLAN_GROUPS)] + [(s, None) for s in SOURCES]
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda j: _compile(j, verbose), jobs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
