"""Builds librbc.so for gfx950 in-tree (paper_1103_2635_amd/librbc.so).

Each tile source is compiled once per 16-feature slab count (-DRBC_KS=1..8) so
the objects build in parallel; everything is linked into one shared library
with a plain C ABI (include/rbc.h).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librbc.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
         # packed fp32 VALU forms stay off (hipcc builds them from plain float code)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]

PER_KS = ["k_tile_mfma.hip", "k_tile_valu.hip"]
PER_KB = ["k_tile_lowp.hip"]
# The item queue's ticket is taken by one lane and consumed an item later;
# the atomic optimizer would read it back at once (it broadcasts the result
# for a per-lane prefix), which puts the queue latency back on the critical
# path.  The tile files have no other atomics it would help.
TILE_FLAGS = ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]
SINGLE = ["k_util.hip", "k_finalize.hip", "k_rbc.hip", "k_oneshot.hip", "k_quant.hip", "rbc_dispatch.cpp", "rbc_api.cpp",
          "rbc_index.cpp", "rbc_timer.cpp", "rbc_tune.cpp"]


def _units():
    units = []
    for src in PER_KS:
        for ks in range(1, 9):
            obj = os.path.join(BUILD, "%s.ks%d.o" % (os.path.splitext(src)[0], ks))
            units.append((src, obj, ["-DRBC_KS=%d" % ks] + TILE_FLAGS))
    for src in PER_KB:
        for kb in range(1, 5):
            obj = os.path.join(BUILD, "%s.kb%d.o" % (os.path.splitext(src)[0], kb))
            units.append((src, obj, ["-DRBC_KB=%d" % kb] + TILE_FLAGS))
    for src in SINGLE:
        if os.path.exists(os.path.join(CSRC, src)):
            units.append((src, os.path.join(BUILD, os.path.splitext(src)[0] + ".o"), []))
    return units


def _compile(unit):
    src, obj, extra = unit
    cmd = [HIPCC] + FLAGS + extra + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
    os.replace(obj + ".tmp", obj)
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile every HIP source for gfx950 and link librbc.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
