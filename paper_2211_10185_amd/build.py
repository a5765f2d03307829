"""Compile the HIP sources of the solver into ``libqfdtd.so`` (gfx950), in-tree.

Usage: ``python -m paper_2211_10185_amd.build`` or ``build()`` from Python.
Objects go to ``paper_2211_10185_amd/_build/``; the shared library is written
next to this file, where the binding loads it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libqfdtd.so")
# (source, object name, extra flags): the transform passes are instantiated
# per lattice size in five groups so that they compile in parallel
SOURCES = [("fft_inst.hip", "fft_inst%d" % g, ["-DQF_GROUP=%d" % g]) for g in range(5)] + [
    ("aux_kernels.hip", "aux_kernels", []), ("qfdtd_api.hip", "qfdtd_api", []),
    ("potential_io.cpp", "potential_io", [])]
# The DFT-stage measurement tool (VALU butterfly against MFMA), a library of its own
STAGE_SOURCES = [("dft_stage_bench.hip", "dft_stage_bench", [])]
STAGE_OUT = os.path.join(HERE, "libdftstage.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code (see the
# target-feature pair below); the compiler then emits scalar FP32 VALU ops.
# -ffp-contract=off: no implicit mul+add fusion; the kernels spell out their
# FMAs, so every instantiation of a pass computes bit-identical results.
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), r.stdout))
    return r.stdout


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    libs = [(OUT, SOURCES), (STAGE_OUT, STAGE_SOURCES)]
    jobs = []
    for _, sources in libs:
        for src, name, extra in sources:
            obj = os.path.join(bdir, name + ".o")
            jobs.append((obj, [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]))
    with cf.ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        for out in ex.map(lambda j: _run(j[1]), jobs):
            if verbose and out.strip():
                print(out)
    for lib, sources in libs:
        tmp = lib + ".tmp"
        objs = [os.path.join(bdir, name + ".o") for _, name, _ in sources]
        _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
        os.replace(tmp, lib)
        if verbose:
            print("built", lib)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
