"""Build the mapcore HIP library for gfx950 (in-tree: ``paper_2412_00291_amd/libmapcore.so``).

Steps: generate the marching-cubes case table from its rule, compile every ``csrc/*.hip``
with hipcc for gfx950 (no fp contraction, no packed fp32), link one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "generated")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmapcore.so")
INCLUDE = os.path.join(ROOT, "include")
SOURCES = ["runtime.hip", "k_integrate.hip", "k_mesh.hip", "k_query.hip", "k_batch.hip", "k_range.hip",
           "k_quality.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC, "-I", GEN]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(GEN, exist_ok=True)
    os.makedirs(OBJ, exist_ok=True)
    _run([sys.executable, os.path.join(CSRC, "gen_mc_table.py"), os.path.join(GEN, "mc_table.inc")])
    objs = []
    jobs = []
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        for src in SOURCES:
            obj = os.path.join(OBJ, src.replace(".hip", ".o"))
            objs.append(obj)
            jobs.append(ex.submit(_run, [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]))
        for j in jobs:
            out = j.result()
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
