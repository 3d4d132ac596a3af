"""Builds libemt.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1903_01081_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libemt.so")
BUILD = os.path.join(PKG, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, object name, extra flags): the step kernels compile once per
# workgroup size so the three builds run in parallel.
SOURCES = [
    ("analysis.cpp", "analysis", []),
    ("api.cpp", "api", []),
    ("aux.hip", "aux", []),
    ("step.hip", "step64", ["-DEMT_BS=64"]),
    ("step.hip", "step256", ["-DEMT_BS=256"]),
    ("step.hip", "step512", ["-DEMT_BS=512"]),
    ("split.hip", "split", []),
    ("scratch.hip", "scratch", []),
    ("steady.hip", "steady", []),
    ("floor.hip", "floor", []),
    ("comp_plan.cpp", "comp_plan", []),
    ("comp.hip", "comp", []),
]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # identical formulas must round identically in every code path
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def _compile(spec) -> str:
    src, name, extra = spec
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, name + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def build(verbose: bool = False) -> str:
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
