"""Build libkry.so (the gfx950 HIP library behind include/kry.h) in-tree.

    python -m paper_1804_01583_amd.build [--resource-usage]

Compiles every source under csrc/ with hipcc for gfx950 and links them into
paper_1804_01583_amd/libkry.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libkry.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["kry_api.cpp", "kry_lanczos.hip", "kry_arnoldi.hip", "kry_expm.hip", "kry_block.hip", "kry_dense.hip", "kry_sell.hip", "kry_errctl.hip", "kry_lz1.hip",
           "kry_lp.hip", "kry_wide.hip", "kry_tune.cpp", "kry_errbig.hip", "kry_small.hip"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, resource_usage: bool) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    cmd = [hipcc()] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    if resource_usage and src.endswith(".hip"):
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if resource_usage and err:
        print(err)
    return obj


def build(resource_usage: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, resource_usage), SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(resource_usage="--resource-usage" in sys.argv)
