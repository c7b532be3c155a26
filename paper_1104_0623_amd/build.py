"""Builds libfind.so in-tree for gfx950 with hipcc.

    python -m paper_1104_0623_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfind.so")
# (source, extra flags): kernels.hip is compiled once per kernel family
SOURCES = [("plan.cpp", []), ("capi.hip", [])] + [("kernels.hip", [f"-DFIND_TU={k}"]) for k in (1, 2, 3, 4, 5, 6, 7)]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _compile(src: str, extra: list, obj: str) -> None:
    cmd = [HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")


def build(verbose: bool = False) -> str:
    """Compile every source and link libfind.so (always recompiles)."""
    from concurrent.futures import ThreadPoolExecutor
    tmp = tempfile.mkdtemp(prefix="findbuild_")
    try:
        objs = [os.path.join(tmp, f"{k}_{s}.o") for k, (s, _) in enumerate(SOURCES)]
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            list(ex.map(lambda p: _compile(p[0][0], p[0][1], p[1]), zip(SOURCES, objs)))
        out_tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out_tmp] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("link of libfind.so failed")
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
