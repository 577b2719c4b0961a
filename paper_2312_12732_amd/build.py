"""Build the mf shared library (libmf.so) for gfx950 with hipcc.

Usage: python -m paper_2312_12732_amd.build   (or call ``build()``)

Every HIP source is compiled for gfx950 only, with the packed-FP32 target
feature disabled (the compiler still emits ordinary FP32/FP64 code).
Objects go to ``_build/`` at the repository root; the library is written next
to this file so that it travels with the package.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libmf.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str, defines=()) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    # hipcc treats .cpp files as HIP too; give every file the gfx950 target so
    # that no device pass runs for the compiler's default architecture.
    cmd = [HIPCC, *COMMON, *defines, "-x", "hip", *DEVICE]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, defines=()) -> str:
    """Compile every source and link libmf.so; returns its path.  defines:
    extra -D options (tuning experiments)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda f: _compile(f, tuple(defines)), sources()))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", *DEVICE, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, defines=[a for a in sys.argv[1:] if a.startswith("-D")])
    sys.exit(0)
