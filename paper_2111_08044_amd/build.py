"""Builds the native library libfloquet.so in-tree with hipcc for gfx950.

    python -m paper_2111_08044_amd.build        (from the repo root)

Every source is compiled each call (objects go to a temporary folder), then
linked into paper_2111_08044_amd/libfloquet.so (the engine) and
paper_2111_08044_amd/libflprobe.so (measurement probes).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfloquet.so")

SOURCES = ["kernels.hip", "noalloc.hip", "capi.cpp", "host_math.cpp", "planner.cpp"]
# measurement probes (csrc/probe.h), a library of their own
PROBE_SOURCES = ["probe.hip"]
PROBE_LIB = os.path.join(PKG, "libflprobe.so")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU ops.
HIPFLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libfloquet.so")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    tmp = tempfile.mkdtemp(prefix="fl_build_")
    try:
        def compile_one(src):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = [hipcc, *HIPFLAGS, "-I", INCLUDE, "-I", CSRC, *lang, "-c",
                   os.path.join(CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
            if verbose and r.stderr.strip():
                print(r.stderr, file=sys.stderr)
            return obj

        with ThreadPoolExecutor(max_workers=min(4, len(SOURCES) + len(PROBE_SOURCES))) as ex:
            objs = list(ex.map(compile_one, SOURCES + PROBE_SOURCES))
        for lib, lib_objs in ((LIB, objs[:len(SOURCES)]), (PROBE_LIB, objs[len(SOURCES):])):
            out_tmp = lib + ".tmp"
            cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *lib_objs, "-o", out_tmp]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"link of {os.path.basename(lib)} failed:\n{r.stdout}\n{r.stderr}")
            os.replace(out_tmp, lib)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
