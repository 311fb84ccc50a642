"""Builds libacch.so (the HIP kernels and the C-ABI host driver) for gfx950 in place.

Each source is compiled to an object file in parallel (one hipcc per source), then
the objects are linked into the shared library."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libacch.so")
SOURCES = ["stencil2d.hip", "schwarz2d.hip", "bandlu2d.hip", "boxilu2d.hip", "krylov.hip", "adjoint2d.hip", "stencil3d.hip",
           "schwarz3d.hip", "noalloc.hip", "solver.cpp", "batch.cpp"]
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _clean(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source into libacch.so next to this file; returns its path."""
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    tmpdir = tempfile.mkdtemp(prefix="acch_build_")
    try:
        def compile_one(src):
            obj = os.path.join(tmpdir, src + ".o")
            cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            proc = subprocess.run(cmd, capture_output=True, text=True)
            return src, obj, proc.returncode, _clean(proc.stdout + proc.stderr)

        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(compile_one, SOURCES))
        for src, _, rc, out in results:
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src} ({rc}):\n{out}")
            if verbose and out.strip():
                print(out)
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for _, o, _, _ in results], "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        proc = subprocess.run(cmd, capture_output=True, text=True)
        if proc.returncode != 0:
            raise RuntimeError(f"link failed ({proc.returncode}):\n{_clean(proc.stdout + proc.stderr)}")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
