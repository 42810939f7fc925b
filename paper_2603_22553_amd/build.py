"""Builds liblpc.so (the HIP C-ABI library) in-tree for gfx950 with hipcc.

The translation units compile in parallel into objects (the sweep in five parts, see
LPC_SWEEP_PART in csrc/sweep.hip), which are then linked into one shared library.
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
LIB = os.path.join(PKG, "liblpc.so")
# (source, extra defines) per translation unit
UNITS = [("api.hip", []), ("analysis.hip", [])] + [
    ("sweep.hip", [f"-DLPC_SWEEP_PART={k}"]) for k in range(5)]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay off: hipcc would otherwise form them from float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=(), jobs: int | None = None) -> str:
    """Compile every source for gfx950 into paper_2603_22553_amd/liblpc.so (always rebuilds)."""
    cc = hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = jobs or max(1, min(len(UNITS), os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="lpc_build_") as tmp:
        objs, cmds = [], []
        for k, (src, defs) in enumerate(UNITS):
            obj = os.path.join(tmp, f"{k}_{os.path.splitext(src)[0]}.o")
            objs.append(obj)
            cmds.append([cc, *HIP_FLAGS, *extra, *defs, *inc, "-c", os.path.join(CSRC, src),
                         "-o", obj])

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(run, cmds))
        for cmd, r in zip(cmds, results):
            if r.returncode != 0:
                sys.stderr.write(r.stderr)
                raise subprocess.CalledProcessError(r.returncode, cmd)
            if verbose and r.stderr:
                sys.stderr.write(r.stderr)
        out = LIB + ".tmp"
        subprocess.run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out],
                       check=True)
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
