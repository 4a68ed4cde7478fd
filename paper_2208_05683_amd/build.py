"""Build libfps.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2208_05683_amd.build

The library is written for gfx950 (MI355X) only.  Packed-FP32 instructions
are disabled for all device code; floating-point contraction is off so every
fused multiply-add in the kernels is one that the source spells out.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfps.so")
SOURCES = ["fps_kernels.hip", "fps_normest.hip", "fps_batch.hip", "fps_dense.hip", "fps_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libfps)")


def compile_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC, "-Wall",
    ]


def build(verbose: bool = False, jobs: int = 2) -> str:
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="fps_build_") as tmp:
        objs = []
        procs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmd = [cc, *compile_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
            objs.append(obj)
        for p, src in procs:
            _, err = p.communicate()
            err = "\n".join(x for x in err.splitlines() if "packed-fp32-ops" not in x)
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{err}")
            if err.strip() and verbose:
                print(err, file=sys.stderr)
        tmp_lib = os.path.join(tmp, "libfps.so")
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        shutil.copyfile(tmp_lib, LIB + ".tmp")
        os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
