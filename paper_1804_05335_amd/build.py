"""Build ``libfdas.so`` (HIP, gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (``-packed-fp32-ops``): the compiler would otherwise
form v_pk_*_f32 from ordinary float code, and those are kept out of this
library.  Implicit FMA contraction is off (``-ffp-contract=off``): the
kernels spell out every fused multiply-add, so each instantiation of the
shared FFT code rounds identically (the plain, batched and interbinned
planes agree bit for bit).  Run ``python -m paper_1804_05335_amd.build`` or
call ``build()``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfdas.so")
SOURCES = ["fdas_api.cpp", "fdas_templates.cpp", "fdas_tune.cpp", "fdas_kernels.hip",
           "fdas_r2c.hip", "fdas_harmonic.hip", "fdas_stream.hip"]

ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-ffp-contract=off",
          "-I", os.path.join(ROOT, "include"),
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the FDAS library needs ROCm to build")
    return path


def build(verbose: bool = False) -> str:
    """Compile all sources and link libfdas.so (always rebuilds)."""
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="fdas_build_") as tmp:
        cmds, objs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            cmd = [cc, f"--offload-arch={ARCH}", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
            if src.endswith(".cpp"):
                cmd.insert(1, "-x")
                cmd.insert(2, "hip")
            if verbose:
                print(" ".join(cmd), flush=True)
            cmds.append(cmd)
            objs.append(obj)
        # the sources compile independently: one compiler process each
        workers = max(1, min(len(cmds), os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            for r in ex.map(lambda c: subprocess.run(c, check=True), cmds):
                pass
        out_tmp = LIB + f".tmp{os.getpid()}"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
