"""Build the HIP library (gfx950) in-tree: paper_2208_01339_amd/libppcg.so.

    python -m paper_2208_01339_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("pp_lib.hip", "pp_batch.hip", "pp_mlp.hip", "pp_noalloc.hip")]
DEPS = SRC + [os.path.join(HERE, "csrc", f) for f in (
    "kernels.hpp", "sym_eig.hpp", "persistent.hpp", "batch.hpp", "common.hpp", "op.hpp", "mlp.hpp", "dfn.hpp",
    "dia_plan.hpp", "lowrank.hpp", "stencil2.hpp")] + [
    os.path.join(ROOT, "include", "pp.h")]
OUT = os.path.join(HERE, "libppcg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-fvisibility=hidden",
    # hipcc -O3 forms packed FP32 instructions by itself; keep them off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = True) -> str:
    """Compile the translation units in parallel (one hipcc each), then link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs, objs = [], []
    for src in SRC:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *compile_flags, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


def stale() -> bool:
    if not os.path.exists(OUT):
        return True
    t = os.path.getmtime(OUT)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    build()
    sys.exit(0)
