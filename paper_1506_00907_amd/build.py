"""Build libdgrtm.so (the HIP library behind include/dgrtm.h) in-tree for gfx950.

Host set-up code is compiled with -ffp-contract=off so that the level assignment and the
other integer results of the set-up are reproducible; the kernels are compiled with packed
FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdgrtm.so")
ARCH = os.environ.get("DGRTM_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libdgrtm)")


def build(verbose: bool = False, jobs: int = 3) -> str:
    hipcc = _hipcc()
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}"]
    units = [
        ("setup.cpp", ["-ffp-contract=off"]),
        ("api.cpp", ["-ffp-contract=off"]),
        # every atomic in the kernels is issued by one lane; the wave-level atomic rewrite would read
        # the step kernel's tile counter back at once, behind the tile copies issued before it
        ("kernels.hip", ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                         "-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]),
        ("noalloc.hip", ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]),
    ]
    procs = []
    objs = []
    for src, flags in units:
        obj = os.path.join(bdir, src + ".o")
        objs.append(obj)
        cmd = [hipcc] + common + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd) + "\n" + out.decode(errors="replace"))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
