"""Builds libifmm.so (HIP, gfx950) in the package directory.

Host C++ is compiled without floating-point contraction so that the octree
keys are reproducible bit for bit; device code is compiled with packed FP32
disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
INC = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libifmm.so")
BUILD = os.path.join(HERE, "_build")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-I", INC, "-I", SRC, "-Wall", "-Wno-unused-function",
              "-Wno-unused-variable", "-Wno-unused-parameter"]
    objs = []
    jobs = [
        ("tree.cpp", ["-x", "c++", "-ffp-contract=off"]),
        ("capi.cpp", ["-x", "c++", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]),
        # matrix-core accumulators in ordinary VGPRs (no copies to and from
        # the accumulation registers around every k-chunk of the GEMM tiles)
        ("engine.hip", ["-x", "hip", "--offload-arch=gfx950", "-ffp-contract=fast",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-mllvm", "-amdgpu-mfma-vgpr-form=1"]),
        ("fmm.hip", ["-x", "hip", "--offload-arch=gfx950", "-ffp-contract=fast",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]),
        ("mlp.hip", ["-x", "hip", "--offload-arch=gfx950", "-ffp-contract=fast",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]),
    ]
    procs = []
    for src, extra in jobs:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [cc] + common + extra + ["-c", os.path.join(SRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        msg = "\n".join(f"--- {s}\n{t}" for s, t in failed)
        raise RuntimeError("HIP build failed:\n" + msg)
    tmp = OUT + ".tmp"
    cmd = [cc, "-shared", "--offload-arch=gfx950", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
