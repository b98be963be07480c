"""Build libpimm.so for gfx950 in-tree with hipcc (host pieces that need quad
precision are compiled with g++)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpimm.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIP_SOURCES = ["context.hip", "client.hip", "server.hip", "mac.hip", "batch.hip", "serve.hip",
               "tune.hip", "profile.hip", "probe.hip", "fc.hip", "noalloc.hip", "mfma.hip", "select.hip",
               "switch.hip"]
HOST_SOURCES = ["cdt.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    # Native FP64 atomic add for the product's split tiles (hipMalloc memory is
    # coarse-grained, where the hardware instruction is valid).
    "-munsafe-fp-atomics",
    # Packed FP32 instructions are kept out of every kernel.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    procs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, "-I" + INCLUDE, "-I" + CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
        while len([p for p, _ in procs if p.poll() is None]) >= jobs:
            procs[0][0].wait()
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        run(["g++", "-O2", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-c",
             os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for p, src in procs:
        err = p.communicate()[1]
        # hipcc's host pass does not know the packed-FP32 feature switch; that note is noise.
        lines = [ln for ln in err.splitlines() if "packed-fp32-ops" not in ln]
        if lines and (verbose or p.returncode != 0):
            print("\n".join(lines), file=sys.stderr)
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}")
    tmp = LIB + ".tmp"
    run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
         "-lquadmath"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
