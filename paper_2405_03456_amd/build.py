"""Build the HIP library libhm.so for gfx950 in-tree.

Host translation units are compiled with -ffp-contract=off so that the
layout's geometric predicates round exactly as written.  Device code is built
for gfx950 only, with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhm.so")
ARCH = os.environ.get("HM_OFFLOAD_ARCH", "gfx950")

# every translation unit of csrc/: host C++ (*.cpp) and device code (*.hip)
HOST_SRCS = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
DEVICE_SRCS = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-ffp-contract=off"]
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("build failed: " + " ".join(cmd))
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link libhm.so.  Always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    inc = ["-I", os.path.join(HERE, "..", "include"), "-I", CSRC]
    jobs = []
    for s in HOST_SRCS:
        o = os.path.join(BUILD, s + ".o")
        jobs.append((o, [hipcc, *COMMON, *inc, "-c", os.path.join(CSRC, s), "-o", o]))
    for s in DEVICE_SRCS:
        o = os.path.join(BUILD, s + ".o")
        jobs.append((o, [hipcc, *COMMON, *DEVICE_FLAGS, *inc, "-x", "hip", "-c", os.path.join(CSRC, s), "-o", o]))
    # translation units compile in parallel (the device ones dominate)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(len(jobs), max(1, os.cpu_count() or 1))) as ex:
        list(ex.map(lambda j: _run(j[1]), jobs))
    objs = [o for o, _ in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
