"""Build the HIP library in-tree for gfx950 (``libtsat.so`` next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtsat.so")
ARCH = os.environ.get("TSAT_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = ["tsat_kernels.hip", "tsat_learned.hip"]
HOST_SOURCES = ["tsat_host.cpp", "tsat_mlp.cpp", "tsat_store.cpp"]
# hipcc's host pass does not know this device feature and warns; harmless.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed: {' '.join(cmd)}")


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-result"]
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        jobs.append((obj, [hipcc, f"--offload-arch={ARCH}", *common, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src),
                           "-o", obj]))
    for src in HOST_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        jobs.append((obj, [hipcc, *common, "-c", os.path.join(CSRC, src), "-o", obj]))
    # independent translation units: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(jobs), 4)) as ex:
        list(ex.map(_run, [cmd for _, cmd in jobs]))
    objs = [obj for obj, _ in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
