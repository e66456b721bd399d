"""Build libmgrav.so in-tree: HIP kernels for gfx950 plus the host-side
tree builder (g++ with OpenMP).  Run ``python paper_1609_08621_amd/build.py``
(by path: importing the package loads the library this replaces)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmgrav.so")
ARCH = os.environ.get("MGRAV_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions stay disabled in all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def source_digest() -> str:
    """First 16 hex digits of the SHA-256 of the kernel sources (csrc/*.hip,
    *.inc, *.h, in name order) and the public header: identifies the build
    in the autotuning cache."""
    import hashlib
    h = hashlib.sha256()
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".inc", ".h")))
    for f in names + ["../../include/mgrav.h"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True, out: str = LIB, extra_flags=()) -> str:
    """Compile and link libmgrav.so (``extra_flags`` go to the HIP compile,
    e.g. -DMGRAV_PP_CHUNK=64 for a tuning variant written to ``out``)."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    tree_o = os.path.join(bdir, "tree_host.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-fopenmp", "-ffp-contract=off", "-Wall",
          "-c", os.path.join(CSRC, "tree_host.cpp"), "-o", tree_o])
    dev_o = os.path.join(bdir, "mgrav.o")
    digest = f'-DMGRAV_SOURCE_DIGEST="{source_digest()}"'
    _run(["hipcc", *HIP_FLAGS, digest, *extra_flags, "-c", os.path.join(CSRC, "mgrav.hip"),
          "-o", dev_o])
    tmp = out + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, dev_o, tree_o,
          "-lgomp"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
