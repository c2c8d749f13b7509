"""Build libsvdag.so (hipcc, gfx950) and the scene generator in-tree."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsvdag.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall", "-pthread",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# Packed FP32 instructions stay off: some of their forms have returned wrong
# results on this toolchain without any error.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = ["builder.cpp", "runtime.cpp", "server.cpp", "tune.cpp", "kernels.hip"]
# the sources whose hash keys tuned configurations and kernel profiles
KERNEL_SOURCES = ["kernels.hip", "svdag_internal.h"]


def kernel_source_hash() -> str:
    """First 16 hex digits of SHA-256 over the kernel sources, in order."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "not a recognized feature for this target" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError(f"build failed: {' '.join(cmd)}")
    if verbose and out.strip():
        print(out)


def build_lib(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    define = f'-DSVD_KERNEL_HASH="{kernel_source_hash()}"'
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        _run([HIPCC, *COMMON, *DEVICE, define, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", "-pthread", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


def build_all(verbose: bool = False):
    from . import scenes
    scenes.build(verbose)
    scenes.build_gpu(verbose)
    return build_lib(verbose)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    from paper_2505_02017_amd import build as b
    b.build_all(verbose=True)
