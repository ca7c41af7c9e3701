"""Build libprhip.so (hipcc, gfx950) in-tree, next to this file."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
SO = os.path.join(PKG, "libprhip.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = [os.path.join(CSRC, "prhip.hip"), os.path.join(CSRC, "apply.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.h", "wave.h", "apply.h")] + [
    os.path.join(INCLUDE, "prhip.h")]

# -ffp-contract=off: every product and sum rounds as written, so the lane
# class reproduces a sequential FP64 sum bit for bit. Packed FP32 ops are
# disabled (no packed-math forms in the generated code).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC, "-o", tmp, *SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose and (r.stdout or r.stderr):
        print(r.stdout + r.stderr)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
