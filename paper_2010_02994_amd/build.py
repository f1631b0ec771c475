"""Build libhawkes.so for gfx950 in-tree with hipcc (no JIT, no torch extension)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhawkes.so")
PEAKS = os.path.join(HERE, "peaks")

# Packed FP32 VALU ops are disabled on purpose: the compiler may form them from
# scalar float code, and the library does not rely on them.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops"]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build_library() -> str:
    srcs = [os.path.join(CSRC, f) for f in ("hawkes.hip", "serve.hip", "mwg.hip", "hmc.hip", "bmds.hip", "noalloc.hip")]
    tmp = LIB + ".tmp"
    _run([_hipcc(), *HIPFLAGS, "-fPIC", "-shared", "-lpthread", *srcs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def build_peaks() -> str:
    _run([_hipcc(), *HIPFLAGS, os.path.join(CSRC, "peaks.hip"), "-o", PEAKS])
    return PEAKS


def build_all() -> None:
    build_library()
    build_peaks()


if __name__ == "__main__":
    build_all()
    print(LIB)
