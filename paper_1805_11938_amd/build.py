"""Build the native parts of the package in-tree.

* ``synth/libsynth.so``  -- seeded input generators (gcc, OpenMP)
* ``libspmv.so``         -- the SpMV library: HIP kernels for gfx950 plus the
  C-ABI declared in ``include/spmv.h`` (hipcc)
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
ARCH = os.environ.get("SPMV_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


def _run(cmd, cwd=None):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} ({r.returncode})")
    return r


def build_synth() -> str:
    src = os.path.join(PKG, "synth", "synth.c")
    out = os.path.join(PKG, "synth", "libsynth.so")
    _run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", out + ".tmp", src, "-lm"])
    os.replace(out + ".tmp", out)
    return out


def build_spmv(jobs: int = 8) -> str | None:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    if not srcs:
        return None
    objdir = os.path.join(ROOT, "_build", "obj")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        cmd = ["hipcc", *HIPCC_FLAGS, "-x", "hip", "-c", s, "-o", o]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    out = os.path.join(PKG, "libspmv.so")
    _run(["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", out + ".tmp", *objs])
    os.replace(out + ".tmp", out)
    return out


def _drain(procs):
    failed = None
    for cmd, p in procs:
        outp, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(" ".join(cmd) + "\n" + outp)
            failed = cmd
    procs.clear()
    if failed:
        raise RuntimeError(f"hipcc failed on {failed[-3]}")


def build() -> None:
    build_synth()
    build_spmv()


if __name__ == "__main__":
    build()
    print("built")
