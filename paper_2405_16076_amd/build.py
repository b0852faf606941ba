"""Builds librid.so (the HIP library behind include/rid.h) for gfx950.

Usage: python -m paper_2405_16076_amd.build   (or build() from Python).
Every HIP source under csrc/ is compiled with hipcc and linked into one shared
library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "librid.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # keep binary32 arithmetic out of the packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(verbose=False, jobs=None):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    srcs = sources()
    with tempfile.TemporaryDirectory(prefix="rid_build_") as tmp:
        objs = []
        procs = []
        for s in srcs:
            o = os.path.join(tmp, os.path.basename(s) + ".o")
            cmd = [hipcc, *HIPCC_FLAGS, "-I", INCLUDE, "-c", s, "-o", o]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(o)
        failed = []
        for s, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            if p.returncode != 0:
                failed.append((s, text))
            elif verbose and text.strip():
                print(text)
        if failed:
            for s, text in failed:
                print(f"--- {s}\n{text}", file=sys.stderr)
            raise RuntimeError("hipcc failed for " + ", ".join(os.path.basename(s) for s, _ in failed))
        tmp_lib = LIB + ".tmp"
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
