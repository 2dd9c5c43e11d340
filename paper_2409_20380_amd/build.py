"""Build the gfx950 shared library ``libebe.so`` in-tree with hipcc.

Usage: ``python -m paper_2409_20380_amd.build`` (also called by the
repository's ``__graft_entry__.build()``).  Always recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libebe.so")
SOURCES = ["topology.cpp", "kernels.hip", "mlp.hip", "batch.hip", "api.hip", "batch_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, extra_flags=None) -> str:
    flags = FLAGS + list(extra_flags or [])
    tmpdir = tempfile.mkdtemp(prefix="ebe_build_")
    try:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            path = os.path.join(CSRC, src)
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = [HIPCC] + flags + lang + ["-c", path, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
            objs.append(obj)
        tmp_lib = LIB + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
