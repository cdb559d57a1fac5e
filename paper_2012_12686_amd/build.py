"""Build the HIP library ``libadorym.so`` for gfx950 in-tree.

Usage: ``python -m paper_2012_12686_amd.build`` (also run by
``__graft_entry__.build()``).  Compiles every ``csrc/*.hip`` unit in
parallel and links them into one shared library next to this file.
Packed-FP32 instructions are disabled (``-packed-fp32-ops``); float atomics
use the hardware instructions; multiply-add contraction is per expression.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libadorym.so")
ARCH = os.environ.get("ADORYM_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",
    # multiply-adds fused only within one source expression, so that kernels
    # with different code around the same arithmetic round identically
    "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning is harmless
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    return res.returncode, err


def build(verbose: bool = True, jobs: int = 0) -> str:
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                                          else os.cpu_count() or 1)), 16)
    with tempfile.TemporaryDirectory(prefix="adorym_build_") as tmp:
        objs, cmds = [], []
        for src in srcs:
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([HIPCC, *FLAGS, "-c", src, "-o", obj])
        if verbose:
            print(f"compiling {len(srcs)} units with {jobs} jobs: {' '.join(cmds[0][:-4])} ...", flush=True)
        with cf.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        for src, (rc, err) in zip(srcs, results):
            if rc != 0:
                sys.stderr.write(err)
                raise RuntimeError(f"hipcc failed on {src}")
        tmp_lib = LIB + ".tmp"
        rc, err = _run([HIPCC, "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp_lib])
        if rc != 0:
            sys.stderr.write(err)
            raise RuntimeError("link failed")
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    build()
