"""Builds libsieve.so (HIP, gfx950) in-tree with hipcc.

Every source under csrc/ is compiled for gfx950 only.  Packed-FP32 VALU
instructions are disabled for all device code (the kernels are integer work;
the flag keeps the compiler from forming them anywhere).

A second library, libsieve_markcount.so, is the same sources built with
SIEVE_MARK_COUNT: its kernels also tally the marks they make
(include/sieve_debug.h), for the test of marking completeness.  The product
path never loads it.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsieve.so")
LIB_MARKCOUNT = os.path.join(HERE, "libsieve_markcount.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["api.hip", "kernels.hip", "server.hip", "stream.hip", "lds_probe.hip", "wide.hip"]

COMMON = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def _compile(src: str, obj: str, defs: tuple) -> None:
    cmd = [HIPCC, *COMMON, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on %s" % src)


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    """Compiles every HIP source and links libsieve.so (and the mark-counting
    build libsieve_markcount.so); returns the path of libsieve.so."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    variants = [(LIB, os.path.join(ROOT, "_build"), ()),
                (LIB_MARKCOUNT, os.path.join(ROOT, "_build", "markcount"), ("-DSIEVE_MARK_COUNT",))]
    jobs = []
    for _, objdir, defs in variants:
        os.makedirs(objdir, exist_ok=True)
        jobs += [(s, os.path.join(objdir, s.replace(".hip", ".o")), defs) for s in srcs]
    with ThreadPoolExecutor(max_workers=min(len(jobs), 8)) as ex:
        list(ex.map(lambda j: _compile(*j), jobs))
    for lib, objdir, _ in variants:
        _link([os.path.join(objdir, s.replace(".hip", ".o")) for s in srcs], lib)
        if verbose:
            print("built", lib)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
