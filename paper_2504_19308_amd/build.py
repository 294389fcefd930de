"""Build the HIP library ``libamm.so`` in-tree for gfx950.

Usage: ``python -m paper_2504_19308_amd.build`` (or ``build()`` from Python).
Every call recompiles all sources.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libamm.so")

SOURCES = ["amm_api.cpp", "amm_export.cpp", "host_logic.cpp", "cd_apply.hip", "cd_decomp.hip", "gemm.hip", "sparse.hip", "csc_build.hip", "cast.hip", "tsvd.hip", "rsvd_small.hip", "tsvd_apply.hip", "tsvd_split.hip", "tsvd_bf16.hip", "sfft.hip", "cd_general.hip", "backward.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed fp32 forms stay off: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False, jobs: int = 6) -> str:
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found")
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    pending = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        cmd = [HIPCC, *FLAGS]
        if src.endswith(".cpp"):
            cmd += ["-x", "hip"]
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        pending.append((src, obj, cmd))
    # compiler output goes to a log file per source (a full pipe would block)
    running, done, failed = [], [], []
    while pending or running:
        while pending and len(running) < jobs:
            src, obj, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            logf = open(os.path.join(objdir, src + ".log"), "w")
            running.append((src, obj, cmd, logf, subprocess.Popen(cmd, stdout=logf, stderr=subprocess.STDOUT)))
        src, obj, cmd, logf, proc = running.pop(0)
        rc = proc.wait()
        logf.close()
        (done if rc == 0 else failed).append((src, obj, cmd))
    if failed:
        for src, _, cmd in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + open(os.path.join(objdir, src + ".log")).read())
        raise RuntimeError("HIP compilation failed: " + ", ".join(f[0] for f in failed))
    objs = [os.path.join(objdir, src.rsplit(".", 1)[0] + ".o") for src in SOURCES]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
