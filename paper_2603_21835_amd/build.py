"""Build libgint.so for gfx950 with hipcc (in-tree).

Each source is compiled to an object in its own hipcc process (in parallel),
then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgint.so")
SOURCES = ["gint_api.hip", "gint_kernels.hip", "gint_contract.hip", "gint_hr.hip", "gint_dphi.hip",
           "gint_sphere.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build(verbose: bool = True) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    with tempfile.TemporaryDirectory(prefix="gint_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[HIPCC, *FLAGS, "-c", s, "-o", o] for s, o in zip(srcs, objs)]
        with ThreadPoolExecutor(max_workers=min(len(cmds), 8)) as ex:
            rcs = list(ex.map(lambda c: _run(c, verbose), cmds))
        if any(rcs):
            raise RuntimeError("hipcc failed compiling libgint.so sources")
        tmp = OUT + ".tmp"
        if _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose):
            raise RuntimeError("hipcc failed linking libgint.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
