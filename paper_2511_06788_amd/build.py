"""Builds the gfx950 shared library ``libope.so`` from ``csrc/*.hip`` with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled, and the objects are linked into one shared library next to
this file.  ``python -m paper_2511_06788_amd.build`` runs it from the command
line.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libope.so")

SOURCES = ["k_stencil.hip", "k_mfma.hip", "k_small.hip", "k_net.hip", "k_check.hip", "k_mg.hip", "k_block.hip",
           "ope_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the packed-fp32 target feature; that warning is expected
    noise = ("packed-fp32-ops", "is not a recognized feature for this target")
    lines = [ln for ln in r.stdout.splitlines() if not any(t in ln for t in noise)]
    if r.returncode != 0:
        raise RuntimeError("command failed (%d): %s\n%s" % (r.returncode, " ".join(cmd), "\n".join(lines)))
    return "\n".join(lines)


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link ``libope.so``; returns its path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = [os.path.join(OUT_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[HIPCC, *CFLAGS, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
        logs = list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    logs.append(_run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]))
    os.replace(tmp, LIB)
    if verbose:
        for log in logs:
            if log.strip():
                print(log)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
