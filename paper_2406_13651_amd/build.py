"""Compile the HIP library libclamp.so for gfx950, in place next to this file.

Every translation unit is compiled with hipcc for gfx950 only, with packed
FP32 instructions disabled (-target-feature -packed-fp32-ops), then linked
into one shared library that the ctypes binding loads.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libclamp.so")
SOURCES = ["kernels.hip", "batch.hip", "range.hip", "regularizers.hip", "cnn.hip", "unet.hip", "api.cpp",
           "cnn_api.cpp", "unet_api.cpp"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("command failed (%d): %s\n%s" % (p.returncode, " ".join(cmd), p.stdout))
    return p.stdout


def build(verbose=False):
    """Compile every source and link libclamp.so; returns the library path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([hipcc()] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        outs = list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    outs.append(_run([hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs))
    os.replace(tmp, LIB)
    if verbose:
        for o in outs:
            if o.strip():
                sys.stdout.write(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
