"""Shared helpers of the test suite (no GPU arithmetic here)."""

import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clamp.h")
LIB = os.path.join(ROOT, "paper_2406_13651_amd", "libclamp.so")


def header_functions():
    """Names of the functions include/clamp.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(clamp_[a-z_]+)\s*\(", text)))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def report(name, value, bound):
    """Print a parity figure so the run log states the error per result."""
    print("PARITY %-48s rel_l2=%.3e bound=%.1e" % (name, value, bound), flush=True)
    return value
