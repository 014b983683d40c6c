"""Shared test helpers: build-if-missing and oracle/GPU comparison utilities."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2106_02764_amd", "libobte.so")
HEADER = os.path.join(ROOT, "include", "obte.h")


def ensure_built():
    if not os.path.exists(LIB):
        from paper_2106_02764_amd import build
        build.build(verbose=False)
    return LIB


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(obte_[a-z0-9_]+)\s*\(", txt)))


def solid_to_full(prob, vec_solid):
    out = np.zeros(prob.mesh.n_cells)
    out[prob.mesh.cells] = vec_solid
    return out


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
