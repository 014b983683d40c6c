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


def on_node_modes(w):
    """A copy of workload `w` whose material is a mode table with one mode on
    every grid node, F_ml = Lambda_m s_l, weighted by the oracle's own grid
    weights alpha_ml (so the interpolation onto the grid is the identity)."""
    import dataclasses
    from oracle.material import material_weights
    wts = material_weights(w.mfp, w.dirs, w.dir_w, w.kappa_m, w.grad_axis)
    F = (w.mfp[:, None, None] * w.dirs[None, :, :]).reshape(-1, w.ndim)
    return dataclasses.replace(w, modes=(F, wts["alpha"].ravel()), name=w.name + "_nodes")
