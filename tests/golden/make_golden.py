"""Write the oracle's reference values for the full-size workloads.

Calls only the CPU oracle (oracle/) on the seeded inputs (inputs/gen.py) and
stores kappa_cc, kappa_face, kappa_fourier, per-MFP kappa and T_L at seeded
sample cells, and the full T_L and J fields (every cell; pores 0) in
<config>_fields.npz.  Run:  python tests/golden/make_golden.py cfg2 [--workers 8]

``cfg5r_adjoint`` stores d kappa / d sigma of that replica at sigma = 1.
``cfg5r`` is the 3D membrane at 16x16x4 cells with the full direction and MFP
sets (the reduced replica of the 64x64x16 case).
``cfg3`` stores kappa_cc / kappa_face of the members of the 64-geometry batch
whose grids are 48x48 or 64x64 (the oracle's cost grows quickly with the grid);
``cfg3big`` those of four larger members, one or more per row width of the
GPU launch classes: 128x128 (#54), 192x192 (#12) and 256x256 (#15, #5).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from inputs import gen  # noqa: E402
from oracle.parallel import source_iteration_parallel  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["cfg2", "cfg3", "cfg3big", "cfg4", "cfg5r", "cfg5r_adjoint"])
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-11)
    a = ap.parse_args()
    if a.config == "cfg3":
        return batch(a)
    if a.config == "cfg3big":
        return batch(a, members=BIG_MEMBERS, name="cfg3big")
    if a.config == "cfg5r_adjoint":
        return adjoint_replica(a)
    w = {"cfg2": gen.config2, "cfg4": gen.config4,
         "cfg5r": lambda: gen.config5(nx=16, nz=4)}[a.config]()
    t0 = time.time()
    r = source_iteration_parallel(w, n_workers=a.workers, tol=a.tol, verbose=True)
    cells = np.nonzero(w.solid.ravel())[0]
    rng = np.random.default_rng(7)
    pick = np.sort(rng.choice(len(cells), size=64, replace=False))
    out = {
        "config": a.config, "source": "oracle.parallel.source_iteration_parallel (FP64, SuperLU per system)",
        "tol": a.tol, "passes": r["passes"], "converged": bool(r["converged"]),
        "kappa_cc": r["kappa_cc"], "kappa_face": r["kappa_face"], "kappa_fourier": r["kappa_fourier"],
        "kappa_per_mfp": list(map(float, r["kappa_per_mfp"])),
        "T_L_sample_cells": [int(cells[i]) for i in pick],
        "T_L_sample": [float(r["T_L"][i]) for i in pick],
        "history_tail": list(map(float, r["history"][-5:])),
        "seconds": time.time() - t0,
        "fields": f"{a.config}_fields.npz",
    }
    here = os.path.dirname(os.path.abspath(__file__))
    T_full = np.zeros(w.n_cells)
    T_full[cells] = r["T_L"]
    J_full = np.zeros((w.n_cells, w.ndim))
    J_full[cells] = r["J"]
    np.savez_compressed(os.path.join(here, f"{a.config}_fields.npz"), T_L=T_full, J=J_full)
    path = os.path.join(here, f"{a.config}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["kappa_cc"], out["passes"])


def adjoint_replica(a):
    """d kappa / d sigma of the 16x16x4 membrane replica at sigma = 1 (serial
    oracle: forward source iteration, then the transposed one)."""
    from oracle.adjoint import adjoint_source_iteration
    from oracle.bte import Problem, source_iteration
    w = gen.config5(nx=16, nz=4)
    t0 = time.time()
    prob = Problem(w)
    r = source_iteration(prob, tol=a.tol)
    ad = adjoint_source_iteration(prob, r["T"], tol=a.tol)
    g = np.zeros(w.n_cells)
    g[prob.mesh.cells] = ad["grad"]
    out = {"config": "cfg5r_adjoint", "tol": a.tol, "passes_forward": r["passes"],
           "passes_adjoint": ad["passes"], "kappa_cc": r["kappa_cc"], "kappa_adj": ad["kappa_adj"],
           "grad": list(map(float, g)), "seconds": time.time() - t0,
           "source": "oracle.bte.source_iteration + oracle.adjoint.adjoint_source_iteration (FP64)"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg5r_adjoint_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, r["kappa_cc"], ad["kappa_adj"])


BIG_MEMBERS = (54, 12, 15, 5)


def batch(a, members=None, name="cfg3"):
    geoms = gen.config3()
    picked = members
    members = []
    t0 = time.time()
    for g, w in enumerate(geoms):
        if picked is None and w.n[0] > 64:
            continue
        if picked is not None and g not in picked:
            continue
        r = source_iteration_parallel(w, n_workers=a.workers, tol=a.tol)
        h = r["history"]
        members.append({"index": g, "n": w.n[0], "L": w.L[0], "passes": r["passes"],
                        "converged": bool(r["converged"]), "kappa_cc": r["kappa_cc"],
                        "kappa_face": r["kappa_face"], "kappa_fourier": r["kappa_fourier"],
                        "history_tail": list(map(float, h[-4:]))})
        print(g, w.n[0], r["passes"], r["kappa_cc"], flush=True)
    out = {"config": name, "tol": a.tol, "members": members, "seconds": time.time() - t0,
           "source": "oracle.parallel.source_iteration_parallel (FP64, SuperLU per system)"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
