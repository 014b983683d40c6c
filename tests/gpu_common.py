"""Helpers for the GPU parity tests (HIP path through the C ABI vs the oracle)."""
import numpy as np
import pytest
import torch

from tests._lib import ensure_built


def require_gpu():
    ensure_built()
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    import paper_2106_02764_amd as P
    return P


def gpu_solve(P, w, want_J=True, sigma=None, **opt):
    s = P.Solver.from_workload(w)
    o = s.opts(**opt)
    sig = sigma if sigma is not None else w.sigma
    out = s.solve(o, sigma=sig, want_T_L=True, want_J=want_J)
    torch.cuda.synchronize()
    res = dict(out)
    res["T_L"] = out["T_L"].cpu().numpy()
    if want_J:
        res["J"] = out["J"].cpu().numpy()
    res["solver"] = s
    res["opts"] = o
    return res


def oracle_full(prob, v):
    out = np.zeros(prob.mesh.n_cells)
    out[prob.mesh.cells] = v
    return out


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
