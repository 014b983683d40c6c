"""GPU: the energy balance reported in obte_stats, and the not-converged
status with a resumable state (both through the C ABI, against the oracle)."""
import os
import tempfile

import numpy as np
import pytest

from oracle.bte import Problem, source_iteration
from tests.gpu_common import gpu_solve, rel, require_gpu
from tests.test_gpu_parity import membrane3d, ragged_porous

pytestmark = pytest.mark.gpu

TIGHT = dict(inner_tol=1e-14, fourier_tol=1e-14, max_inner=200)


@pytest.fixture(scope="module")
def P():
    return require_gpu()


@pytest.mark.parametrize("name", ["ragged", "membrane3d"])
@pytest.mark.parametrize("prec", [0, 1])
def test_energy_residual_vs_oracle(P, name, prec):
    """Section Model: T_L conserves energy at the fixed point.  After K
    passes the residual of the last pass against the T_L it was solved with
    equals the oracle's (same definition, same passes)."""
    w = {"ragged": ragged_porous, "membrane3d": membrane3d}[name]()
    K = 5
    r = gpu_solve(P, w, want_J=False, precision=prec, outer_tol=0.0, max_outer=K, **TIGHT)
    ref = source_iteration(Problem(w), n_passes=r["outer_iters"])
    assert ref["energy_residual"] > 1e-6            # not trivially zero after K passes
    tol = 1e-8 if prec == 0 else 1e-3
    assert abs(r["energy_residual"] - ref["energy_residual"]) <= tol * ref["energy_residual"]
    # at the fixed point it vanishes (to the convergence level)
    rc = gpu_solve(P, w, want_J=False, outer_tol=1e-12, **TIGHT)
    assert rc["status"] == 0
    assert rc["energy_residual"] < 1e-9


def test_not_converged_status_and_resume(P):
    """max_outer = 3: OBTE_ERR_NOT_CONVERGED with the results of the 3 passes
    written; the checkpoint of that state resumes to the converged answer of
    an uninterrupted run (bitwise in FP64)."""
    w = ragged_porous()
    s = P.Solver.from_workload(w)
    o = s.opts(outer_tol=1e-10, max_outer=3, **TIGHT)
    ws = s.ensure_workspace(o)
    with pytest.raises(P.ObteError) as e:
        P.obte.obte_solve(s.mesh, o, None, ws, stream=s.stream, raise_not_converged=True)
    assert e.value.status == P.obte.OBTE_ERR_NOT_CONVERGED
    st = s.solve(o, want_T_L=True)
    assert st["status"] == P.obte.OBTE_ERR_NOT_CONVERGED and st["outer_iters"] == 3
    ref3 = source_iteration(Problem(w), n_passes=3)
    assert abs(st["kappa"] - ref3["kappa_cc"]) <= 1e-10 * abs(ref3["kappa_cc"])
    k3, _ = s.kappa()
    assert k3 == st["kappa"]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "state.bin")
        s.checkpoint_save(path)
        s2 = P.Solver.from_workload(w)
        o2 = s2.opts(outer_tol=1e-10, max_outer=5000, init=1, **TIGHT)
        s2.ensure_workspace(o2)
        s2.checkpoint_load(path)
        done = s2.solve(o2, want_T_L=True)
    full = gpu_solve(P, w, want_J=False, outer_tol=1e-10, max_outer=5000, **TIGHT)
    assert done["status"] == 0 and full["status"] == 0
    assert done["outer_iters"] == full["outer_iters"]
    assert done["kappa"] == full["kappa"]
    assert np.array_equal(done["T_L"].cpu().numpy(), full["T_L"])


def test_checkpoint_save_rejects_without_touching_the_file(P):
    """A rejected save (another workspace than the last solve's) returns
    OBTE_ERR_ARG and leaves an existing file as it was."""
    import torch
    w = ragged_porous()
    s = P.Solver.from_workload(w)
    s.solve(s.opts(outer_tol=1e-6), want_T_L=False)
    other = torch.empty_like(s.workspace)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "keep.bin")
        with open(path, "wb") as f:
            f.write(b"previous contents")
        with pytest.raises(P.ObteError) as e:
            P.obte.obte_checkpoint_save(s.mesh, other, path)
        assert e.value.status == P.obte.OBTE_ERR_ARG
        assert open(path, "rb").read() == b"previous contents"
