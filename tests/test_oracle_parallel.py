"""Pin of the multi-process oracle (the paper's per-core split of the
directions, section "Implementation", Algorithm 1) against the serial
source iteration: the same passes must give the same kappa_cc, kappa_face,
per-MFP kappa and T_L up to the order of the sums.  The parallel form wrote
the full-size reference values in tests/golden/, so it is pinned here on
cases the serial oracle runs in seconds."""
import numpy as np
import pytest

from inputs import gen
from oracle.bte import Problem, source_iteration
from oracle.parallel import source_iteration_parallel
from tests.test_gpu_parity import ragged_porous

CASES = {
    # 70 x 37 porous cell, two pores (one across the periodic boundary)
    "ragged2d": ragged_porous,
    # the membrane geometry (through-pore, diffuse top and bottom) at 8x8x3
    "membrane3d": lambda: gen.config5(nx=8, nz=3, n_theta=4, n_phi=8, n_mfp=3),
}


@pytest.mark.parametrize("name", list(CASES))
def test_parallel_matches_serial(name):
    w = CASES[name]()
    n_passes = 25
    ref = source_iteration(Problem(w), n_passes=n_passes)
    for workers in (1, 3):
        r = source_iteration_parallel(w, n_workers=workers, n_passes=n_passes)
        assert r["passes"] == ref["passes"] == n_passes
        for key in ("kappa_cc", "kappa_face", "kappa_fourier"):
            assert abs(r[key] - ref[key]) <= 1e-13 * abs(ref[key]), (workers, key)
        assert np.max(np.abs(r["kappa_per_mfp"] - ref["kappa_per_mfp"])) <= 1e-13 * abs(ref["kappa_cc"])
        assert np.max(np.abs(r["history"] - ref["history"])) <= 1e-13 * abs(ref["kappa_cc"])
        scale = np.max(np.abs(ref["T_L"]))
        assert np.max(np.abs(r["T_L"] - ref["T_L"])) <= 1e-13 * scale, workers
        assert np.max(np.abs(r["J"] - ref["J"])) <= 1e-13 * np.max(np.abs(ref["J"])), workers


def test_parallel_converged_stop_matches_serial():
    """With the stop test of Algorithm 1 both forms stop after the same pass."""
    w = CASES["ragged2d"]()
    ref = source_iteration(Problem(w), tol=1e-9)
    r = source_iteration_parallel(w, n_workers=2, tol=1e-9)
    assert r["converged"] and ref["converged"]
    assert r["passes"] == ref["passes"]
    assert abs(r["kappa_cc"] - ref["kappa_cc"]) <= 1e-13 * abs(ref["kappa_cc"])
