"""GPU: systems whose wrap map is provably weak (gain bound q^ny <= 0.1,
checked on the oracle's operator in test_wrap_gain.py) take the correction
e = r with no Krylov sweep when the forcing term allows it; the others still
run BiCGSTAB; the result is unchanged.  With no forcing term (inner_rtol 0)
a pass still solves every wrap to inner_tol."""
import numpy as np
import pytest

from tests.gpu_common import require_gpu
from tests.test_gpu_parity import ragged_porous

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def gain_bounds(w, sigma_min):
    """q^ny per system (index m * n_dir + l)."""
    h = w.L[1] / w.n[1]
    cy = np.abs(np.asarray(w.mfp)[:, None] * np.asarray(w.dirs)[None, :, 1]) / h
    return ((cy / (sigma_min + cy)) ** w.n[1]).ravel()


@pytest.mark.parametrize("prec", [0, 1])
def test_weak_wraps_skip_the_krylov_sweep(P, prec):
    w = ragged_porous()
    s = P.Solver.from_workload(w)
    tol = 1e-8 if prec == 0 else 1e-5
    o = s.opts(precision=prec, inner_rtol=0.3, lag_wrap=1, inner_tol=tol, outer_tol=1e-7,
               fourier_tol=1e-8, max_outer=2000)
    out = s.solve(o, want_T_L=False)
    assert out["status"] == 0
    its, sws = s.system_counts()
    rho = gain_bounds(w, 1.0)
    weak = rho <= 0.1          # the step must cut the residual tenfold
    assert weak.sum() >= 5 and (~weak).sum() >= 5
    # phase A only: one sweep per pass, no inner iteration
    assert np.all(sws[weak] == out["outer_iters"]), (sws[weak], out["outer_iters"])
    assert np.all(its[weak] == 0)
    assert sws[~weak].max() > out["outer_iters"]
    # and the same conductivity as a tightly solved wrap (both near their
    # fixed point: 1e-7 relative change)
    ref = s.solve(s.opts(precision=0, inner_tol=1e-13, outer_tol=1e-12, fourier_tol=1e-12, accel=8,
                         max_outer=4000), want_T_L=False)
    assert abs(out["kappa"] - ref["kappa"]) <= (1e-5 if prec == 0 else 1e-4) * ref["kappa"]


def test_no_forcing_term_keeps_exact_passes(P):
    """inner_rtol = 0: the sweep-free step is taken only where it already
    meets inner_tol, so K passes still match the oracle's exact passes."""
    from oracle.bte import Problem, source_iteration
    w = ragged_porous()
    s = P.Solver.from_workload(w)
    o = s.opts(inner_rtol=0.0, inner_tol=1e-14, fourier_tol=1e-14, outer_tol=0.0, max_outer=6, max_inner=200)
    out = s.solve(o, want_T_L=True)
    ref = source_iteration(Problem(w), n_passes=out["outer_iters"])
    assert abs(out["kappa"] - ref["kappa_cc"]) <= 1e-10 * abs(ref["kappa_cc"])
