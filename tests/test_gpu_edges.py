"""Edge cases of the 2D path against the oracle: the widest row (nx = 256,
four cells per lane) and a ragged one, the smallest grid, non-periodic y
(walls along the row direction) and non-periodic x with the gradient along
y, a single MFP with four directions, and a pore column that blocks the
gradient axis (kappa -> 0)."""
import dataclasses

import numpy as np
import pytest

from inputs import gen
from oracle.bte import Problem, source_iteration
from tests.gpu_common import gpu_solve, oracle_full, rel, require_gpu

pytestmark = pytest.mark.gpu
NM = 1e-9


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def _pore_cols(nx, ny, c0, c1):
    s = np.ones((ny, nx), np.uint8)
    s[:, c0:c1] = 0
    return s


def _rows_pore(nx, ny):
    # a 24 x 3 pore in the middle rows, one across the x boundary
    s = np.ones((ny, nx), np.uint8)
    s[2:5, nx // 2 - 12: nx // 2 + 12] = 0
    s[5:7, nx - 5:] = 0
    s[5:7, :4] = 0
    return s


def _block(nx, ny):
    s = np.ones((ny, nx), np.uint8)
    s[ny // 3: ny // 3 + max(1, ny // 3), nx // 3: nx // 3 + max(1, nx // 4)] = 0
    return s


EDGE = {
    "max_width": lambda: gen.small_2d(256, 8, solid=_rows_pore(256, 8), n_dir=8,
                                      n_mfp=2, L=256 * NM, Ly=8 * NM, mfp_hi=100 * NM),
    "ragged_cpl4": lambda: gen.small_2d(250, 8, solid=_rows_pore(250, 8), n_dir=8, n_mfp=2, L=250 * NM,
                                        Ly=8 * NM, mfp_hi=100 * NM),
    "minimal_grid": lambda: gen.small_2d(2, 2, n_dir=4, n_mfp=2),
    "y_walls": lambda: dataclasses.replace(gen.small_2d(12, 9, solid=_block(12, 9), n_dir=8, n_mfp=3),
                                           periodic=(1, 0, 0)),
    "x_walls_grad_y": lambda: dataclasses.replace(
        gen.small_2d(9, 12, solid=_block(9, 12), n_dir=8, n_mfp=3, grad_axis=1), periodic=(0, 1, 0)),
    "one_mfp": lambda: gen.small_2d(12, 10, solid=_block(12, 10), n_dir=4, n_mfp=1),
}


@pytest.mark.parametrize("name", list(EDGE))
def test_edge_converged(P, name):
    w = EDGE[name]()
    prob = Problem(w)
    ref = source_iteration(prob, tol=1e-13, max_passes=20000)
    # the slowest of these contract at rho ~ 0.99: stop on the estimated error
    r = gpu_solve(P, w, outer_tol=1e-12, stop_rule=1, inner_tol=1e-14, fourier_tol=1e-14, max_inner=200,
                  max_outer=20000)
    assert r["status"] == 0
    assert abs(r["kappa"] - ref["kappa_cc"]) <= 1e-10 * abs(ref["kappa_cc"])
    assert abs(r["kappa_face"] - ref["kappa_face"]) <= 1e-10 * abs(ref["kappa_face"])
    assert rel(r["T_L"], oracle_full(prob, ref["T_L"])) < 1e-10
    Jref = np.zeros((w.n_cells, w.ndim))
    Jref[prob.mesh.cells] = ref["J"]
    assert rel(r["J"], Jref) < 1e-10
    r32 = gpu_solve(P, w, want_J=False, precision=1, outer_tol=1e-9, inner_tol=1e-6, fourier_tol=1e-12,
                    max_outer=20000)
    assert abs(r32["kappa"] - ref["kappa_cc"]) <= 1e-4 * abs(ref["kappa_cc"])


def test_blocked_gradient_axis(P):
    """A pore column across every row: no path along x, so the flux through
    the cell vanishes; GPU and oracle agree pass for pass on a kappa that
    tends to 0 (absolute bar against the bulk 150 W/m/K)."""
    w = gen.small_2d(12, 8, solid=_pore_cols(12, 8, 5, 7), n_dir=8, n_mfp=3)
    prob = Problem(w)
    K = 8
    r = gpu_solve(P, w, outer_tol=0.0, max_outer=K, inner_tol=1e-14, fourier_tol=1e-14, max_inner=200)
    ref = source_iteration(prob, n_passes=r["outer_iters"])
    assert abs(r["kappa"] - ref["kappa_cc"]) <= 1e-10 * 150.0
    assert abs(r["kappa_fourier"]) <= 1e-9 * 150.0
    assert rel(r["T_L"], oracle_full(prob, ref["T_L"])) < 1e-10
