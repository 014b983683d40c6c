"""The gain bound of the wrap map that lets the pass kernels skip the Krylov
sweep of a weakly coupled system (CPU, on the oracle's discrete operator).

A system (sigma + Lambda A_l) x = b of Appendix A, Eq. (iter2) on a grid
periodic along y splits into the sweep operator M0 (the y-wrap couplings
removed) and the wrap couplings.  With the wrap inflow u entering the first
row of the sweep and the map G: u -> Lambda c_y x(last row) (c_y = |s_y| / h_y),
the kernels use |G|_2 <= q^ny with q = Lambda c_y / (sigma_min + Lambda c_y).
The bound is checked on the oracle's assembled operator with pores and a
varying sigma, and shown tight (equal) for a pore-free cell with uniform
sigma, where the uniform inflow is an eigenvector with eigenvalue q^ny."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from inputs import gen
from oracle.bte import Problem

NM = 1e-9


def wrap_map(prob, m, l):
    """Dense G of system (m, l) and the bound q^ny."""
    me, mat = prob.mesh, prob.mat
    sy = float(mat.dirs[l, 1])
    ny = me.n[1]
    if sy == 0.0:
        return np.zeros((0, 0)), 0.0
    side_in = 0 if sy > 0 else 1
    y_first, y_last = (0, ny - 1) if sy > 0 else (ny - 1, 0)
    M = prob.system_matrix(m, l).tolil()
    pairs = []
    for i in range(me.n_solid):
        j = me.nbr[i, 1, side_in]
        if me.coord[i, 1] == y_first and j >= 0 and me.coord[j, 1] == y_last:
            pairs.append((i, j))
    cy = mat.mfp[m] * abs(sy) / me.h[1]
    for i, j in pairs:
        assert abs(M[i, j] + cy) <= 1e-12 * cy          # the wrap coupling entry
        M[i, j] = 0.0
    lu = spla.splu(M.tocsc())
    G = np.zeros((len(pairs), len(pairs)))
    for k, (i, _) in enumerate(pairs):
        e = np.zeros(me.n_solid)
        e[i] = 1.0
        x = lu.solve(e)
        G[:, k] = cy * x[[j for _, j in pairs]]
    smin = float(prob.sigma.min())
    q = cy / (smin + cy)
    return G, q ** ny


def test_gain_bound_with_pores_and_sigma():
    rng = np.random.default_rng(5)
    L = 60 * NM
    s = gen.circles_mask(14, 11, L, L * 11 / 14, [(15 * NM, 20 * NM), (50 * NM, 5 * NM)], [9 * NM, 7 * NM])
    w = gen.small_2d(14, 11, solid=s, n_dir=12, n_mfp=6, L=L, Ly=L * 11 / 14,
                     sigma=rng.uniform(0.4, 2.5, 14 * 11))
    prob = Problem(w)
    seen = []
    for m in range(prob.mat.n_mfp):
        for l in range(prob.mat.n_dir):
            G, bound = wrap_map(prob, m, l)
            if G.size == 0:
                continue
            g2 = np.linalg.norm(G, 2)
            assert g2 <= bound * (1 + 1e-10) + 1e-300, (m, l, g2, bound)
            seen.append(bound)
    # the check covers strongly and weakly coupled systems alike
    assert min(seen) < 1e-6 and max(seen) > 0.3


@pytest.mark.parametrize("grad_axis", [0, 1])
def test_gain_bound_tight_without_pores(grad_axis):
    w = gen.small_2d(9, 7, n_dir=8, n_mfp=4, grad_axis=grad_axis, sigma=np.full(63, 1.3))
    prob = Problem(w)
    for m in range(prob.mat.n_mfp):
        for l in range(prob.mat.n_dir):
            G, bound = wrap_map(prob, m, l)
            if G.size == 0:
                continue
            g2 = np.linalg.norm(G, 2)
            assert abs(g2 - bound) <= 1e-10 * bound + 1e-300, (m, l, g2, bound)
            # the uniform inflow is scaled by exactly q^ny
            one = np.ones(G.shape[0])
            assert np.allclose(G @ one, bound * one, rtol=1e-10, atol=1e-300)
