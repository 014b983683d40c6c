"""Mode tables on the vectorial-MFP grid (oracle; FP64).  Test
infrastructure only: nothing here is used by the GPU path.

Appendix A: the aMFP-BTE interpolates each mode's vectorial MFP onto the
grid F_ml = Lambda_m s_l with weights c^mu_ml, and the grid weights are
D_ml = sum_mu c^mu_ml D_mu (T_L) and S_ml = sum_mu c^mu_ml S_mu (flux), with
D_mu = alpha_mu / sum alpha and S_mu = alpha_mu F_mu (alpha = C / tau).
The paper does not fix c (reading: linear in Lambda between the bracketing
MFP nodes, times linear in angle between the bracketing directions; 2D:
azimuth, cyclic; 3D: polar bins times azimuth on a tensor direction grid;
outside the MFP range, or beyond the outermost polar bin centres, the weight
goes to the end node).

Without interpolation (Eq. iter3, the mode-resolved iteration) every moving
mode is its own system with transport vector F_mu (Material(..., exact=True)).

The mode-resolved conductivity (Eq. mode-resolved) in the cell-centred form
used for kappa_eff: kappa_mu = L S_mu,g / (dT N_tot) sum_ml c^mu_ml sum_i
(T_iml - <T_L>), which sums to kappa_eff over the modes because S_ml =
sum_mu c S_mu and sum_mu S_mu = 0.  The temperatures of the periodic problem
are fixed only up to a common constant; kappa_eff does not depend on it, a
single mode's share does (by S_mu,g times the constant).  The paper does not
say which constant (reading: deviations from the mean lattice temperature
over the solid cells, <T_L> = sum_ml D_ml sum_i T_iml / N_solid, so each
kappa_mu is unchanged when every T moves by the same amount).

Section Material, rta2DSym: a 2D domain (uniform along z) takes 3D modes
through their in-plane part F_mu,xy; the out-of-plane part does not enter the
2D transport operator.  A mode whose vectorial MFP is zero (in 2D: one that
moves only along z) satisfies T_mu = T_L exactly (Eq. iter3 with F_mu = 0),
so it drops out of T_L = sum D T once the remaining weights are renormalised:
such modes get no grid weight, D_mu is alpha_mu over the sum of alpha of the
moving modes, and their kappa_mu is 0.
"""
from __future__ import annotations

import math

import numpy as np


def _bracket_linear(nodes, x):
    """[(index, weight)] of the linear interpolation of x on sorted nodes
    (clamped to the end nodes)."""
    if x <= nodes[0]:
        return [(0, 1.0)]
    if x >= nodes[-1]:
        return [(len(nodes) - 1, 1.0)]
    a = int(np.searchsorted(nodes, x, side="right")) - 1
    t = (x - nodes[a]) / (nodes[a + 1] - nodes[a])
    return [(a, 1.0 - t), (a + 1, t)]


def _bracket_cyclic(angles, x):
    """Linear interpolation on sorted angles in [0, 2 pi) with wrap-around."""
    n = len(angles)
    x = x % (2 * math.pi)
    b = int(np.searchsorted(angles, x, side="right"))
    a = (b - 1) % n
    b = b % n
    lo = angles[a]
    gap = (angles[b] - lo) % (2 * math.pi)
    t = ((x - lo) % (2 * math.pi)) / gap
    return [(a, 1.0 - t), (b, t)]


def project(F, nd):
    """The part of the vectorial MFPs a domain of nd dimensions sees
    (rta2DSym: 3D modes in a 2D domain keep their in-plane components)."""
    F = np.asarray(F, float)
    if F.shape[1] < nd:
        raise ValueError("mode table has fewer components than the domain")
    return F[:, :nd]


def interp_weights(mfp, dirs, F):
    """For each mode the list of (m, l, c) with nonzero weight (empty for a
    mode with zero vectorial MFP)."""
    mfp = np.asarray(mfp, float)
    dirs = np.asarray(dirs, float)
    nd = dirs.shape[1]
    F = project(F, nd)
    m_order = np.argsort(mfp)
    m_nodes = mfp[m_order]
    out = []
    if nd == 2:
        ang = np.arctan2(dirs[:, 1], dirs[:, 0]) % (2 * math.pi)
        l_order = np.argsort(ang)
        l_nodes = ang[l_order]
        for f in F:
            lam = float(np.hypot(f[0], f[1]))
            if lam == 0.0:
                out.append([])
                continue
            wm = _bracket_linear(m_nodes, lam)
            wl = _bracket_cyclic(l_nodes, math.atan2(f[1], f[0]))
            out.append([(int(m_order[i]), int(l_order[j]), a * b) for i, a in wm for j, b in wl])
        return out
    th = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
    ph = np.arctan2(dirs[:, 1], dirs[:, 0]) % (2 * math.pi)
    th_nodes = np.unique(np.round(th, 12))
    ph_nodes = np.unique(np.round(ph, 12))
    index = {}
    for l in range(len(dirs)):
        key = (int(np.argmin(np.abs(th_nodes - th[l]))), int(np.argmin(np.abs(ph_nodes - ph[l]))))
        index[key] = l
    if len(index) != len(th_nodes) * len(ph_nodes):
        raise ValueError("3D mode interpolation needs a tensor (polar x azimuth) direction grid")
    for f in F:
        lam = float(np.linalg.norm(f))
        if lam == 0.0:
            out.append([])
            continue
        wm = _bracket_linear(m_nodes, lam)
        wt = _bracket_linear(th_nodes, math.acos(max(-1.0, min(1.0, f[2] / lam))))
        wp = _bracket_cyclic(ph_nodes, math.atan2(f[1], f[0]))
        out.append([(int(m_order[i]), index[(j, k)], a * b * c)
                    for i, a in wm for j, b in wt for k, c in wp])
    return out


def grid_weights(mfp, dirs, F, alpha, grad_axis=0):
    """D (n_mfp, n_dir), S (n_mfp, n_dir, ndim) and the Fourier conductivity
    per axis sum_mu alpha_mu F_mu,a^2 from a mode table."""
    alpha = np.asarray(alpha, float)
    n_mfp, n_dir, nd = len(mfp), len(dirs), np.asarray(dirs).shape[1]
    F = project(F, nd)
    D = np.zeros((n_mfp, n_dir))
    S = np.zeros((n_mfp, n_dir, nd))
    moving = np.linalg.norm(F, axis=1) > 0.0
    Dmu = np.where(moving, alpha, 0.0) / alpha[moving].sum()
    for mu, terms in enumerate(interp_weights(mfp, dirs, F)):
        for m, l, c in terms:
            D[m, l] += c * Dmu[mu]
            S[m, l] += c * alpha[mu] * F[mu]
    kappa_axis = np.array([np.sum(alpha * F[:, a] ** 2) for a in range(nd)])
    return D, S, kappa_axis


def kappa_modes(prob, T):
    """kappa_mu of every mode from the per-system solutions T (n_mfp, n_dir,
    n_solid) of a converged solve (kappa_cc form, T measured from the mean
    lattice temperature)."""
    mat, me = prob.mat, prob.mesh
    F, alpha = mat.modes
    F = project(F, mat.dirs.shape[1])
    g = me.grad_axis
    tot = T.sum(axis=2)                                   # sum_i T_iml
    tot_L = float(np.sum(mat.D * tot))                    # sum_i T_L,i = N_solid <T_L>
    pref = me.L[g] / (me.dT * me.n_cells)
    out = np.zeros(len(alpha))
    if mat.exact:
        # one system per moving mode: c is the identity
        terms_of = [[] for _ in range(len(alpha))]
        for k, mu in enumerate(mat.moving):
            terms_of[mu] = [(0, k, 1.0)]
    else:
        terms_of = interp_weights(mat.mfp, mat.dirs, F)
    for mu, terms in enumerate(terms_of):
        # sum_ml c = 1: the interpolated sum of (T - <T_L>)
        out[mu] = pref * alpha[mu] * F[mu, g] * (sum(c * tot[m, l] for m, l, c in terms) - tot_L)
    return out
