"""Material weights on the vectorial-MFP grid (oracle; FP64).

Paper, section "Model": in the RTA the lattice pseudo-temperature is the
C/tau-weighted mean of the mode temperatures and the flux is sum_mu S_mu T_mu
with S_mu = C_mu v_mu.  Appendix A defines D_ml (the T_L weights) and S_ml (the
flux weights) on the grid F_ml = Lambda_m s_l.

With MFP F = tau v, C v = (C/tau) F, so writing alpha = C/tau:
  D_ml = alpha_ml / sum alpha,    S_ml = alpha_ml Lambda_m s_l,
and the bulk conductivity along the gradient axis g is sum alpha Lambda^2 s_g^2.
The per-MFP kernel kappa_m is spread over directions with the quadrature
weights w_l and normalised by the discrete second moment mu_g = sum w s_g^2,
so that the discrete bulk conductivity equals sum kappa_m exactly:
  alpha_ml = kappa_m w_l / (Lambda_m^2 mu_g).

Diffuse (thermalising) walls, section "Model": phonons leaving a wall take one
temperature, weighted by the outgoing flux ReLu(S_ml . n); the normalised
weights per wall orientation are returned by ``wall_weights``.
"""
from __future__ import annotations

import numpy as np


class Material:
    def __init__(self, mfp, dirs, dir_w, kappa_m, grad_axis=0, modes=None, exact=False):
        mfp = np.asarray(mfp, float)
        dirs = np.asarray(dirs, float)
        dir_w = np.asarray(dir_w, float)
        kappa_m = np.asarray(kappa_m, float)
        self.mfp, self.dirs, self.dir_w, self.kappa_m = mfp, dirs, dir_w, kappa_m
        self.n_mfp, self.n_dir = len(mfp), len(dir_w)
        self.ndim = dirs.shape[1]
        self.grad_axis = grad_axis
        self.modes = modes
        self.exact = bool(exact and modes is not None)
        if self.exact:
            # Eq. iter3: one system per moving mode, no interpolation.  The
            # grid degenerates to one 'MFP' of 1 and the modes' own vectorial
            # MFPs as transport vectors (the operators take F_mu directly).
            from .modes import project
            F, alpha = modes
            alpha = np.asarray(alpha, float)
            Fp = project(F, dirs.shape[1])
            moving = np.linalg.norm(Fp, axis=1) > 0.0
            Fm, am = Fp[moving], alpha[moving]
            self.moving = np.flatnonzero(moving)
            self.mfp = np.array([1.0])
            self.dirs = Fm
            self.dir_w = am / am.sum()
            self.kappa_m = np.array([np.nan])
            self.n_mfp, self.n_dir = 1, len(am)
            self.mu = float("nan")
            self.D = (am / am.sum())[None, :]
            self.S = (am[:, None] * Fm)[None, :, :]
            self.kappa_axis = np.array([np.sum(am * Fm[:, a] ** 2) for a in range(self.ndim)])
            self.alpha = am[None, :].copy()
            return
        if modes is not None:
            # grid weights interpolated from a mode table (oracle/modes.py)
            from .modes import grid_weights, project
            F, alpha = modes
            self.mu = float(np.sum(dir_w * dirs[:, grad_axis] ** 2))
            self.D, self.S, self.kappa_axis = grid_weights(mfp, dirs, F, alpha, grad_axis)
            # sum alpha_mu c over the moving modes: the T_L weights unnormalised
            moving = np.linalg.norm(project(F, dirs.shape[1]), axis=1) > 0.0
            self.alpha = self.D * float(np.sum(np.asarray(alpha, float)[moving]))
            return
        w = material_weights(mfp, dirs, dir_w, kappa_m, grad_axis)
        self.mu = w["mu"]
        self.alpha = w["alpha"]        # (n_mfp, n_dir)
        self.D = w["D"]                # (n_mfp, n_dir)
        self.S = w["S"]                # (n_mfp, n_dir, ndim)
        self.kappa_axis = w["kappa_axis"]   # (ndim,)

    def system_index(self, m, l):
        """Systems are numbered m-major: sys = m * n_dir + l."""
        return m * self.n_dir + l


def material_weights(mfp, dirs, dir_w, kappa_m, grad_axis=0):
    mu = float(np.sum(dir_w * dirs[:, grad_axis] ** 2))
    alpha = kappa_m[:, None] * dir_w[None, :] / (mfp[:, None] ** 2 * mu)
    D = alpha / alpha.sum()
    S = alpha[:, :, None] * mfp[:, None, None] * dirs[None, :, :]
    kappa_axis = np.array([np.sum(alpha * mfp[:, None] ** 2 * dirs[None, :, a] ** 2)
                           for a in range(dirs.shape[1])])
    return {"mu": mu, "alpha": alpha, "D": D, "S": S, "kappa_axis": kappa_axis}


def wall_weights(S, normal):
    """Normalised outgoing-flux weights ReLu(S_ml . n) / sum ReLu(S . n)."""
    sn = np.tensordot(S, np.asarray(normal, float), axes=([2], [0]))
    r = np.maximum(sn, 0.0)
    return r / r.sum()
