"""Adjoint d kappa_cc / d sigma (oracle; FP64).

The paper lists differentiability as future work (section "Conclusion"); the
adjoint here is derived from the discrete system of Appendix A, Eq. (iter2),
with the per-cell relaxation-rate multiplier sigma:

  M(sigma) T = p,   kappa = k^T T,   k_iml = L_g S_ml,g / (dT N_cells),

  M = blockdiag(sigma + Lambda_m A_l) - C_L - C_w,
  (C_L T)_iml = sigma_i sum D T_i,   (C_w T)_iml = Lambda_m sum_f Bw_l[i,f] T_w,f.

Then d kappa / d sigma_i = -lambda^T (dM/dsigma_i) T with M^T lambda = k, and
dM/dsigma_i only touches the rows of cell i with entries T_iml - T_L,i:

  d kappa / d sigma_i = - sum_ml lambda_iml (T_iml - T_L,i).

The transposed source iteration lags C^T exactly as the forward one lags C:
  (sigma + Lambda_m A_l^T) lambda_ml = k_ml + D_ml Psi + sum_{walls f at i} Wout_ml(f) Phi_f,
  Psi_i = sigma_i sum_ml lambda_iml,
  Phi_f = sum_ml Lambda_m Bw_l[i(f), f] lambda_{i(f) ml}.
It reuses the forward LU factors with a transposed solve.  M is singular
(constants), but k sums to zero, the gradient is blind to both null spaces,
and p^T lambda = kappa at convergence (used as the stopping functional).
"""
from __future__ import annotations

import numpy as np


def k_weights(prob):
    me, g = prob.mesh, prob.mesh.grad_axis
    return me.L[g] / (me.dT * me.n_cells) * prob.mat.S[:, :, g]      # (n_mfp, n_dir)


def gradient_from(prob, T, lam):
    """-(sum_ml lambda (T - T_L)) per solid cell; T, lam: (n_mfp, n_dir, n_solid)."""
    T_L = np.einsum("ml,mli->i", prob.mat.D, T)
    return -np.einsum("mli,mli->i", lam, T - T_L[None, None, :])


def adjoint_source_iteration(prob, T, tol=1e-12, max_passes=5000, n_passes=None,
                             cache_lu=True):
    me, mat = prob.mesh, prob.mat
    kw = k_weights(prob)
    ns = me.n_solid
    Psi = np.zeros(ns)
    Phi = np.zeros(me.n_walls)
    lam = np.zeros((mat.n_mfp, mat.n_dir, ns))
    hist = []
    prev = None
    n_done = 0
    converged = False
    while True:
        Psi_new = np.zeros(ns)
        Phi_new = np.zeros(me.n_walls)
        kadj = 0.0
        for l in range(mat.n_dir):
            _, jump, Bw = prob.ops[l]
            for m in range(mat.n_mfp):
                b = np.full(ns, kw[m, l]) + mat.D[m, l] * Psi
                if me.n_walls:
                    np.add.at(b, prob.wall_cell, prob.wout[:, m, l] * Phi)
                x = prob.lu(m, l, cache_lu).solve(b, trans="T")
                lam[m, l] = x
                Psi_new += prob.sigma * x
                if me.n_walls:
                    Phi_new += mat.mfp[m] * (Bw.T @ x)
                kadj += mat.mfp[m] * float(jump @ x)
        n_done += 1
        hist.append(kadj)
        Psi, Phi = Psi_new, Phi_new
        if n_passes is not None:
            if n_done >= n_passes:
                break
        else:
            if prev is not None and abs(kadj - prev) <= tol * abs(kadj):
                converged = True
                break
            if n_done >= max_passes:
                break
        prev = kadj
    grad = gradient_from(prob, T, lam)
    return {"lambda": lam, "grad": grad, "kappa_adj": hist[-1], "history": np.asarray(hist),
            "passes": n_done, "converged": converged}


def adjoint_dense(prob, T):
    """Dense bordered solve of M^T lambda = k (tiny meshes)."""
    from .bte import dense_coupled_matrix
    mat, ns = prob.mat, prob.mesh.n_solid
    M, _ = dense_coupled_matrix(prob)
    N = M.shape[0]
    kw = k_weights(prob)
    k = np.repeat(kw.reshape(-1), ns)
    B = np.zeros((N + 1, N + 1))
    B[:N, :N] = M.T
    B[:N, N] = 1.0
    B[N, :N] = 1.0
    sol = np.linalg.solve(B, np.concatenate([k, [0.0]]))
    lam = sol[:N].reshape(mat.n_mfp, mat.n_dir, ns)
    return {"lambda": lam, "grad": gradient_from(prob, T, lam), "border": sol[N]}
