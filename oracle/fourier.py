"""Fourier first guess (oracle; FP64, direct sparse solve).

Paper, section "Implementation" (Eq. fourier_iter) and Appendix B: the first
guess of the BTE iteration is the heat-conduction solution of
div(kappa grad T) = 0 over the solid with adiabatic pore walls and the applied
temperature difference across the periodic boundary.  On an orthogonal grid
the secondary (non-orthogonal) flux of Appendix B vanishes and the face
gradient is the plain two-point difference (T_j + delta dT - T_i) / h, so the
finite-volume balance is

  sum_faces kappa_a / h_a^2 (T_j + delta_f dT - T_i) = 0    (each solid cell).

kappa_a is the diagonal of the discrete bulk tensor, sum alpha Lambda^2 s_a^2.
The system is singular (T is fixed up to a constant); the oracle borders it
with the constraint mean(T) = 0.  kappa_fourier is the Appendix-B plane flux
through the hot contact:  (L_g / (dT A)) sum_faces A_f kappa_g (T_j + dT - T_i)/h_g.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def fourier_matrix(mesh, kappa_axis):
    rows, cols, vals = [], [], []
    rhs = np.zeros(mesh.n_solid)
    for i in range(mesh.n_solid):
        for a in range(mesh.ndim):
            k = kappa_axis[a] / mesh.h[a] ** 2
            for side in (0, 1):
                j = mesh.nbr[i, a, side]
                if j < 0:
                    continue            # pore or outer wall: adiabatic
                rows += [i, i]
                cols += [i, j]
                vals += [-k, k]
                rhs[i] -= k * mesh.jump[i, a, side] * mesh.dT
    Lap = sp.csr_matrix((vals, (rows, cols)), shape=(mesh.n_solid, mesh.n_solid))
    return Lap, rhs


def fourier_solve(mesh, kappa_axis):
    """Return (T_F over solid cells with mean zero, kappa_fourier)."""
    Lap, rhs = fourier_matrix(mesh, kappa_axis)
    n = mesh.n_solid
    one = np.ones((n, 1))
    B = sp.bmat([[Lap, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]], format="csc")
    sol = spla.spsolve(B, np.concatenate([rhs, [0.0]]))
    T = sol[:n]
    return T, kappa_fourier(mesh, kappa_axis, T)


def kappa_fourier(mesh, kappa_axis, T):
    g = mesh.grad_axis
    tot = 0.0
    for j, i in mesh.plane_pairs():
        tot += kappa_axis[g] * (T[j] + mesh.dT - T[i]) / mesh.h[g]
    return mesh.L[g] / (mesh.dT * mesh.n_perp) * tot


def dirichlet_energy_kappa(mesh, kappa_axis, T):
    """Green's identity for the discrete solution: kappa_F (dT/L)^2 V equals
    sum over faces of kappa_a ((T_j + delta dT - T_i)/h_a)^2 V_cell (each face
    once).  Independent of the plane-flux formula; used to pin it."""
    e = 0.0
    for i in range(mesh.n_solid):
        for a in range(mesh.ndim):
            j = mesh.nbr[i, a, 1]
            if j < 0:
                continue
            d = (T[j] + mesh.jump[i, a, 1] * mesh.dT - T[i]) / mesh.h[a]
            e += kappa_axis[a] * d * d
    g = mesh.grad_axis
    return e / mesh.n_cells * (mesh.L[g] / mesh.dT) ** 2
