"""aMFP-BTE source iteration, kappa, flux and dense brute force (oracle; FP64).

Paper references:
  * section "Model", Eq. (rta): MFP form of the RTA BTE,
      F_ml . grad T_ml + sigma (T_ml - T_L) = 0,  F_ml = Lambda_m s_l,
    with the per-cell relaxation-rate multiplier sigma (sigma = 1 in the plain
    method);
  * Appendix A, Eq. (iter2): upwind finite volumes.  For direction s_l the
    stiffness A_l has the outgoing face flux sum_f a_f ReLu(s_l . n_f) on the
    diagonal of row i and -a_f ReLu(-s_l . n_f) towards the upwind solid
    neighbour j; incoming flux through a pore wall carries the wall
    temperature T_w and through the periodic plane of the gradient axis the
    applied difference dT (the perturbation P);
  * section "Model": T_L = sum D_ml T_ml, diffuse walls with outgoing-flux
    weights ReLu(S . n) / sum ReLu(S . n);
  * section "Implementation", Eq. (iter) and Algorithm 1: source iteration
    with all couplings (T_L, T_w) lagged to the previous pass, one LU per
    (m, l) system computed once and reused, stop on the relative change of
    kappa;
  * Eq. (keff) and the kappa formula of Appendix A: kappa_face is the upwind
    flux through the hot contact (the periodic plane of the gradient axis);
    kappa_cc is the volume average of the cell-centred flux J = sum S_ml T_ml
    (section "Model") times L / dT.  Both are reported; kappa_cc is primary.

Sign conventions (the paper leaves them open): the image across the periodic
plane satisfies T(x + L) = T(x) - dT, so heat flows towards +g and kappa > 0;
wall inflow adds +Lambda a |s.n| T_w to the right-hand side.
"""
from __future__ import annotations

import math
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fourier import fourier_solve
from .material import Material, wall_weights
from .mesh import Mesh


def upwind_operator(mesh, s):
    """Sparse A_l (n_solid^2), the periodic-jump inflow vector (already times
    dT) and the wall-inflow matrix Bw (n_solid x n_walls) for direction s."""
    n = mesh.n_solid
    idx = np.arange(n)
    diag = np.zeros(n)
    jump = np.zeros(n)
    r, c, v = [idx], [idx], [None]
    br, bc, bv = [], [], []
    for a in range(mesh.ndim):
        sa = float(s[a])
        if sa == 0.0:
            continue
        coef = abs(sa) / mesh.h[a]
        diag += coef                                   # outgoing face of axis a
        side_in = 0 if sa > 0 else 1                   # incoming face of axis a
        j = mesh.nbr[:, a, side_in]
        m = j >= 0
        r.append(idx[m]); c.append(j[m]); v.append(np.full(m.sum(), -coef))
        jump[m] += coef * mesh.jump[m, a, side_in] * mesh.dT
        w = mesh.wall_id[:, a, side_in]
        mw = w >= 0
        br.append(idx[mw]); bc.append(w[mw]); bv.append(np.full(mw.sum(), coef))
    v[0] = diag
    A = sp.csr_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))), shape=(n, n))
    if br:
        Bw = sp.csr_matrix((np.concatenate(bv), (np.concatenate(br), np.concatenate(bc))),
                           shape=(n, mesh.n_walls))
    else:
        Bw = sp.csr_matrix((n, mesh.n_walls))
    return A, jump, Bw


class Problem:
    """Mesh + material + per-direction operators for one geometry."""

    def __init__(self, work=None, *, mesh=None, mat=None, sigma=None):
        if work is not None:
            mesh = Mesh(work.n, work.L, work.solid, work.periodic, work.grad_axis, work.dT,
                        ndim=work.ndim)
            mat = Material(work.mfp, work.dirs, work.dir_w, work.kappa_m, work.grad_axis,
                           modes=getattr(work, "modes", None), exact=getattr(work, "modes_exact", False))
            sigma = work.sigma
        self.mesh, self.mat = mesh, mat
        if sigma is None:
            self.sigma = np.ones(mesh.n_solid)
        else:
            sigma = np.asarray(sigma, float)
            self.sigma = sigma[mesh.cells] if sigma.size == mesh.n_cells else sigma.copy()
        self.ops = [upwind_operator(mesh, mat.dirs[l]) for l in range(mat.n_dir)]
        # outgoing wall weights per wall face and system: (n_walls, n_mfp, n_dir)
        self.wout = np.zeros((mesh.n_walls, mat.n_mfp, mat.n_dir))
        cache = {}
        for f in range(mesh.n_walls):
            key = tuple(mesh.walls[f, 1:])
            if key not in cache:
                cache[key] = wall_weights(mat.S, mesh.wall_normal(f))
            self.wout[f] = cache[key]
        self.wall_cell = mesh.walls[:, 0] if mesh.n_walls else np.zeros(0, np.int64)
        self.pairs = mesh.plane_pairs()
        self._lu = {}

    # -- per-system pieces -------------------------------------------------
    def system_matrix(self, m, l):
        A = self.ops[l][0]
        return (sp.diags(self.sigma) + self.mat.mfp[m] * A).tocsc()

    def lu(self, m, l, cache=True):
        key = (m, l)
        if key in self._lu:
            return self._lu[key]
        f = spla.splu(self.system_matrix(m, l))
        if cache:
            self._lu[key] = f
        return f

    def rhs(self, m, l, T_L, T_w):
        _, jump, Bw = self.ops[l]
        return self.sigma * T_L + self.mat.mfp[m] * (jump + Bw @ T_w)

    # -- functionals ----------------------------------------------------------
    def kappa_cc_system(self, m, l, x):
        g, me = self.mesh.grad_axis, self.mesh
        return me.L[g] / (me.dT * me.n_cells) * self.mat.S[m, l, g] * x.sum()

    def kappa_face_system(self, m, l, x):
        g, me = self.mesh.grad_axis, self.mesh
        if len(self.pairs) == 0:
            return 0.0
        j, i = self.pairs[:, 0], self.pairs[:, 1]
        sg = self.mat.dirs[l, g]
        up = x[j] + me.dT if sg > 0 else x[i]
        return me.L[g] / (me.dT * me.n_perp) * self.mat.S[m, l, g] * up.sum()


def kappa_cc(prob, T):
    """T: (n_mfp, n_dir, n_solid).  Volume-averaged cell-centred flux * L/dT."""
    me, g = prob.mesh, prob.mesh.grad_axis
    return me.L[g] / (me.dT * me.n_cells) * float(np.sum(prob.mat.S[:, :, g] * T.sum(axis=2)))


def kappa_face(prob, T):
    return float(sum(prob.kappa_face_system(m, l, T[m, l])
                     for m in range(prob.mat.n_mfp) for l in range(prob.mat.n_dir)))


def flux_map(prob, T):
    """J_i = sum_ml S_ml T_iml  (n_solid, ndim)."""
    return np.einsum("mla,mli->ia", prob.mat.S, T)


def lattice_temperature(prob, T):
    return np.einsum("ml,mli->i", prob.mat.D, T)


def wall_temperature(prob, T):
    if prob.mesh.n_walls == 0:
        return np.zeros(0)
    return np.einsum("fml,mlf->f", prob.wout, T[:, :, prob.wall_cell])


def source_iteration(prob, tol=1e-8, max_passes=2000, n_passes=None, T_L0=None, T_w0=None,
                     keep_T=True, cache_lu=True, verbose=False, time_limit=None):
    """Algorithm 1.  Returns a dict with kappa_cc (primary), kappa_face,
    kappa_fourier, T_L (mean over solid cells subtracted), J, history, T."""
    me, mat = prob.mesh, prob.mat
    # the first guess: the problem's own heat-conduction solve where it has
    # one (unstructured meshes), else the orthogonal-grid one
    T_F, kF = prob.fourier() if hasattr(prob, "fourier") else fourier_solve(me, mat.kappa_axis)
    T_L = T_F.copy() if T_L0 is None else np.asarray(T_L0, float).copy()
    if T_w0 is not None:
        T_w = np.asarray(T_w0, float).copy()
    else:
        T_w = T_L[prob.wall_cell].copy() if me.n_walls else np.zeros(0)
    hist, hist_face = [], []
    kprev = None
    T = np.zeros((mat.n_mfp, mat.n_dir, me.n_solid)) if keep_T else None
    n_done = 0
    converged = False
    t0 = time.perf_counter()
    kml = np.zeros((mat.n_mfp, mat.n_dir))
    kfml = np.zeros((mat.n_mfp, mat.n_dir))
    T_L_used = T_L
    while True:
        T_L_new = np.zeros(me.n_solid)
        T_w_new = np.zeros(me.n_walls)
        for l in range(mat.n_dir):
            for m in range(mat.n_mfp):
                x = prob.lu(m, l, cache_lu).solve(prob.rhs(m, l, T_L, T_w))
                T_L_new += mat.D[m, l] * x
                if me.n_walls:
                    T_w_new += prob.wout[:, m, l] * x[prob.wall_cell]
                kml[m, l] = prob.kappa_cc_system(m, l, x)
                kfml[m, l] = prob.kappa_face_system(m, l, x)
                if keep_T:
                    T[m, l] = x
        n_done += 1
        k = float(kml.sum())
        hist.append(k)
        hist_face.append(float(kfml.sum()))
        T_L_used = T_L
        T_L, T_w = T_L_new, T_w_new
        if verbose:
            print(f"pass {n_done}: kappa_cc={k:.12g}", flush=True)
        if n_passes is not None:
            if n_done >= n_passes:
                break
        else:
            if kprev is not None and abs(k - kprev) <= tol * abs(k):
                converged = True
                break
            if n_done >= max_passes:
                break
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
        kprev = k
    out = {
        "kappa": hist[-1], "kappa_cc": hist[-1], "kappa_face": hist_face[-1],
        "kappa_fourier": kF, "kappa_per_mfp": kml.sum(axis=1).copy(),
        "kappa_ml": kml.copy(),
        "history": np.asarray(hist), "history_face": np.asarray(hist_face),
        "passes": n_done, "converged": converged,
        "T_L": T_L - T_L.mean(), "T_L_raw": T_L, "T_w": T_w, "T_F": T_F,
        "T_L_used": T_L_used, "seconds": time.perf_counter() - t0,
    }
    if keep_T:
        out["T"] = T
        out["J"] = flux_map(prob, T)
        # energy balance of the last pass against the T_L it was solved with
        res = np.einsum("ml,mli->i", mat.alpha, T - T_L_used[None, None, :]) * prob.sigma
        out["energy_residual"] = float(np.max(np.abs(res)) /
                                       max(np.einsum("ml,mli->", mat.alpha, np.abs(T)) / me.n_solid, 1e-300))
    return out


# ---------------------------------------------------------------------------
# dense brute force of the whole coupled system (tiny meshes only)
# ---------------------------------------------------------------------------

def dense_coupled_matrix(prob):
    """Assemble M T = p over all DoF directly, face by face, eliminating T_L
    and T_w.  Written independently of ``upwind_operator``."""
    me, mat = prob.mesh, prob.mat
    ns, nm, nd = me.n_solid, mat.n_mfp, mat.n_dir
    N = ns * nm * nd
    M = np.zeros((N, N))
    p = np.zeros(N)

    def idx(m, l, i):
        return (m * nd + l) * ns + i

    # outgoing wall weights, computed here from S directly
    for m in range(nm):
        for l in range(nd):
            s = mat.dirs[l]
            lam = mat.mfp[m]
            for i in range(ns):
                r = idx(m, l, i)
                M[r, r] += prob.sigma[i]
                for m2 in range(nm):
                    for l2 in range(nd):
                        M[r, idx(m2, l2, i)] -= prob.sigma[i] * mat.D[m2, l2]
                for a in range(me.ndim):
                    for side in (0, 1):
                        nsign = 1.0 if side == 1 else -1.0
                        sn = s[a] * nsign                     # s . n_face
                        coef = lam / me.h[a]
                        if sn > 0:
                            M[r, r] += coef * sn                # outflow
                            continue
                        if sn == 0:
                            continue
                        j = me.nbr[i, a, side]
                        if j >= 0:
                            M[r, idx(m, l, j)] -= coef * (-sn)
                            p[r] += coef * (-sn) * me.jump[i, a, side] * me.dT
                        else:
                            # wall: T_w = sum over outgoing (m2,l2) of S.n T / sum S.n
                            num = np.zeros((nm, nd))
                            for m2 in range(nm):
                                for l2 in range(nd):
                                    q = mat.S[m2, l2, a] * nsign
                                    if q > 0:
                                        num[m2, l2] = q
                            num /= num.sum()
                            for m2 in range(nm):
                                for l2 in range(nd):
                                    if num[m2, l2] > 0:
                                        M[r, idx(m2, l2, i)] -= coef * (-sn) * num[m2, l2]
    return M, p


def dense_solve(prob):
    """Solve the singular coupled system with the gauge sum_i T_L,i = 0.
    Returns T with shape (n_mfp, n_dir, n_solid)."""
    me, mat = prob.mesh, prob.mat
    M, p = dense_coupled_matrix(prob)
    N = len(p)
    c = np.zeros(N)
    ns = me.n_solid
    for m in range(mat.n_mfp):
        for l in range(mat.n_dir):
            c[(m * mat.n_dir + l) * ns:(m * mat.n_dir + l + 1) * ns] = mat.D[m, l]
    B = np.zeros((N + 1, N + 1))
    B[:N, :N] = M
    B[:N, N] = 1.0
    B[N, :N] = c
    sol = np.linalg.solve(B, np.concatenate([p, [0.0]]))
    return sol[:N].reshape(mat.n_mfp, mat.n_dir, ns), M, p, sol[N]
