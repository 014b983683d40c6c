"""Unstructured 2D finite volumes (oracle; FP64): mesh geometry, the upwind
BTE operator and the non-orthogonal heat-conduction first guess.

TEST INFRASTRUCTURE ONLY (see the package header).

Paper references:
  * section "Geometry module": a periodic cell meshed by polygons (GMSH
    Delaunay triangles in the paper; ``inputs.gen.unstructured_2d`` makes the
    non-orthogonal stand-in meshes used here);
  * Appendix A (the aMFP-BTE): the mesh enters only through the face vectors
    R_ij = A_ij n_ij / V_i.  For direction s the upwind operator A_l has
    sum_f ReLu(s . n_f) A_f / V_i on the diagonal of row i (wall faces
    included) and -ReLu(-s . n_f) A_f / V_i towards the upwind neighbour j;
    inflow through a wall carries T_w, inflow across the periodic plane of the
    gradient axis carries the applied difference;
  * Appendix "Heat conduction equation", Eqs. (balance)-(final2): the face
    gradient is the primary (two-point) part along the centroid line plus the
    secondary flux, which is taken from the previous iterate (Eqs. grad5,
    grad3, grad2, final, pert2); cell gradients by least squares over the
    neighbours (Eqs. lq, mm), face gradients interpolated between the two
    cells.

Geometry (plain definitions): polygon area by the shoelace formula, centroid
of the polygon's area, face length and the outward unit normal of each
counter-clockwise edge, (dy, -dx) / |e|.  An interior face joins solid cells
i and j; d_ij runs from the centroid of i to the centroid of j's periodic
image seen from i, and that image carries T_j + delta dT with
T(x + L_g) = T(x) - dT along the gradient axis (delta = -(image shift along
g)).  Faces towards pore cells are diffuse walls.  Wall faces are numbered by
(solid cell, corner order), interior faces by first appearance in the same
order.

Readings where the appendix is ambiguous:
  * Eq. (ortho) and Eq. (lq) give the periodic term R^P opposite signs; both
    are read as the difference to j's image, T_j + delta dT - T_i;
  * the face gradient is the linear interpolation of the two cell gradients
    at the point where d_ij crosses the face: g_f = (1 - w) g_i + w g_j with
    w the fraction of d_ij from i to that point (the appendix names the
    distance but neither its normalisation nor which cell it weighs);
  * a cell with fewer independent neighbour directions than dimensions (a
    triangle with two wall faces) takes the minimum-norm least-squares
    gradient;
  * the diagonal of Eq. (final) sums over k with n_ik . d_ik (the printed
    n_ij . d_ik is read as an index slip).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .material import Material, wall_weights


class UMesh:
    def __init__(self, L, nodes, cells, shifts, solid, grad_axis=0, dT=1.0):
        self.L = (float(L[0]), float(L[1]))
        self.ndim = 2
        self.grad_axis = int(grad_axis)
        self.dT = float(dT)
        Lv = np.asarray(self.L)
        nodes = np.asarray(nodes, float)
        cells = np.asarray(cells, np.int64)
        shifts = np.asarray(shifts, np.int64)
        sol = np.asarray(solid, bool).ravel()
        self.n_cells = len(cells)
        self.cells = np.nonzero(sol)[0]                 # solid index -> cell
        self.n_solid = len(self.cells)
        self.sid = -np.ones(self.n_cells, np.int64)
        self.sid[self.cells] = np.arange(self.n_solid)
        self.volume_box = float(Lv[0] * Lv[1])
        # corner positions of every cell in its own frame
        P = nodes[cells] + shifts * Lv                  # (n_cells, nv, 2)
        Q = np.roll(P, -1, axis=1)
        cross = P[:, :, 0] * Q[:, :, 1] - Q[:, :, 0] * P[:, :, 1]
        area = 0.5 * cross.sum(axis=1)
        if np.any(area <= 0):
            raise ValueError("cells must be counter-clockwise and non-degenerate")
        cx = ((P[:, :, 0] + Q[:, :, 0]) * cross).sum(axis=1) / (6 * area)
        cy = ((P[:, :, 1] + Q[:, :, 1]) * cross).sum(axis=1) / (6 * area)
        cen = np.stack([cx, cy], axis=1)
        self.V = area[self.cells]
        self.xc = cen[self.cells]
        # edges keyed by their two node ids and the relative shift of the
        # second node, so that both sides of a face find each other
        nv = cells.shape[1]
        edges = {}
        for c in range(self.n_cells):
            for k in range(nv):
                a, b = cells[c, k], cells[c, (k + 1) % nv]
                sa, sb = shifts[c, k], shifts[c, (k + 1) % nv]
                key = (a, b, tuple(sb - sa)) if a < b else (b, a, tuple(sa - sb))
                edges.setdefault(key, []).append((c, k))
        for key, occ in edges.items():
            if len(occ) != 2:
                raise ValueError(f"edge {key} is not shared by exactly two cells")
        fi, fj, fA, fn, fd, fdel, fw, fmid = [], [], [], [], [], [], [], []
        wi, wA, wn = [], [], []
        seen = set()
        self._face_of = {}
        # per solid cell, its faces in corner order: (kind, index, sign)
        self.cell_faces = [[] for _ in range(self.n_solid)]
        for c in self.cells:
            i = self.sid[c]
            for k in range(nv):
                a, b = cells[c, k], cells[c, (k + 1) % nv]
                sa, sb = shifts[c, k], shifts[c, (k + 1) % nv]
                key = (a, b, tuple(sb - sa)) if a < b else (b, a, tuple(sa - sb))
                pa, pb = P[c, k], P[c, (k + 1) % nv]
                e = pb - pa
                length = float(np.hypot(e[0], e[1]))
                nrm = np.array([e[1], -e[0]]) / length
                other = [o for o in edges[key] if o != (c, k)][0]
                c2, k2 = other
                if not sol[c2]:
                    self.cell_faces[i].append(("w", len(wi), 1))
                    wi.append(i); wA.append(length); wn.append(nrm)
                    continue
                if key in seen:
                    f = self._face_of[key]
                    self.cell_faces[i].append(("f", f, -1))
                    continue
                seen.add(key)
                # image offset bringing c2 into c's frame: node a sits at
                # shifts[c, k] in c and at the shift of the same node in c2
                ka = [q for q in range(nv) if cells[c2, q] == a]
                off = None
                for q in ka:
                    cand = shifts[c, k] - shifts[c2, q]
                    qb = [r for r in range(nv) if cells[c2, r] == b]
                    if any(np.array_equal(shifts[c, (k + 1) % nv] - shifts[c2, r], cand) for r in qb):
                        off = cand
                        break
                if off is None:
                    raise ValueError("inconsistent periodic shifts on a shared edge")
                j = self.sid[c2]
                d = cen[c2] + off * Lv - cen[c]
                self._face_of[key] = len(fi)
                self.cell_faces[i].append(("f", len(fi), 1))
                fi.append(i); fj.append(j); fA.append(length); fn.append(nrm); fd.append(d)
                fdel.append(-float(off[self.grad_axis]))
                # where the centroid line crosses the face: fraction of d
                t = float(np.dot(pa - cen[c], nrm) / np.dot(d, nrm))
                fw.append(t)
                fmid.append(0.5 * (pa + pb))
        self.fi = np.asarray(fi, np.int64)
        self.fj = np.asarray(fj, np.int64)
        self.fA = np.asarray(fA)
        self.fn = np.asarray(fn).reshape(-1, 2)
        self.fd = np.asarray(fd).reshape(-1, 2)
        self.fdelta = np.asarray(fdel)
        self.fw = np.asarray(fw)
        self.n_faces = len(self.fi)
        self.wall_cell = np.asarray(wi, np.int64)
        self.wA = np.asarray(wA)
        self.wn = np.asarray(wn).reshape(-1, 2)
        self.n_walls = len(self.wall_cell)

    def wall_normal(self, f):
        return self.wn[f]

    def cut_faces(self):
        """Interior faces across the periodic plane of the gradient axis,
        oriented from the cell on the + side of the cut (delta = +1)."""
        out = []
        for f in range(self.n_faces):
            if self.fdelta[f] > 0:
                out.append((f, self.fi[f], self.fj[f], self.fn[f], self.fd[f]))
            elif self.fdelta[f] < 0:
                out.append((f, self.fj[f], self.fi[f], -self.fn[f], -self.fd[f]))
        return out

    @property
    def A_perp(self):
        return self.L[1 - self.grad_axis]


def upwind_operator_u(um, s):
    """Sparse A_l (n_solid^2), the periodic-jump inflow (times dT) and the
    wall-inflow matrix Bw (n_solid x n_walls) for direction s."""
    n = um.n_solid
    s = np.asarray(s, float)[:2]
    diag = np.zeros(n)
    jump = np.zeros(n)
    r, c, v = [], [], []
    for f in range(um.n_faces):
        i, j, nrm, A = um.fi[f], um.fj[f], um.fn[f], um.fA[f]
        sn = float(np.dot(s, nrm))
        if sn > 0:          # out of i, into j
            diag[i] += sn * A / um.V[i]
            r.append(j); c.append(i); v.append(-sn * A / um.V[j])
            jump[j] += sn * A / um.V[j] * (-um.fdelta[f]) * um.dT
        elif sn < 0:        # out of j, into i
            diag[j] += -sn * A / um.V[j]
            r.append(i); c.append(j); v.append(sn * A / um.V[i])
            jump[i] += -sn * A / um.V[i] * um.fdelta[f] * um.dT
    br, bc, bv = [], [], []
    for w in range(um.n_walls):
        i, nrm, A = um.wall_cell[w], um.wn[w], um.wA[w]
        sn = float(np.dot(s, nrm))
        if sn > 0:
            diag[i] += sn * A / um.V[i]
        elif sn < 0:
            br.append(i); bc.append(w); bv.append(-sn * A / um.V[i])
    A_l = sp.csr_matrix((np.concatenate([diag, v]), (np.concatenate([np.arange(n), r]),
                                                      np.concatenate([np.arange(n), c]))), shape=(n, n))
    Bw = sp.csr_matrix((bv, (br, bc)), shape=(n, um.n_walls))
    return A_l, jump, Bw


# ---------------------------------------------------------------------------
# heat conduction with the explicit secondary flux
# ---------------------------------------------------------------------------

def lsq_gradient_weights(um):
    """Per solid cell: the neighbour list, d to each neighbour's image, the
    jump of each image, and W_i = pinv(M_i) (rows of M_i: d_ij)."""
    nb = [[] for _ in range(um.n_solid)]
    for f in range(um.n_faces):
        i, j, d, dl = um.fi[f], um.fj[f], um.fd[f], um.fdelta[f]
        nb[i].append((j, d, dl))
        nb[j].append((i, -d, -dl))
    W = []
    for i in range(um.n_solid):
        if nb[i]:
            M = np.array([d for _, d, _ in nb[i]])
            W.append(np.linalg.pinv(M))
        else:
            W.append(np.zeros((2, 0)))
    return nb, W


def cell_gradients(um, T, nb, W):
    """Eqs. (lq), (mm): least-squares gradient of T at every solid cell."""
    g = np.zeros((um.n_solid, 2))
    for i in range(um.n_solid):
        if nb[i]:
            q = np.array([T[j] + dl * um.dT - T[i] for j, _, dl in nb[i]])
            g[i] = W[i] @ q
    return g


def face_gradients(um, g):
    w = um.fw[:, None]
    return (1 - w) * g[um.fi] + w * g[um.fj]


def fourier_parts(um, kappa_axis):
    """Volume-scaled Eq. (final): the primary-flux Laplacian (a_f on the
    off-diagonals, a_f = A_f n.K n / (n . d)), the perturbation P (Eq. pert2)
    and the vectors c_f = A_f (d (n.K n)/(n.d) - K n) of the secondary term."""
    K = np.diag(np.asarray(kappa_axis, float)[:2])
    n = um.n_solid
    nKn = np.einsum("fa,ab,fb->f", um.fn, K, um.fn)
    nd = np.einsum("fa,fa->f", um.fn, um.fd)
    a = um.fA * nKn / nd
    rows = np.concatenate([um.fi, um.fj, um.fi, um.fj])
    cols = np.concatenate([um.fj, um.fi, um.fi, um.fj])
    vals = np.concatenate([a, a, -a, -a])
    Lap = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    P = np.zeros(n)
    np.add.at(P, um.fi, -a * um.fdelta * um.dT)
    np.add.at(P, um.fj, a * um.fdelta * um.dT)
    cvec = um.fA[:, None] * (um.fd * (nKn / nd)[:, None] - um.fn @ K)
    return Lap, P, cvec


def secondary(um, cvec, gf):
    """B of Eq. (final), volume-scaled: sum over faces of g_f . c_f (with the
    sign of each side)."""
    b = np.einsum("fa,fa->f", gf, cvec)
    B = np.zeros(um.n_solid)
    np.add.at(B, um.fi, b)
    np.add.at(B, um.fj, -b)
    return B


def fourier_nonorth(um, kappa_axis, tol=1e-13, max_iter=1000, primary_only=False):
    """Eq. (final2): A T^(n) = S T^(n-1) + P, each step a direct solve with
    the mean fixed to zero, until max |T^(n) - T^(n-1)| <= tol max |T^(n)|.
    Returns (T over solid cells, kappa_F, iterations)."""
    Lap, P, cvec = fourier_parts(um, kappa_axis)
    nb, W = lsq_gradient_weights(um)
    n = um.n_solid
    one = np.ones((n, 1))
    Bm = sp.bmat([[Lap, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]], format="csc")
    lu = spla.splu(Bm)
    T = np.zeros(n)
    it = 0
    for it in range(1, max_iter + 1):
        B = np.zeros(n) if primary_only else secondary(um, cvec, face_gradients(um, cell_gradients(um, T, nb, W)))
        Tn = lu.solve(np.concatenate([P + B, [0.0]]))[:n]
        done = np.max(np.abs(Tn - T)) <= tol * max(np.max(np.abs(Tn)), 1e-300)
        T = Tn
        if done or primary_only:
            break
    return T, kappa_fourier_u(um, kappa_axis, T, nb, W, primary_only), it


def kappa_fourier_u(um, kappa_axis, T, nb=None, W=None, primary_only=False):
    """Heat flow through the periodic cut of the gradient axis (primary +
    secondary face flux) times L_g / (dT A_perp)."""
    K = np.diag(np.asarray(kappa_axis, float)[:2])
    if nb is None:
        nb, W = lsq_gradient_weights(um)
    gf = np.zeros((um.n_faces, 2)) if primary_only else face_gradients(um, cell_gradients(um, T, nb, W))
    tot = 0.0
    for f, i, j, nrm, d in um.cut_faces():
        nKn = float(nrm @ K @ nrm)
        nd = float(nrm @ d)
        g = gf[f]
        # K grad T . n A_f with grad T = primary + secondary, i's frame (j's image hotter)
        F = um.fA[f] * (nKn / nd * (T[j] + um.dT - T[i]) + g @ K @ nrm - nKn * (g @ d) / nd)
        tot += F
    return um.L[um.grad_axis] / (um.dT * um.A_perp) * tot


# ---------------------------------------------------------------------------
# the aMFP-BTE on the unstructured mesh
# ---------------------------------------------------------------------------

class UProblem:
    """Mesh + material + per-direction operators; the same interface as
    oracle.bte.Problem, so oracle.bte.source_iteration runs it unchanged."""

    def __init__(self, work, fourier_tol=1e-13):
        self.mesh = um = UMesh(work.L, work.nodes, work.cells, work.shifts, work.solid, work.grad_axis, work.dT)
        self.mat = mat = Material(work.mfp, work.dirs, work.dir_w, work.kappa_m, work.grad_axis)
        sig = work.sigma
        self.sigma = np.ones(um.n_solid) if sig is None else np.asarray(sig, float)[um.cells].copy()
        self.ops = [upwind_operator_u(um, mat.dirs[l]) for l in range(mat.n_dir)]
        self.wout = np.zeros((um.n_walls, mat.n_mfp, mat.n_dir))
        for f in range(um.n_walls):
            self.wout[f] = wall_weights(mat.S, um.wn[f])
        self.wall_cell = um.wall_cell
        self.fourier_tol = fourier_tol
        self._lu = {}

    def fourier(self):
        T, kF, _ = fourier_nonorth(self.mesh, self.mat.kappa_axis, tol=self.fourier_tol)
        return T, kF

    def system_matrix(self, m, l):
        return (sp.diags(self.sigma) + self.mat.mfp[m] * self.ops[l][0]).tocsc()

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

    def kappa_cc_system(self, m, l, x):
        um, g = self.mesh, self.mesh.grad_axis
        return um.L[g] / (um.dT * um.volume_box) * self.mat.S[m, l, g] * float(np.dot(um.V, x))

    def kappa_face_system(self, m, l, x):
        um = self.mesh
        S = self.mat.S[m, l, :2]
        tot = 0.0
        for f, i, j, nrm, _ in um.cut_faces():
            sn = float(S @ nrm)
            up = x[i] if sn > 0 else x[j] + um.dT
            tot -= um.fA[f] * sn * up          # flow from i to j, counted along +g
        return um.L[um.grad_axis] / (um.dT * um.A_perp) * tot


def dense_coupled_matrix_u(prob):
    """The whole coupled system M T = p over all DoF (T_L and T_w
    eliminated), assembled cell by cell from each cell's own face list and
    independently of ``upwind_operator_u`` (tiny meshes only)."""
    um, mat = prob.mesh, prob.mat
    ns, nm, nd = um.n_solid, mat.n_mfp, mat.n_dir
    N = ns * nm * nd
    M = np.zeros((N, N))
    p = np.zeros(N)

    def idx(m, l, i):
        return (m * nd + l) * ns + i

    for m in range(nm):
        for l in range(nd):
            s = mat.dirs[l, :2]
            lam = mat.mfp[m]
            for i in range(ns):
                r = idx(m, l, i)
                M[r, r] += prob.sigma[i]
                for m2 in range(nm):
                    for l2 in range(nd):
                        M[r, idx(m2, l2, i)] -= prob.sigma[i] * mat.D[m2, l2]
                for kind, f, sign in um.cell_faces[i]:
                    if kind == "w":
                        nrm, A = um.wn[f], um.wA[f]
                    else:
                        nrm, A = sign * um.fn[f], um.fA[f]
                    sn = float(s @ nrm)
                    coef = lam * A / um.V[i]
                    if sn > 0:
                        M[r, r] += coef * sn
                        continue
                    if sn == 0:
                        continue
                    if kind == "f":
                        j = um.fj[f] if sign > 0 else um.fi[f]
                        delta = um.fdelta[f] * sign
                        M[r, idx(m, l, j)] -= coef * (-sn)
                        p[r] += coef * (-sn) * delta * um.dT
                    else:
                        # wall: T_w = sum over systems leaving through it
                        q = np.maximum(np.einsum("mla,a->ml", mat.S[:, :, :2], nrm), 0.0)
                        q /= q.sum()
                        for m2 in range(nm):
                            for l2 in range(nd):
                                if q[m2, l2] > 0:
                                    M[r, idx(m2, l2, i)] -= coef * (-sn) * q[m2, l2]
    return M, p


def dense_solve_u(prob):
    """Solve the singular coupled system with the gauge sum_i T_L,i = 0;
    T has shape (n_mfp, n_dir, n_solid)."""
    um, mat = prob.mesh, prob.mat
    M, p = dense_coupled_matrix_u(prob)
    N = len(p)
    ns = um.n_solid
    c = np.zeros(N)
    for m in range(mat.n_mfp):
        for l in range(mat.n_dir):
            c[(m * mat.n_dir + l) * ns:(m * mat.n_dir + l + 1) * ns] = mat.D[m, l]
    B = np.zeros((N + 1, N + 1))
    B[:N, :N] = M
    B[:N, N] = 1.0
    B[N, :N] = c
    sol = np.linalg.solve(B, np.concatenate([p, [0.0]]))
    return sol[:N].reshape(mat.n_mfp, mat.n_dir, ns)
