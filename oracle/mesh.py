"""Structured finite-volume mesh with face classes (oracle).

Paper, section "Geometry module" and Appendix A: the cell is a cuboid, periodic
along every axis unless declared adiabatic; pores are carved out of the
material; the mesh enters the discrete BTE only through the face vectors
R_ij = A_ij n_ij / V_i between neighbours, the periodic pairs R^P_ij that
carry the applied temperature difference, and the wall sides g_si = A_s / V_i.
On a uniform orthogonal grid A_f / V_i = 1 / h_axis for every face.

Face classes of a solid cell's face (axis a, side -/+):
  * interior   - the neighbour (with periodic wrap) is solid;
  * jump       - an interior face that crosses the periodic boundary of the
                 gradient axis; the image across it is hotter by dT when
                 entering the cell at index 0 from below (delta = +1) and
                 colder by dT when entering the last cell from above
                 (delta = -1), i.e. T(x + L) = T(x) - dT;
  * wall       - the neighbour is a pore cell, or the face is an outer face of
                 a non-periodic axis (diffuse, thermalising surface).
Cells are numbered x fastest: c = ix + nx (iy + ny iz).
"""
from __future__ import annotations

import numpy as np


class Mesh:
    def __init__(self, n, L, solid, periodic, grad_axis=0, dT=1.0, ndim=None):
        nx, ny, nz = (int(v) for v in n)
        self.n = (nx, ny, nz)
        self.ndim = int(ndim if ndim is not None else (3 if nz > 1 else 2))
        self.L = tuple(float(v) for v in L)
        self.h = tuple(self.L[a] / self.n[a] for a in range(3))
        self.periodic = tuple(int(p) for p in periodic)
        self.grad_axis = int(grad_axis)
        self.dT = float(dT)
        if not self.periodic[self.grad_axis]:
            raise ValueError("the gradient axis must be periodic")
        sol = np.asarray(solid, np.uint8).reshape(-1)
        if sol.size != nx * ny * nz:
            raise ValueError("solid mask size mismatch")
        self.solid = sol
        self.n_cells = sol.size
        self.cells = np.nonzero(sol)[0]                  # solid index -> cell
        self.n_solid = len(self.cells)
        self.sid = -np.ones(self.n_cells, np.int64)      # cell -> solid index
        self.sid[self.cells] = np.arange(self.n_solid)
        c = self.cells
        self.coord = np.stack([c % nx, (c // nx) % ny, c // (nx * ny)], axis=1)

        nd = self.ndim
        # per solid cell, axis, side (0 = '-' face, 1 = '+' face)
        self.nbr = -np.ones((self.n_solid, nd, 2), np.int64)
        self.jump = np.zeros((self.n_solid, nd, 2))
        self.wall_id = -np.ones((self.n_solid, nd, 2), np.int64)
        walls = []
        for i in range(self.n_solid):
            for a in range(nd):
                for side in (0, 1):
                    step = 1 if side == 1 else -1
                    q = list(self.coord[i])
                    q[a] += step
                    wrapped = False
                    if q[a] < 0 or q[a] >= self.n[a]:
                        if not self.periodic[a]:
                            self.wall_id[i, a, side] = len(walls)
                            walls.append((i, a, side))
                            continue
                        q[a] %= self.n[a]
                        wrapped = True
                    cc = q[0] + nx * (q[1] + ny * q[2])
                    j = self.sid[cc]
                    if j < 0:
                        self.wall_id[i, a, side] = len(walls)
                        walls.append((i, a, side))
                        continue
                    self.nbr[i, a, side] = j
                    if wrapped and a == self.grad_axis:
                        self.jump[i, a, side] = 1.0 if side == 0 else -1.0
        self.walls = np.asarray(walls, np.int64).reshape(-1, 3)
        self.n_walls = len(self.walls)

    def wall_normal(self, f):
        _, a, side = self.walls[f]
        nvec = np.zeros(self.ndim)
        nvec[a] = 1.0 if side == 1 else -1.0
        return nvec

    def plane_pairs(self):
        """Solid pairs (j, i) across the periodic plane of the gradient axis:
        j at index N-1 and i at index 0 with equal transverse indices."""
        g = self.grad_axis
        pairs = []
        for i in range(self.n_solid):
            if self.coord[i, g] == 0:
                j = self.nbr[i, g, 0]
                if j >= 0:
                    pairs.append((j, i))
        return np.asarray(pairs, np.int64).reshape(-1, 2)

    @property
    def n_perp(self):
        return self.n_cells // self.n[self.grad_axis]
