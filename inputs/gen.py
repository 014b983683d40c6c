"""Seeded synthetic workloads for the aMFP-BTE hot path.

This module produces *inputs only*: grid sizes, solid masks, cell sizes, the
MFP grid, the per-MFP conductivity kernel, the direction set with its
quadrature weights and the relaxation-rate multiplier field.  It holds none of
the method's arithmetic (no material weights, no operators, no reductions), so
both the CPU oracle and the GPU library can consume the same arrays without
sharing any solver code.

Stand-in for the paper's data: the paper runs ab-initio silicon at 300 K
(section "Material", file ``rta_Si_300``) which is not available here.  A
synthetic Si-like kernel replaces it: per-MFP conductivity weights follow a
lognormal in the MFP (median 300 nm, sigma_ln = 1.5), evaluated at the MFP
nodes in log space and normalised to a bulk conductivity of 150 W/m/K.

Directions follow the "uniform spherical grid" of Appendix A: in 2D the
in-plane angles phi_l = 2 pi (l + 1/2) / N_Omega with equal weights; in 3D
polar bins theta_k = (k + 1/2) pi / N_theta (bin-centre directions, weights
equal to the bin's solid angle over 4 pi) times uniform azimuths.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NM = 1e-9


@dataclass
class Workload:
    """One geometry + material description (all host arrays, SI units)."""

    name: str
    ndim: int
    n: tuple            # (nx, ny, nz); nz = 1 in 2D
    L: tuple            # (Lx, Ly, Lz) in metres
    periodic: tuple     # per axis, 1 = periodic
    solid: np.ndarray   # uint8, shape (nz, ny, nx) flattened x-fastest when raveled
    grad_axis: int
    dT: float
    mfp: np.ndarray     # (n_mfp,) metres
    kappa_m: np.ndarray  # (n_mfp,) W/m/K
    dirs: np.ndarray    # (n_dir, ndim) unit vectors
    dir_w: np.ndarray   # (n_dir,) weights summing to 1
    sigma: np.ndarray | None = None   # per-cell multiplier (flattened), None => 1
    meta: dict = field(default_factory=dict)
    # optional mode table: (F (n_modes, ndim) vectorial MFPs in metres,
    # alpha (n_modes,) C/tau weights); when set, the grid weights come from it
    modes: tuple | None = None
    # with a mode table: solve one system per mode (Eq. iter3) instead of
    # interpolating onto the (MFP, direction) grid
    modes_exact: bool = False

    @property
    def n_cells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_solid(self) -> int:
        return int(self.solid.sum())

    @property
    def n_systems(self) -> int:
        return int(len(self.mfp) * len(self.dir_w))

    @property
    def dof(self) -> int:
        return self.n_solid * self.n_systems


# --------------------------------------------------------------------------
# material inputs
# --------------------------------------------------------------------------

def mfp_grid(n_mfp: int, lo: float, hi: float) -> np.ndarray:
    """MFP magnitudes log-spaced from lo to hi (metres)."""
    return np.logspace(math.log10(lo), math.log10(hi), n_mfp)


def lognormal_kernel(mfp: np.ndarray, median: float = 300 * NM,
                     sigma_ln: float = 1.5, kappa_bulk: float = 150.0) -> np.ndarray:
    """Per-MFP conductivity weights: lognormal density in ln(Lambda) sampled at
    the nodes (node rule in log space), normalised to sum to kappa_bulk."""
    w = np.exp(-np.log(mfp / median) ** 2 / (2.0 * sigma_ln ** 2))
    return kappa_bulk * w / w.sum()


def directions_2d(n_dir: int):
    phi = 2.0 * math.pi * (np.arange(n_dir) + 0.5) / n_dir
    dirs = np.stack([np.cos(phi), np.sin(phi)], axis=1)
    return dirs, np.full(n_dir, 1.0 / n_dir)


def directions_3d(n_theta: int, n_phi: int):
    k = np.arange(n_theta)
    th = (k + 0.5) * math.pi / n_theta
    th_lo = k * math.pi / n_theta
    th_hi = (k + 1) * math.pi / n_theta
    w_th = 0.5 * (np.cos(th_lo) - np.cos(th_hi))   # solid angle / 4 pi
    ph = 2.0 * math.pi * (np.arange(n_phi) + 0.5) / n_phi
    dirs, w = [], []
    for a in range(n_theta):
        for b in range(n_phi):
            dirs.append([math.sin(th[a]) * math.cos(ph[b]),
                         math.sin(th[a]) * math.sin(ph[b]),
                         math.cos(th[a])])
            w.append(w_th[a] / n_phi)
    w = np.asarray(w)
    return np.asarray(dirs), w / w.sum()


# --------------------------------------------------------------------------
# geometry inputs (rasterisation of pores onto cell centres)
# --------------------------------------------------------------------------

def square_block_mask(nx: int, ny: int, lo: int, hi: int) -> np.ndarray:
    s = np.ones((1, ny, nx), np.uint8)
    s[0, lo:hi, lo:hi] = 0
    return s


def circles_mask(nx: int, ny: int, Lx: float, Ly: float, centres, radii) -> np.ndarray:
    """Pore iff a cell centre lies strictly inside a circle or one of its
    periodic images (pores crossing the boundary are repeated)."""
    hx, hy = Lx / nx, Ly / ny
    xc = (np.arange(nx) + 0.5) * hx
    yc = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(xc, yc)
    pore = np.zeros((ny, nx), bool)
    for (cx, cy), r in zip(centres, radii):
        for ox in (-Lx, 0.0, Lx):
            for oy in (-Ly, 0.0, Ly):
                pore |= (X - cx - ox) ** 2 + (Y - cy - oy) ** 2 < r * r
    return (~pore).astype(np.uint8)[None]


def stripe_mask(nx: int, ny: int, n_solid_rows: int) -> np.ndarray:
    """Channel: solid rows [0, n_solid_rows), pore rows above (diffuse walls)."""
    s = np.zeros((1, ny, nx), np.uint8)
    s[0, :n_solid_rows, :] = 1
    return s


def gaussian_random_field(n: int, ell: float, rng: np.random.Generator) -> np.ndarray:
    """Smooth GRF on an n x n torus: white noise filtered by exp(-k^2 ell^2/4)
    (covariance exp(-r^2 / 2 ell^2), ell in cells), standardised."""
    w = rng.standard_normal((n, n))
    k = 2.0 * math.pi * np.fft.fftfreq(n)
    KX, KY = np.meshgrid(k, k)
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * np.exp(-(KX ** 2 + KY ** 2) * ell ** 2 / 4.0)))
    return (f - f.mean()) / f.std()


def sigma_from_field(z: np.ndarray) -> np.ndarray:
    """Map a standard-normal field to sigma = 2^(2 Phi(z) - 1) in (0.5, 2)."""
    from scipy.special import ndtr
    return np.power(2.0, 2.0 * ndtr(z) - 1.0)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def _mat2d(n_dir, n_mfp, hi):
    mfp = mfp_grid(n_mfp, 1 * NM, hi)
    dirs, w = directions_2d(n_dir)
    return mfp, lognormal_kernel(mfp), dirs, w


def config1() -> Workload:
    """32x32 periodic cell, centred 16x16 square pore (porosity 0.25), L=100 nm,
    24 directions, 10 MFPs 1 nm..10 um, FP64."""
    mfp, km, dirs, w = _mat2d(24, 10, 10e-6)
    L = 100 * NM
    return Workload("cfg1", 2, (32, 32, 1), (L, L, L), (1, 1, 0),
                    square_block_mask(32, 32, 8, 24), 0, 1.0, mfp, km, dirs, w)


def config2(n: int = 128, n_dir: int = 48, n_mfp: int = 30) -> Workload:
    """128x128 periodic cell, one centred circular pore r = L*U[0.2,0.35]
    (seeded), L=100 nm, 48 directions, 30 MFPs 1 nm..100 um."""
    rng = np.random.default_rng(2106027642)
    L = 100 * NM
    r = L * rng.uniform(0.2, 0.35)
    mfp, km, dirs, w = _mat2d(n_dir, n_mfp, 100e-6)
    solid = circles_mask(n, n, L, L, [(L / 2, L / 2)], [r])
    return Workload("cfg2", 2, (n, n, 1), (L, L, L), (1, 1, 0), solid, 0, 1.0,
                    mfp, km, dirs, w, meta={"pore_radius": r})


def config3_geometry(g: int, n_dir: int = 48, n_mfp: int = 30) -> Workload:
    """Geometry g of the 64-geometry batch (seed [2106027643, g])."""
    rng = np.random.default_rng([2106027643, g])
    sizes = [48, 64, 96, 128, 192, 256]
    mfp, km, dirs, w = _mat2d(n_dir, n_mfp, 100e-6)
    while True:
        N = int(sizes[rng.integers(0, len(sizes))])
        L = rng.uniform(50, 500) * NM
        n_p = int(rng.integers(1, 5))
        phi = rng.uniform(0.10, 0.40)
        parts = rng.dirichlet(np.ones(n_p)) * phi
        radii = np.sqrt(parts * L * L / math.pi)
        h = L / N
        centres = []
        ok = True
        for k in range(n_p):
            for _ in range(200):
                c = rng.uniform(0, L, 2)
                good = True
                for (q, rq) in zip(centres, radii[:len(centres)]):
                    d = np.abs(c - np.asarray(q))
                    d = np.minimum(d, L - d)
                    if np.hypot(*d) < radii[k] + rq + 2 * h:
                        good = False
                        break
                # a pore must not touch its own periodic image
                if 2 * radii[k] + 2 * h > L:
                    good = False
                if good:
                    centres.append(tuple(c))
                    break
            else:
                ok = False
                break
        if not ok:
            continue
        solid = circles_mask(N, N, L, L, centres, radii)
        por = 1.0 - solid.mean()
        if 0.10 <= por <= 0.40:
            return Workload(f"cfg3_g{g}", 2, (N, N, 1), (L, L, L), (1, 1, 0), solid, 0, 1.0,
                            mfp, km, dirs, w,
                            meta={"centres": centres, "radii": list(radii), "porosity": por})


def config3(n_geom: int = 64):
    return [config3_geometry(g) for g in range(n_geom)]


def config4(n: int = 128) -> Workload:
    """128x128 periodic cell without pores, L=100 nm, 48 dirs, 30 MFPs, with a
    smooth seeded relaxation-rate multiplier sigma in (0.5, 2)."""
    rng = np.random.default_rng(2106027644)
    L = 100 * NM
    mfp, km, dirs, w = _mat2d(48, 30, 100e-6)
    z = gaussian_random_field(n, 8.0, rng)
    sigma = sigma_from_field(z).ravel()
    return Workload("cfg4", 2, (n, n, 1), (L, L, L), (1, 1, 0), np.ones((1, n, n), np.uint8),
                    0, 1.0, mfp, km, dirs, w, sigma=sigma)


def config4_fd_cells(n: int = 128, count: int = 32) -> np.ndarray:
    rng = np.random.default_rng(2106027645)
    return rng.choice(n * n, size=count, replace=False)


def config5(nx: int = 64, nz: int = 16, n_theta: int = 12, n_phi: int = 24,
            n_mfp: int = 30) -> Workload:
    """3D membrane: nx x nx x nz grid, periodic in x and y, diffuse top/bottom,
    centred cylindrical through-pore r = 0.3 L, L = 200 nm, t = 50 nm."""
    L, t = 200 * NM, 50 * NM
    mfp = mfp_grid(n_mfp, 1 * NM, 100e-6)
    km = lognormal_kernel(mfp)
    dirs, w = directions_3d(n_theta, n_phi)
    s2 = circles_mask(nx, nx, L, L, [(L / 2, L / 2)], [0.3 * L])[0]
    solid = np.repeat(s2[None], nz, axis=0)
    return Workload("cfg5", 3, (nx, nx, nz), (L, L, t), (1, 1, 0), solid.astype(np.uint8),
                    0, 1.0, mfp, km, dirs, w)


def small_2d(nx: int, ny: int, solid=None, n_dir: int = 8, n_mfp: int = 3,
             L: float = 100 * NM, mfp_lo: float = 1 * NM, mfp_hi: float = 10e-6,
             grad_axis: int = 0, sigma=None, Ly=None) -> Workload:
    """Small 2D case for tests (fully periodic unless the mask has pores)."""
    if solid is None:
        solid = np.ones((1, ny, nx), np.uint8)
    mfp = mfp_grid(n_mfp, mfp_lo, mfp_hi)
    dirs, w = directions_2d(n_dir)
    Ly = L if Ly is None else Ly
    return Workload(f"small_{nx}x{ny}", 2, (nx, ny, 1), (L, Ly, L), (1, 1, 0),
                    np.asarray(solid, np.uint8).reshape(1, ny, nx), grad_axis, 1.0,
                    mfp, lognormal_kernel(mfp), dirs, w,
                    sigma=None if sigma is None else np.asarray(sigma, float).ravel())


def small_3d(nx: int, ny: int, nz: int, solid=None, n_theta: int = 4, n_phi: int = 8,
             n_mfp: int = 3, L: float = 200 * NM, t: float = 50 * NM,
             periodic_z: int = 0, sigma=None) -> Workload:
    if solid is None:
        solid = np.ones((nz, ny, nx), np.uint8)
    mfp = mfp_grid(n_mfp, 1 * NM, 10e-6)
    dirs, w = directions_3d(n_theta, n_phi)
    return Workload(f"small3d_{nx}x{ny}x{nz}", 3, (nx, ny, nz), (L, L, t), (1, 1, periodic_z),
                    np.asarray(solid, np.uint8).reshape(nz, ny, nx), 0, 1.0,
                    mfp, lognormal_kernel(mfp), dirs, w,
                    sigma=None if sigma is None else np.asarray(sigma, float).ravel())


def with_modes(w: Workload, n_modes: int, seed: int,
               mfp_lo: float | None = None, mfp_hi: float | None = None, dim3: bool = False,
               n_static: int = 0) -> Workload:
    """A copy of `w` whose material is a synthetic mode table.

    n_modes modes (n_modes/2 random ones and their reverses -F, so the table
    carries no net flux) with log-uniform |F| in [mfp_lo, mfp_hi] (default: a
    bit beyond the grid, so some modes are clamped), uniform random directions,
    and weights from the same lognormal kernel in ln|F| (median 300 nm,
    sigma_ln 1.5) divided by |F|^2, scaled to a bulk conductivity of 150 W/m/K
    along the gradient axis.  dim3 (2D workloads): 3D modes, directions
    uniform on the sphere (the library keeps their in-plane part); n_static
    more modes moving only along z (zero in-plane MFP), weight like the rest."""
    import dataclasses
    rng = np.random.default_rng(seed)
    nd = w.ndim
    lo = w.mfp.min() / 2 if mfp_lo is None else mfp_lo
    hi = w.mfp.max() * 2 if mfp_hi is None else mfp_hi
    half = n_modes // 2
    lam = np.exp(rng.uniform(np.log(lo), np.log(hi), half))
    if dim3 and nd == 2:
        v = rng.standard_normal((half, 3))
        s = v / np.linalg.norm(v, axis=1, keepdims=True)
        F = np.concatenate([lam[:, None] * s, -lam[:, None] * s])
        lam2 = np.concatenate([lam, lam])
        alpha = np.exp(-np.log(lam2 / 300e-9) ** 2 / (2 * 1.5 ** 2)) / lam2 ** 2
        if n_static:
            fz = np.exp(rng.uniform(np.log(lo), np.log(hi), n_static))
            F = np.concatenate([F, np.stack([0 * fz, 0 * fz, fz], axis=1)])
            alpha = np.concatenate([alpha, np.exp(-np.log(fz / 300e-9) ** 2 / (2 * 1.5 ** 2)) / fz ** 2])
        alpha *= 150.0 / float(np.sum(alpha * F[:, w.grad_axis] ** 2))
        return dataclasses.replace(w, modes=(F, alpha), name=w.name + f"_modes3d{n_modes}")
    if nd == 2:
        ph = rng.uniform(0.0, 2.0 * math.pi, half)
        s = np.stack([np.cos(ph), np.sin(ph)], axis=1)
    else:
        v = rng.standard_normal((half, 3))
        s = v / np.linalg.norm(v, axis=1, keepdims=True)
    F = np.concatenate([lam[:, None] * s, -lam[:, None] * s])
    lam = np.concatenate([lam, lam])
    dens = np.exp(-np.log(lam / 300e-9) ** 2 / (2 * 1.5 ** 2))
    alpha = dens / lam ** 2
    alpha *= 150.0 / float(np.sum(alpha * F[:, w.grad_axis] ** 2))
    return dataclasses.replace(w, modes=(F, alpha), name=w.name + f"_modes{n_modes}")


# ---------------------------------------------------------------------------
# Unstructured (non-orthogonal) 2D meshes.  The paper meshes its geometries
# with GMSH Delaunay triangles (section "Geometry module"); there is no mesher
# here, so a periodic node lattice is displaced by a smooth periodic field
# (distorted quadrilaterals, or triangles from splitting each quadrilateral
# along alternating diagonals).  Only node positions and connectivity are
# produced: areas, centroids, normals and every operator are the consumers'.
# ---------------------------------------------------------------------------

@dataclass
class UWorkload:
    """A periodic 2D cell meshed by polygons (counter-clockwise node lists).

    nodes:  (n_nodes, 2) positions in metres, inside [0, Lx) x [0, Ly) before
            the displacement;
    cells:  (n_cells, nv) node ids (nv = 3 or 4);
    shifts: (n_cells, nv, 2) periodic image of each corner: the corner lies at
            nodes[id] + shifts * (Lx, Ly);
    solid:  (n_cells,) uint8 (0 = pore).
    Both axes are periodic; the applied difference dT is along grad_axis."""

    name: str
    L: tuple
    nodes: np.ndarray
    cells: np.ndarray
    shifts: np.ndarray
    solid: np.ndarray
    grad_axis: int
    dT: float
    mfp: np.ndarray
    kappa_m: np.ndarray
    dirs: np.ndarray
    dir_w: np.ndarray
    sigma: np.ndarray | None = None
    meta: dict = field(default_factory=dict)
    ndim: int = 2

    @property
    def n_cells(self) -> int:
        return int(len(self.cells))

    @property
    def n_solid(self) -> int:
        return int(self.solid.sum())

    @property
    def n_systems(self) -> int:
        return int(len(self.mfp) * len(self.dirs))


def unstructured_2d(nx: int, ny: int, L: float = 100 * NM, Ly: float | None = None, amp: float = 0.25,
                    tri: bool = True, seed: int = 0, pores=(), n_dir: int = 8, n_mfp: int = 3,
                    mfp_lo: float = 1 * NM, mfp_hi: float = 10e-6, grad_axis: int = 0,
                    sigma=None) -> UWorkload:
    """nx x ny node lattice displaced by amp * h times a seeded sum of four
    periodic Fourier modes (amp = 0: the orthogonal grid); quadrilaterals, or
    two triangles per quadrilateral.  pores: ((cx, cy), r) circles (with
    periodic images) removing the cells whose undisplaced centre lies inside."""
    Ly = L if Ly is None else Ly
    hx, hy = L / nx, Ly / ny
    rng = np.random.default_rng([2106027646, seed])
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    X0, Y0 = I.ravel() * hx, J.ravel() * hy
    disp = np.zeros((nx * ny, 2))
    if amp:
        for axis, h in ((0, hx), (1, hy)):
            f = np.zeros(nx * ny)
            for p, q in ((1, 0), (0, 1), (1, 1), (2, 1)):
                a, ph = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
                f += a * np.sin(2 * np.pi * (p * X0 / L + q * Y0 / Ly) + ph)
            disp[:, axis] = amp * h * f / max(np.max(np.abs(f)), 1e-300)
    nodes = np.stack([X0, Y0], axis=1) + disp

    def corner(i, j):
        return (i % nx) + nx * (j % ny), (i // nx, j // ny)

    cells, shifts, centres = [], [], []
    for j in range(ny):
        for i in range(nx):
            q = [(i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)]
            if tri:
                if (i + j) % 2 == 0:
                    polys = [[q[0], q[1], q[2]], [q[0], q[2], q[3]]]
                else:
                    polys = [[q[0], q[1], q[3]], [q[1], q[2], q[3]]]
            else:
                polys = [q]
            for poly in polys:
                ids, sh = zip(*(corner(a, b) for a, b in poly))
                cells.append(ids)
                shifts.append(sh)
                centres.append(np.mean([(a * hx, b * hy) for a, b in poly], axis=0))
    cells = np.asarray(cells, np.int64)
    shifts = np.asarray(shifts, np.int64)
    centres = np.asarray(centres)
    pore = np.zeros(len(cells), bool)
    for (cx, cy), r in pores:
        for ox in (-L, 0.0, L):
            for oy in (-Ly, 0.0, Ly):
                pore |= (centres[:, 0] - cx - ox) ** 2 + (centres[:, 1] - cy - oy) ** 2 < r * r
    mfp = mfp_grid(n_mfp, mfp_lo, mfp_hi)
    dirs, w = directions_2d(n_dir)
    return UWorkload(f"u{'tri' if tri else 'quad'}_{nx}x{ny}_a{amp:g}", (L, Ly), nodes, cells, shifts,
                     (~pore).astype(np.uint8), grad_axis, 1.0, mfp, lognormal_kernel(mfp), dirs, w,
                     sigma=None if sigma is None else np.asarray(sigma, float).ravel(),
                     meta={"nx": nx, "ny": ny, "amp": amp, "tri": tri, "seed": seed})


CONFIGS = {"cfg1": config1, "cfg2": config2, "cfg4": config4, "cfg5": config5}
