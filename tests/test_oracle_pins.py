"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, brute force, invariants, limits), not against itself."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from inputs import gen
from oracle.bte import (Problem, dense_solve, kappa_cc, kappa_face, source_iteration,
                        upwind_operator, lattice_temperature, wall_temperature)
from oracle.fourier import dirichlet_energy_kappa, fourier_solve
from oracle.material import Material, wall_weights
from oracle.mesh import Mesh
from oracle.adjoint import adjoint_dense, adjoint_source_iteration, gradient_from
from tests._lib import on_node_modes

NM = 1e-9


# ---------------------------------------------------------------- material (a1)

@pytest.mark.parametrize("ndim", [2, 3])
def test_material_moments(ndim):
    mfp = gen.mfp_grid(7, 1 * NM, 10e-6)
    km = gen.lognormal_kernel(mfp)
    dirs, w = gen.directions_2d(24) if ndim == 2 else gen.directions_3d(6, 12)
    mat = Material(mfp, dirs, w, km)
    assert abs(km.sum() - 150.0) < 1e-12
    # bulk conductivity along the gradient axis equals the kernel sum
    assert abs(np.sum(mat.alpha * mfp[:, None] ** 2 * dirs[None, :, 0] ** 2) - 150.0) < 1e-11
    assert abs(mat.D.sum() - 1.0) < 1e-14
    assert np.all(np.abs(mat.S.sum(axis=(0, 1))) < 1e-12 * np.abs(mat.S).sum())
    if ndim == 2:
        assert abs(mat.mu - 0.5) < 1e-15
        assert abs(mat.kappa_axis[1] - 150.0) < 1e-11       # isotropic in-plane
    else:
        th = (np.arange(6) + 0.5) * math.pi / 6
        wt = 0.5 * (np.cos(np.arange(6) * math.pi / 6) - np.cos((np.arange(6) + 1) * math.pi / 6))
        mu = 0.5 * np.sum(wt * np.sin(th) ** 2)
        assert abs(mat.mu - mu) < 1e-14


def test_wall_weights_balance():
    mfp = gen.mfp_grid(5, 1 * NM, 1e-6)
    dirs, w = gen.directions_3d(4, 8)
    mat = Material(mfp, dirs, w, gen.lognormal_kernel(mfp))
    for a in range(3):
        for sgn in (-1.0, 1.0):
            n = np.zeros(3)
            n[a] = sgn
            ww = wall_weights(mat.S, n)
            assert abs(ww.sum() - 1.0) < 1e-14
            assert np.all(ww >= 0)
            # outgoing and incoming flux balance for a centrally symmetric set
            sn = np.tensordot(mat.S, n, axes=([2], [0]))
            assert abs(np.maximum(sn, 0).sum() - np.maximum(-sn, 0).sum()) < 1e-12 * np.abs(sn).sum()


# ---------------------------------------------------------------- operator (a6)

def _mesh(nx, ny, solid=None, L=100 * NM):
    if solid is None:
        solid = np.ones((1, ny, nx), np.uint8)
    return Mesh((nx, ny, 1), (L, L, L), solid, (1, 1, 0), 0, 1.0, ndim=2)


def test_upwind_row_sums_and_linear_field():
    me = _mesh(7, 5)
    dirs, _ = gen.directions_2d(12)
    xc = (me.coord[:, 0] + 0.5) * me.h[0]
    for s in dirs:
        A, jump, _ = upwind_operator(me, s)
        # no walls: outgoing flux equals incoming flux for a constant field
        assert np.max(np.abs(A @ np.ones(me.n_solid))) < 1e-15 * np.abs(A).max()
        # linear field T = -dT x / L with the periodic jump: the upwind
        # difference is exact, A T - jump = s . grad T
        T = -me.dT * xc / me.L[0]
        g = s[0] * (-me.dT / me.L[0])
        assert np.allclose(A @ T - jump, g, rtol=1e-10, atol=1e-6 / me.L[0])


def test_upwind_inverse_stochastic_and_transpose():
    me = _mesh(6, 5)
    dirs, _ = gen.directions_2d(8)
    for l, s in enumerate(dirs):
        A, _, _ = upwind_operator(me, s)
        Minv = np.linalg.inv(np.eye(me.n_solid) + 40 * NM * A.toarray())
        assert Minv.min() > -1e-14
        assert np.allclose(Minv.sum(axis=1), 1.0, atol=1e-12)
        # A_l^T equals the operator of the reversed direction
        Ar, _, _ = upwind_operator(me, -s)
        assert np.allclose(A.toarray().T, Ar.toarray(), rtol=0, atol=1e-6)


def test_upwind_transpose_with_pores():
    s = np.ones((1, 6, 6), np.uint8)
    s[0, 2:4, 1:3] = 0
    me = _mesh(6, 6, s)
    dirs, _ = gen.directions_2d(8)
    rng = np.random.default_rng(0)
    for s_ in dirs:
        A, _, _ = upwind_operator(me, s_)
        Ar, _, _ = upwind_operator(me, -s_)
        x, y = rng.standard_normal(me.n_solid), rng.standard_normal(me.n_solid)
        assert abs(y @ (A @ x) - x @ (Ar @ y)) < 1e-12 * np.abs(A).sum()


# ---------------------------------------------------------------- bulk (P3)

@pytest.mark.parametrize("sig", [1.0, 1.7])
def test_bulk_closed_form_2d(sig):
    w = gen.small_2d(8, 6, n_dir=12, n_mfp=4, sigma=np.full(48, sig))
    p = Problem(w)
    r = source_iteration(p, tol=1e-14)
    kb = w.kappa_m.sum()
    assert abs(r["kappa_cc"] - kb / sig) < 1e-12 * kb
    h = w.L[0] / 8
    kf = kb / sig + 0.5 * h * np.sum(p.mat.alpha * p.mat.mfp[:, None] * np.abs(p.mat.dirs[None, :, 0]))
    assert abs(r["kappa_face"] - kf) < 1e-12 * kb
    assert abs(r["kappa_fourier"] - kb) < 1e-12 * kb
    T, TL = r["T"], lattice_temperature(p, r["T"])
    pred = w.dT * p.mat.mfp[:, None, None] * p.mat.dirs[None, :, 0, None] / (sig * w.L[0])
    assert np.allclose(T - TL[None, None, :], pred, rtol=1e-10, atol=1e-12)


def test_bulk_closed_form_3d_with_walls_periodic_z():
    w = gen.small_3d(4, 4, 3, n_theta=4, n_phi=8, n_mfp=3, periodic_z=1)
    p = Problem(w)
    r = source_iteration(p, tol=1e-14)
    assert abs(r["kappa_cc"] - 150.0) < 1e-11
    assert abs(r["kappa_fourier"] - 150.0) < 1e-11


# ---------------------------------------------------------------- channel (P4)

def _channel_kappa(p, n_rows, ny, axis_perp, sig=1.0):
    mat, me = p.mat, p.mesh
    tot = 0.0
    for m in range(mat.n_mfp):
        for l in range(mat.n_dir):
            kml = mat.alpha[m, l] * mat.mfp[m] ** 2 * mat.dirs[l, 0] ** 2
            r = mat.mfp[m] * abs(mat.dirs[l, axis_perp]) / (sig * me.h[axis_perp])
            q = r / (1 + r)
            tot += kml / sig * (n_rows - q * (1 - q ** n_rows) / (1 - q))
    return tot / ny


def test_channel_closed_form_2d():
    ny, nh = 10, 6
    w = gen.small_2d(5, ny, solid=gen.stripe_mask(5, ny, nh), n_dir=16, n_mfp=4,
                     mfp_hi=1e-6)
    p = Problem(w)
    r = source_iteration(p, tol=1e-14)
    pred = _channel_kappa(p, nh, ny, 1)
    assert abs(r["kappa_cc"] - pred) < 1e-12 * pred
    # Fourier: only the solid fraction conducts
    assert abs(r["kappa_fourier"] - 150.0 * nh / ny) < 1e-11
    # walls take the lattice temperature of their cell
    TL = lattice_temperature(p, r["T"])
    assert np.allclose(wall_temperature(p, r["T"]), TL[p.wall_cell], atol=1e-12)


def test_channel_closed_form_3d_slab():
    nz = 5
    w = gen.small_3d(3, 3, nz, n_theta=6, n_phi=8, n_mfp=3)
    p = Problem(w)
    r = source_iteration(p, tol=1e-14)
    pred = _channel_kappa(p, nz, nz, 2)
    assert abs(r["kappa_cc"] - pred) < 1e-12 * pred


# ---------------------------------------------------------------- brute force (P5)

@pytest.mark.parametrize("nx,ny,block", [(4, 4, (1, 3, 1, 3)), (6, 5, (1, 3, 2, 5)), (5, 4, (0, 2, 3, 4))])
def test_source_iteration_matches_dense(nx, ny, block):
    s = np.ones((1, ny, nx), np.uint8)
    y0, y1, x0, x1 = block
    s[0, y0:y1, x0:x1] = 0
    w = gen.small_2d(nx, ny, solid=s, n_dir=8, n_mfp=3)
    p = Problem(w)
    Td, _, _, border = dense_solve(p)
    assert abs(border) < 1e-12
    r = source_iteration(p, tol=1e-15, max_passes=20000)
    assert abs(r["kappa_cc"] - kappa_cc(p, Td)) < 1e-11 * abs(kappa_cc(p, Td))
    assert abs(r["kappa_face"] - kappa_face(p, Td)) < 1e-11 * abs(kappa_face(p, Td))
    TLd = lattice_temperature(p, Td)
    assert np.max(np.abs(r["T_L"] - (TLd - TLd.mean()))) < 1e-11


def test_dense_3d_membrane_small():
    s = np.ones((2, 3, 3), np.uint8)
    s[:, 1, 1] = 0
    w = gen.small_3d(3, 3, 2, solid=s, n_theta=2, n_phi=4, n_mfp=2)
    p = Problem(w)
    Td, _, _, _ = dense_solve(p)
    r = source_iteration(p, tol=1e-15, max_passes=20000)
    assert abs(r["kappa_cc"] - kappa_cc(p, Td)) < 1e-11 * abs(kappa_cc(p, Td))


# ---------------------------------------------------------------- conservation (P6)

def _face_flux_divergence(p, T, T_w):
    """Total upwind energy flux out of each solid cell, built face by face."""
    me, mat = p.mesh, p.mat
    div = np.zeros(me.n_solid)
    for i in range(me.n_solid):
        for a in range(me.ndim):
            for side in (0, 1):
                n = 1.0 if side == 1 else -1.0
                Sn = mat.S[:, :, a] * n
                out = Sn > 0
                j = me.nbr[i, a, side]
                up = np.where(out, T[:, :, i], 0.0)
                if j >= 0:
                    up = np.where(out, up, T[:, :, j] + me.jump[i, a, side] * me.dT)
                else:
                    up = np.where(out, up, T_w[me.wall_id[i, a, side]])
                div[i] += np.sum(Sn * up) / me.h[a]
    return div


def test_conservation_cfg1_like():
    s = gen.square_block_mask(12, 12, 3, 9)
    w = gen.small_2d(12, 12, solid=s, n_dir=12, n_mfp=4)
    p = Problem(w)
    r = source_iteration(p, tol=1e-13, max_passes=5000)
    T = r["T"]
    T_w = wall_temperature(p, T)
    div = _face_flux_divergence(p, T, T_w)
    scale = np.abs(p.mat.S).sum() / p.mesh.h[0]
    assert np.max(np.abs(div)) < 1e-10 * scale
    # the plane flux is the same through every x-plane
    me = p.mesh
    fl = []
    for k in range(me.n[0]):
        tot = 0.0
        for i in range(me.n_solid):
            if me.coord[i, 0] != k:
                continue
            j = me.nbr[i, 0, 0]
            if j < 0:
                continue
            up = np.where(p.mat.dirs[None, :, 0] > 0, T[:, :, j] + me.jump[i, 0, 0] * me.dT, T[:, :, i])
            tot += np.sum(p.mat.S[:, :, 0] * up)
        fl.append(tot * me.L[0] / (me.dT * me.n_perp))
    assert np.ptp(fl) < 1e-10 * abs(fl[0])
    assert abs(fl[0] - r["kappa_face"]) < 1e-10 * abs(fl[0])
    # energy balance of the last pass against its lagged T_L
    assert r["energy_residual"] < 1e-10


# ---------------------------------------------------------------- Fourier (P7)

def test_fourier_dirichlet_identity_and_symmetry():
    s = gen.circles_mask(24, 24, 1.0, 1.0, [(0.5, 0.5)], [0.3])
    me = Mesh((24, 24, 1), (1.0, 1.0, 1.0), s, (1, 1, 0), 0, 1.0, ndim=2)
    kap = np.array([150.0, 150.0])
    T, kF = fourier_solve(me, kap)
    assert abs(dirichlet_energy_kappa(me, kap, T) - kF) < 1e-10 * kF
    me_y = Mesh((24, 24, 1), (1.0, 1.0, 1.0), s, (1, 1, 0), 1, 1.0, ndim=2)
    _, kFy = fourier_solve(me_y, kap)
    assert abs(kFy - kF) < 1e-10 * kF


@pytest.mark.parametrize("phi", [0.05, 0.1, 0.2])
def test_fourier_eucken_maxwell(phi):
    n = 160
    r = math.sqrt(phi / math.pi)
    s = gen.circles_mask(n, n, 1.0, 1.0, [(0.5, 0.5)], [r])
    me = Mesh((n, n, 1), (1.0, 1.0, 1.0), s, (1, 1, 0), 0, 1.0, ndim=2)
    _, kF = fourier_solve(me, np.array([1.0, 1.0]))
    por = 1 - s.mean()
    em = (1 - por) / (1 + por)
    assert abs(kF - em) < 0.02 * em


# ---------------------------------------------------------------- symmetry (P8)

def test_mirror_symmetry_and_isotropy():
    s = gen.square_block_mask(10, 10, 3, 7)
    w = gen.small_2d(10, 10, solid=s, n_dir=8, n_mfp=3)
    p = Problem(w)
    r = source_iteration(p, tol=1e-13, max_passes=5000)
    me = p.mesh
    J = np.zeros((10, 10, 2))
    J[me.coord[:, 1], me.coord[:, 0]] = r["J"]
    Jm = J[::-1]                                   # y-mirror
    assert np.allclose(J[..., 0], Jm[..., 0], atol=1e-10 * np.abs(J).max())
    assert np.allclose(J[..., 1], -Jm[..., 1], atol=1e-10 * np.abs(J).max())
    wy = gen.small_2d(10, 10, solid=s, n_dir=8, n_mfp=3, grad_axis=1)
    ry = source_iteration(Problem(wy), tol=1e-13, max_passes=5000)
    assert abs(ry["kappa_cc"] - r["kappa_cc"]) < 1e-10 * r["kappa_cc"]


# ---------------------------------------------------------------- diffusive limit (P9)

def test_diffusive_limit():
    s = gen.square_block_mask(10, 10, 3, 7)
    errs = []
    for scale in (1e-3, 1e-4):
        L = 100 * NM
        w = gen.small_2d(10, 10, solid=s, n_dir=8, n_mfp=3, mfp_lo=scale * L / 10 / 100,
                         mfp_hi=scale * L / 10)
        p = Problem(w)
        r = source_iteration(p, tol=1e-13, max_passes=20000, n_passes=None)
        TF = r["T_F"] - r["T_F"].mean()
        errs.append(np.max(np.abs(r["T_L"] - TF)))
    assert errs[0] < 1e-2
    assert errs[1] < errs[0] / 5          # error shrinks with Lambda / h


# ---------------------------------------------------------------- adjoint (P10)

def test_adjoint_bulk_closed_form():
    w = gen.small_2d(5, 4, n_dir=8, n_mfp=3, sigma=np.full(20, 1.3))
    p = Problem(w)
    r = source_iteration(p, tol=1e-14)
    a = adjoint_source_iteration(p, r["T"], tol=1e-14)
    pred = -150.0 / (1.3 ** 2 * 20)
    assert np.allclose(a["grad"], pred, rtol=1e-9)
    assert abs(a["kappa_adj"] - r["kappa_cc"]) < 1e-10 * r["kappa_cc"]


def test_adjoint_dense_and_fd():
    s = np.ones((1, 4, 4), np.uint8)
    s[0, 1:3, 1:3] = 0
    rng = np.random.default_rng(3)
    sig = rng.uniform(0.5, 2.0, 16)
    w = gen.small_2d(4, 4, solid=s, n_dir=8, n_mfp=2, sigma=sig)
    p = Problem(w)
    Td, _, _, _ = dense_solve(p)
    ad = adjoint_dense(p, Td)
    ai = adjoint_source_iteration(p, Td, tol=1e-15, max_passes=50000)
    assert np.allclose(ai["grad"], ad["grad"], rtol=1e-9, atol=1e-12 * np.abs(ad["grad"]).max())
    # central finite differences of the dense forward kappa (step 1e-4:
    # truncation ~h^2, roundoff ~eps*cond/h)
    h = 1e-4
    for c in [0, 3, 5, 15]:
        if not s.ravel()[c]:
            continue
        k = []
        for d in (h, -h):
            sp_ = sig.copy()
            sp_[c] += d
            pp = Problem(gen.small_2d(4, 4, solid=s, n_dir=8, n_mfp=2, sigma=sp_))
            k.append(kappa_cc(pp, dense_solve(pp)[0]))
        fd = (k[0] - k[1]) / (2 * h)
        i = p.mesh.sid[c]
        assert abs(fd - ad["grad"][i]) < 1e-6 * max(abs(fd), 1e-3)


def test_adjoint_scaling_identity():
    s = np.ones((1, 4, 4), np.uint8)
    s[0, 1:3, 1:2] = 0
    sig = np.random.default_rng(5).uniform(0.6, 1.8, 16)
    base = dict(solid=s, n_dir=8, n_mfp=2, sigma=sig)
    p = Problem(gen.small_2d(4, 4, **base))
    Td = dense_solve(p)[0]
    g = adjoint_dense(p, Td)["grad"]
    k0 = kappa_cc(p, Td)
    L = 100 * NM
    eps = 1e-5
    kp = kappa_cc(*(lambda q: (q, dense_solve(q)[0]))(Problem(gen.small_2d(4, 4, L=L * (1 + eps), **base))))
    km = kappa_cc(*(lambda q: (q, dense_solve(q)[0]))(Problem(gen.small_2d(4, 4, L=L * (1 - eps), **base))))
    LdkdL = (kp - km) / (2 * eps)
    lhs = float(np.sum(p.sigma * g))
    assert abs(lhs - (LdkdL - k0)) < 1e-6 * abs(k0)


# ------------------------------------------------- mode tables (interpolation)

from oracle.modes import interp_weights, kappa_modes  # noqa: E402


def test_modes_on_node_identity():
    """Modes sitting on the grid nodes with the kernel's weights: every c is a
    single 1, the grid weights equal the kernel path's, and kappa_mu is the
    per-system kappa."""
    w0 = gen.small_2d(8, 6, solid=gen.square_block_mask(8, 6, 2, 5), n_dir=8, n_mfp=3)
    wn = on_node_modes(w0)
    F, _ = wn.modes
    W = interp_weights(w0.mfp, w0.dirs, F)
    for mu, terms in enumerate(W):
        assert len(terms) == 1 or max(c for _, _, c in terms) > 1 - 1e-12
        m, l, c = max(terms, key=lambda t: t[2])
        assert (m, l) == divmod(mu, len(w0.dir_w)) and abs(c - 1.0) < 1e-12
    p0, pn = Problem(w0), Problem(wn)
    assert np.allclose(pn.mat.D, p0.mat.D, rtol=1e-12, atol=0)
    assert np.allclose(pn.mat.S, p0.mat.S, rtol=1e-12, atol=1e-12 * np.abs(p0.mat.S).max())
    r = source_iteration(pn, tol=1e-13)
    km = kappa_modes(pn, r["T"])
    # the per-system kappa measured from the mean lattice temperature
    g = w0.grad_axis
    tot_L = float(np.sum(pn.mat.D * r["T"].sum(axis=2)))
    shift = pn.mesh.L[g] / (pn.mesh.dT * pn.mesh.n_cells) * pn.mat.S[:, :, g] * tot_L
    assert np.allclose(km, (r["kappa_ml"] - shift).ravel(), rtol=1e-10, atol=1e-12 * r["kappa_cc"])


@pytest.mark.parametrize("nd", [2, 3])
def test_modes_weights_properties(nd):
    """c >= 0 and sum c = 1 per mode; in range, the weights reproduce |F|
    (linear in Lambda) and the angle (linear in angle) exactly."""
    if nd == 2:
        w = gen.with_modes(gen.small_2d(4, 4, n_dir=12, n_mfp=5), 200, 3)
    else:
        w = gen.with_modes(gen.small_3d(3, 3, 2, n_theta=6, n_phi=8, n_mfp=4), 200, 4)
    F, _ = w.modes
    W = interp_weights(w.mfp, w.dirs, F)
    lam = np.linalg.norm(F, axis=1)
    for mu, terms in enumerate(W):
        cs = np.array([c for _, _, c in terms])
        assert np.all(cs >= -1e-15) and abs(cs.sum() - 1.0) < 1e-12
        if w.mfp.min() < lam[mu] < w.mfp.max():
            assert abs(sum(c * w.mfp[m] for m, _, c in terms) - lam[mu]) < 1e-12 * lam[mu]
        # angle: weighted mean of the bracketing directions' angles (unwrapped
        # around the mode's own angle) equals the mode's angle
        if nd == 2:
            phi = math.atan2(F[mu, 1], F[mu, 0])
            a = [c * ((math.atan2(w.dirs[l, 1], w.dirs[l, 0]) - phi + math.pi) % (2 * math.pi) - math.pi)
                 for _, l, c in terms]
            assert abs(sum(a)) < 1e-12
        else:
            th = math.acos(F[mu, 2] / lam[mu])
            ths = np.unique(np.round(np.arccos(w.dirs[:, 2]), 12))
            if ths.min() < th < ths.max():
                t = sum(c * math.acos(max(-1.0, min(1.0, w.dirs[l, 2]))) for _, l, c in terms)
                assert abs(t - th) < 1e-12


def test_modes_bulk_closed_form_and_sum_rule():
    """No pores: kappa_cc = sum_ml S_ml,x Lambda_m s_x,l with the interpolated
    S (the bulk closed form with any T_L weights); with pores the
    mode-resolved kappa sums to kappa_cc (S_ml = sum_mu c S_mu)."""
    wb = gen.with_modes(gen.small_2d(8, 6, n_dir=8, n_mfp=3), 40, 1)
    p = Problem(wb)
    r = source_iteration(p, tol=1e-13)
    cf = float(np.sum(p.mat.S[:, :, 0] * wb.mfp[:, None] * wb.dirs[None, :, 0]))
    assert abs(r["kappa_cc"] - cf) < 1e-11 * cf
    # bulk, per mode: every T_ml - T_L is Lambda_m s_l,x dT / L in every cell
    # (the upwind difference of a linear profile is exact), so kappa_mu =
    # alpha_mu F_mu,x sum_ml c Lambda_m s_l,x
    F, alpha = wb.modes
    kmb = kappa_modes(p, r["T"])
    proj = np.array([sum(c * wb.mfp[m] * wb.dirs[l, 0] for m, l, c in t)
                     for t in interp_weights(wb.mfp, wb.dirs, F)])
    assert np.max(np.abs(kmb - alpha * F[:, 0] * proj)) < 1e-11 * cf
    wp = gen.with_modes(gen.small_2d(10, 8, solid=gen.square_block_mask(10, 8, 3, 6), n_dir=8, n_mfp=3),
                        60, 5)
    p = Problem(wp)
    r = source_iteration(p, tol=1e-13)
    km = kappa_modes(p, r["T"])
    assert abs(km.sum() - r["kappa_cc"]) < 1e-12 * abs(r["kappa_cc"])
    # gauge: the temperatures are fixed up to a common constant, which no
    # kappa_mu may see
    km2 = kappa_modes(p, r["T"] + 0.37)
    assert np.max(np.abs(km2 - km)) < 1e-12 * abs(r["kappa_cc"])



def test_modes_projection_and_static_modes():
    """3D modes in a 2D domain act through their in-plane part, and modes
    with zero in-plane MFP (T_mu = T_L exactly) drop out: appending them,
    with any weight, leaves the solution unchanged."""
    from oracle.modes import grid_weights
    w0 = gen.small_2d(10, 8, solid=gen.square_block_mask(10, 8, 3, 6), n_dir=8, n_mfp=3)
    w3 = gen.with_modes(w0, 40, 13, dim3=True)
    ws = gen.with_modes(w0, 40, 13, dim3=True, n_static=7)
    F3, a3 = w3.modes
    Fs, as_ = ws.modes
    assert Fs.shape[1] == 3 and np.all(Fs[40:, :2] == 0.0)
    assert np.array_equal(Fs[:40], F3)
    # the in-plane part explicitly (2 columns) gives the same grid weights
    D2, S2, k2 = grid_weights(w0.mfp, w0.dirs, F3[:, :2], a3)
    D3, S3, k3 = grid_weights(w0.mfp, w0.dirs, F3, a3)
    assert np.array_equal(D2, D3) and np.array_equal(S2, S3) and np.array_equal(k2, k3)
    # static modes: same D after renormalisation over the moving ones
    Dst, Sst, kst = grid_weights(w0.mfp, w0.dirs, Fs, as_ * 1.0)
    scale = as_[:40].sum() / a3.sum()
    assert np.allclose(Sst, S3 * scale, rtol=1e-14, atol=0)
    assert np.allclose(Dst, D3, rtol=1e-14, atol=0)
    p3, ps = Problem(w3), Problem(ws)
    r3 = source_iteration(p3, tol=1e-13)
    rs = source_iteration(ps, tol=1e-13)
    assert abs(rs["kappa_cc"] - scale * r3["kappa_cc"]) < 1e-11 * abs(r3["kappa_cc"])
    assert np.allclose(rs["T_L"], r3["T_L"], rtol=0, atol=1e-11)
    km = kappa_modes(ps, rs["T"])
    assert np.all(km[40:] == 0.0)
    assert abs(km.sum() - rs["kappa_cc"]) < 1e-12 * abs(rs["kappa_cc"])


def test_exact_modes_on_nodes_equal_kernel_path():
    """Eq. iter3 (one system per mode) with the modes on the grid nodes and
    the kernel's weights is the grid problem itself, systems renumbered."""
    import dataclasses
    w0 = gen.small_2d(10, 8, solid=gen.square_block_mask(10, 8, 3, 6), n_dir=8, n_mfp=3)
    we = dataclasses.replace(on_node_modes(w0), modes_exact=True)
    p0, pe = Problem(w0), Problem(we)
    assert pe.mat.n_mfp == 1 and pe.mat.n_dir == 24
    r0 = source_iteration(p0, tol=1e-13)
    re = source_iteration(pe, tol=1e-13)
    assert abs(re["kappa_cc"] - r0["kappa_cc"]) < 1e-11 * r0["kappa_cc"]
    assert abs(re["kappa_face"] - r0["kappa_face"]) < 1e-11 * r0["kappa_face"]
    assert np.allclose(re["T_L"], r0["T_L"], rtol=0, atol=1e-11)
    # kappa_mu with c = I is the per-system share (from the mean T_L)
    km = kappa_modes(pe, re["T"])
    g = 0
    tot_L = float(np.sum(p0.mat.D * r0["T"].sum(axis=2)))
    shift = p0.mesh.L[g] / (p0.mesh.dT * p0.mesh.n_cells) * p0.mat.S[:, :, g] * tot_L
    assert np.allclose(km, (r0["kappa_ml"] - shift).ravel(), rtol=1e-9, atol=1e-11 * r0["kappa_cc"])


def test_exact_modes_bulk_closed_form():
    """No pores: every mode's T - T_L is F_mu,x dT / L, so kappa = sum_mu
    alpha_mu F_mu,x^2 and kappa_mu = alpha_mu F_mu,x^2 (static modes: 0)."""
    import dataclasses
    w = dataclasses.replace(gen.with_modes(gen.small_2d(8, 6, n_dir=8, n_mfp=3), 30, 3, dim3=True,
                                           n_static=3), modes_exact=True)
    p = Problem(w)
    r = source_iteration(p, tol=1e-13)
    F, alpha = w.modes
    assert abs(r["kappa_cc"] - np.sum(alpha * F[:, 0] ** 2)) < 1e-11 * r["kappa_cc"]
    km = kappa_modes(p, r["T"])
    assert np.allclose(km, alpha * F[:, 0] ** 2, rtol=1e-10, atol=1e-12 * r["kappa_cc"])
