"""Pins of the unstructured-mesh oracle (oracle/umesh.py) against what the
paper and the mathematics fix, independently of the oracle's own formulas:

  * on an orthogonal quadrilateral mesh it reduces to the structured-grid
    oracle (operators, Fourier first guess, K source-iteration passes);
  * on distorted meshes: the upwind operator's row sums equal its wall
    inflow (a uniform temperature with equal wall values is a solution), and
    V A_l transposed is V A_(-l) (Appendix A's face vectors);
  * least-squares cell gradients are exact for linear fields (Eqs. lq, mm);
  * the heat-conduction solve with the explicit secondary flux (Eqs. grad5
    to final2) is exact for the linear profile of a pore-free distorted cell
    and returns kappa_F = kappa_bulk, while the primary flux alone is not;
  * bulk kappa_cc equals the closed form sum alpha Lambda^2 s_g^2 on every
    pore-free mesh (energy conservation across the periodic cell);
  * the source iteration reaches the dense brute-force solution of the whole
    coupled system, and its energy balance vanishes at the fixed point."""
import numpy as np
import pytest

from inputs import gen
from oracle.bte import Problem, source_iteration, upwind_operator
from oracle.fourier import fourier_solve
from oracle.material import Material
from oracle.mesh import Mesh
from oracle.umesh import (UMesh, UProblem, cell_gradients, dense_solve_u, fourier_nonorth,
                          lsq_gradient_weights, upwind_operator_u)

NM = 1e-9


def umesh_of(w):
    return UMesh(w.L, w.nodes, w.cells, w.shifts, w.solid, w.grad_axis, w.dT)


def structured_twin(w, nx, ny):
    ws = gen.small_2d(nx, ny, solid=w.solid.reshape(1, ny, nx), n_dir=len(w.dirs), n_mfp=len(w.mfp),
                      L=w.L[0], Ly=w.L[1], grad_axis=w.grad_axis, sigma=w.sigma)
    return ws


@pytest.mark.parametrize("grad_axis", [0, 1])
def test_orthogonal_quads_reduce_to_structured(grad_axis):
    nx, ny = 10, 8
    sig = np.random.default_rng(3).uniform(0.6, 1.8, nx * ny)
    w = gen.unstructured_2d(nx, ny, amp=0.0, tri=False, pores=[((48 * NM, 52 * NM), 24 * NM)],
                            n_dir=8, n_mfp=3, grad_axis=grad_axis, sigma=sig)
    ws = structured_twin(w, nx, ny)
    um = umesh_of(w)
    ms = Mesh(ws.n, ws.L, ws.solid, ws.periodic, ws.grad_axis, ws.dT, ndim=2)
    assert um.n_solid == ms.n_solid and um.n_walls == ms.n_walls
    # wall faces pair up by (cell, outward normal)
    key_u = {(int(um.wall_cell[f]), tuple(np.round(um.wn[f]).astype(int))): f for f in range(um.n_walls)}
    perm = [key_u[(int(ms.walls[f, 0]), tuple(ms.wall_normal(f).astype(int)))] for f in range(ms.n_walls)]
    for l in range(len(w.dirs)):
        Au, ju, Bu = upwind_operator_u(um, w.dirs[l])
        As, js, Bs = upwind_operator(ms, w.dirs[l])
        scale = abs(As).max()
        assert abs(Au - As).max() <= 1e-13 * scale
        assert np.max(np.abs(ju - js)) <= 1e-13 * scale
        assert abs(Bu[:, perm] - Bs).max() <= 1e-13 * scale
    mat = Material(w.mfp, w.dirs, w.dir_w, w.kappa_m, grad_axis)
    Tu, ku, it = fourier_nonorth(um, mat.kappa_axis)
    Ts, ks = fourier_solve(ms, mat.kappa_axis)
    assert it <= 2                                   # the secondary flux vanishes
    assert np.max(np.abs(Tu - Ts)) <= 1e-12 * np.max(np.abs(Ts))
    assert abs(ku - ks) <= 1e-12 * ks
    ru = source_iteration(UProblem(w), n_passes=5)
    rs = source_iteration(Problem(ws), n_passes=5)
    for k in ("kappa_cc", "kappa_face", "kappa_fourier"):
        assert abs(ru[k] - rs[k]) <= 1e-12 * abs(rs[k]), k
    assert np.max(np.abs(ru["T_L"] - rs["T_L"])) <= 1e-12 * np.max(np.abs(rs["T_L"]))


@pytest.mark.parametrize("tri", [False, True])
def test_operator_identities_on_distorted_mesh(tri):
    w = gen.unstructured_2d(9, 7, amp=0.3, tri=tri, seed=4, pores=[((40 * NM, 60 * NM), 22 * NM)],
                            n_dir=12, n_mfp=2)
    um = umesh_of(w)
    assert um.n_walls > 0
    V = np.diag(um.V)
    for l in range(len(w.dirs)):
        A, _, Bw = upwind_operator_u(um, w.dirs[l])
        ones = np.ones(um.n_solid)
        assert np.max(np.abs(A @ ones - Bw @ np.ones(um.n_walls))) <= 1e-12 * abs(A).max()
        Am, _, _ = upwind_operator_u(um, -w.dirs[l])
        lhs = (V @ A.toarray()).T
        assert np.max(np.abs(lhs - V @ Am.toarray())) <= 1e-12 * np.max(np.abs(lhs))


@pytest.mark.parametrize("tri", [False, True])
def test_lsq_gradient_exact_for_linear_fields(tri):
    w = gen.unstructured_2d(9, 8, amp=0.3, tri=tri, seed=6, pores=[((50 * NM, 50 * NM), 20 * NM)])
    um = umesh_of(w)
    nb, W = lsq_gradient_weights(um)
    # linear field consistent with the periodic images: T(x + L_g) = T(x) - dT
    G = np.array([-um.dT / um.L[0], 0.37 / um.L[1]])
    G[1] = 0.0 if um.grad_axis == 0 else G[1]
    T = um.xc @ G
    g = cell_gradients(um, T, nb, W)
    full = [i for i in range(um.n_solid) if len(nb[i]) >= 2 and np.linalg.matrix_rank(
        np.array([d for _, d, _ in nb[i]])) == 2]
    assert len(full) > 0.8 * um.n_solid
    assert np.max(np.abs(g[full] - G)) <= 1e-9 * np.max(np.abs(G))


@pytest.mark.parametrize("tri", [False, True])
@pytest.mark.parametrize("grad_axis", [0, 1])
def test_fourier_exact_on_linear_profile(tri, grad_axis):
    w = gen.unstructured_2d(9, 7, amp=0.3, tri=tri, seed=5, grad_axis=grad_axis, L=80 * NM, Ly=60 * NM)
    um = umesh_of(w)
    mat = Material(w.mfp, w.dirs, w.dir_w, w.kappa_m, grad_axis)
    T, kF, it = fourier_nonorth(um, mat.kappa_axis)
    lin = -um.dT / um.L[grad_axis] * um.xc[:, grad_axis]
    lin -= lin.mean()
    assert np.max(np.abs(T - lin)) <= 1e-11 * np.max(np.abs(lin))
    assert abs(kF - mat.kappa_axis[grad_axis]) <= 1e-10 * mat.kappa_axis[grad_axis]
    assert it > 2
    # the two-point flux alone is not exact on this mesh
    Tp, kp, _ = fourier_nonorth(um, mat.kappa_axis, primary_only=True)
    assert np.max(np.abs(Tp - lin)) > 1e-3 * np.max(np.abs(lin))


def test_fourier_with_pores_converges():
    w = gen.unstructured_2d(12, 12, amp=0.25, tri=True, seed=8, pores=[((50 * NM, 50 * NM), 25 * NM)])
    um = umesh_of(w)
    mat = Material(w.mfp, w.dirs, w.dir_w, w.kappa_m, 0)
    T, kF, it = fourier_nonorth(um, mat.kappa_axis, tol=1e-13)
    assert it < 1000
    assert 0.0 < kF < mat.kappa_axis[0]
    # Maxwell-Eucken for the pore fraction the mesh carries
    phi = 1.0 - float(np.sum(um.V)) / um.volume_box
    me = mat.kappa_axis[0] * (1 - phi) / (1 + phi)
    assert abs(kF - me) <= 0.05 * me


@pytest.mark.parametrize("tri", [False, True])
@pytest.mark.parametrize("grad_axis", [0, 1])
def test_bulk_kappa_cc_closed_form(tri, grad_axis):
    w = gen.unstructured_2d(8, 8, amp=0.3, tri=tri, seed=1, n_dir=8, n_mfp=3, grad_axis=grad_axis)
    prob = UProblem(w)
    r = source_iteration(prob, tol=1e-13, max_passes=200)
    assert abs(r["kappa_cc"] - prob.mat.kappa_axis[grad_axis]) <= 1e-11 * prob.mat.kappa_axis[grad_axis]


def test_source_iteration_reaches_dense_solution():
    w = gen.unstructured_2d(5, 4, amp=0.25, tri=True, seed=2, pores=[((50 * NM, 50 * NM), 18 * NM)],
                            n_dir=4, n_mfp=2, sigma=np.random.default_rng(9).uniform(0.7, 1.5, 40))
    prob = UProblem(w)
    T = dense_solve_u(prob)
    r = source_iteration(prob, tol=1e-15, max_passes=6000)
    TL = np.einsum("ml,mli->i", prob.mat.D, T)
    TL -= TL.mean()
    assert np.max(np.abs(TL - r["T_L"])) <= 1e-9 * np.max(np.abs(TL))
    kd = sum(prob.kappa_cc_system(m, l, T[m, l]) for m in range(2) for l in range(4))
    assert abs(kd - r["kappa_cc"]) <= 1e-9 * abs(kd)
    assert r["energy_residual"] < 1e-10
