"""GPU: unstructured 2D meshes (distorted quadrilaterals and triangles)
against the oracle (oracle/umesh.py): the non-orthogonal heat-conduction
first guess (Appendix B, Eq. (final2)), K passes of Algorithm 1 and the
converged kappa; and, on an orthogonal quadrilateral mesh, against the
structured-grid GPU path."""
import numpy as np
import pytest
import torch

from inputs import gen
from oracle.bte import source_iteration
from oracle.material import Material
from oracle.umesh import UMesh, UProblem, fourier_nonorth
from tests.gpu_common import rel, require_gpu

pytestmark = pytest.mark.gpu
NM = 1e-9

CASES = {
    "tri_pore": lambda: gen.unstructured_2d(14, 12, amp=0.3, tri=True, seed=3,
                                            pores=[((45 * NM, 55 * NM), 24 * NM)], n_dir=8, n_mfp=3),
    "quad_pore_gy": lambda: gen.unstructured_2d(13, 11, amp=0.25, tri=False, seed=4, grad_axis=1,
                                                pores=[((30 * NM, 40 * NM), 20 * NM)], n_dir=12, n_mfp=3,
                                                sigma=np.random.default_rng(2).uniform(0.6, 1.6, 143)),
    "tri_bulk": lambda: gen.unstructured_2d(10, 9, amp=0.3, tri=True, seed=5, n_dir=8, n_mfp=2),
    # levels wider than a wavefront and more than 64 periodic faces per
    # direction (several wrap slots per lane)
    "tri_big": lambda: gen.unstructured_2d(48, 40, amp=0.3, tri=True, seed=6, L=200 * NM, Ly=160 * NM,
                                           pores=[((100 * NM, 80 * NM), 45 * NM)], n_dir=8, n_mfp=3),
}


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def full(um, v):
    out = np.zeros(um.n_cells)
    out[um.cells] = v
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_fourier_vs_oracle(P, name):
    w = CASES[name]()
    s = P.UMeshSolver.from_workload(w)
    r = s.fourier(tol=1e-13, cg_tol=1e-14)
    um = UMesh(w.L, w.nodes, w.cells, w.shifts, w.solid, w.grad_axis, w.dT)
    mat = Material(w.mfp, w.dirs, w.dir_w, w.kappa_m, w.grad_axis)
    T, kF, it = fourier_nonorth(um, mat.kappa_axis, tol=1e-13)
    assert r["status"] == 0
    assert abs(r["kappa_fourier"] - kF) <= 1e-10 * abs(kF)
    assert rel(r["T"].cpu().numpy(), full(um, T)) <= 1e-10
    assert abs(r["outer_iters"] - it) <= 2


@pytest.mark.parametrize("name", list(CASES))
def test_lockstep_passes_vs_oracle(P, name):
    """K passes of Algorithm 1, every system solved exactly (the periodic
    coupling to 1e-14): kappa_cc, kappa_face and every cell of T_L."""
    w = CASES[name]()
    K = 4
    s = P.UMeshSolver.from_workload(w)
    o = s.opts(outer_tol=0.0, max_outer=K, inner_tol=1e-14, max_inner=200, fourier_tol=1e-13)
    r = s.solve(o, sigma=w.sigma)
    assert r["outer_iters"] == K
    prob = UProblem(w)
    ref = source_iteration(prob, n_passes=K)
    assert abs(r["kappa"] - ref["kappa_cc"]) <= 1e-10 * abs(ref["kappa_cc"])
    assert abs(r["kappa_face"] - ref["kappa_face"]) <= 1e-10 * abs(ref["kappa_face"])
    assert abs(r["kappa_fourier"] - ref["kappa_fourier"]) <= 1e-10 * abs(ref["kappa_fourier"])
    assert rel(r["T_L"].cpu().numpy(), full(prob.mesh, ref["T_L"])) <= 1e-10
    assert all(n >= 1 for n in s.levels())
    if name == "tri_big":
        assert s.n_solid > 64 * 20


def test_converged_vs_oracle(P):
    w = CASES["tri_pore"]()
    s = P.UMeshSolver.from_workload(w)
    r = s.solve(s.opts(outer_tol=1e-12, max_outer=3000, inner_tol=1e-14, max_inner=200, fourier_tol=1e-13))
    assert r["status"] == 0
    ref = source_iteration(UProblem(w), tol=1e-12, max_passes=3000)
    assert abs(r["outer_iters"] - ref["passes"]) <= 1
    # both stop at a 1e-12 relative change (contraction < 0.95 here)
    assert abs(r["kappa"] - ref["kappa_cc"]) <= 1e-10 * abs(ref["kappa_cc"])
    assert rel(r["T_L"].cpu().numpy(), full(UMesh(w.L, w.nodes, w.cells, w.shifts, w.solid), ref["T_L"])) <= 1e-9


def test_bulk_closed_form(P):
    w = CASES["tri_bulk"]()
    s = P.UMeshSolver.from_workload(w)
    r = s.solve(s.opts(outer_tol=1e-13, max_outer=200, inner_tol=1e-14, max_inner=200, fourier_tol=1e-13))
    kb = Material(w.mfp, w.dirs, w.dir_w, w.kappa_m, 0).kappa_axis[0]
    assert abs(r["kappa"] - kb) <= 1e-10 * kb
    assert abs(r["kappa_fourier"] - kb) <= 1e-10 * kb


def test_orthogonal_quads_match_structured_gpu_path(P):
    """Unperturbed quadrilaterals are the structured grid: both GPU paths
    reach the same kappa."""
    nx, ny = 16, 12
    w = gen.unstructured_2d(nx, ny, amp=0.0, tri=False, pores=[((50 * NM, 50 * NM), 26 * NM)], n_dir=8, n_mfp=3)
    ws = gen.small_2d(nx, ny, solid=w.solid.reshape(1, ny, nx), n_dir=8, n_mfp=3, L=w.L[0], Ly=w.L[1])
    s = P.UMeshSolver.from_workload(w)
    o = dict(outer_tol=1e-12, max_outer=3000, inner_tol=1e-14, max_inner=200, fourier_tol=1e-13)
    r = s.solve(s.opts(**o))
    ss = P.Solver.from_workload(ws)
    rs = ss.solve(ss.opts(**o), want_T_L=True)
    assert r["status"] == 0 and rs["status"] == 0
    assert abs(r["kappa"] - rs["kappa"]) <= 1e-10 * abs(rs["kappa"])
    assert abs(r["kappa_face"] - rs["kappa_face"]) <= 1e-10 * abs(rs["kappa_face"])
    assert rel(r["T_L"].cpu().numpy(), rs["T_L"].cpu().numpy()) <= 1e-9


def test_umesh_rejections(P):
    w = CASES["tri_bulk"]()
    s = P.UMeshSolver.from_workload(w)
    for kw in (dict(precision=1), dict(accel=4), dict(init=1)):
        with pytest.raises(P.ObteError) as e:
            s.solve(s.opts(**kw))
        assert e.value.status == P.obte.OBTE_ERR_ARG
    r = s.solve(s.opts(outer_tol=0.0, max_outer=2))
    assert r["status"] == P.obte.OBTE_ERR_NOT_CONVERGED and r["outer_iters"] == 2


def test_forcing_term_same_fixed_point(P):
    """A forcing term on the periodic-face solves (part of the coupling left
    to later passes) converges to the same kappa and T_L, in fewer inner
    iterations."""
    w = CASES["tri_pore"]()
    s = P.UMeshSolver.from_workload(w)
    base = dict(outer_tol=1e-12, max_outer=5000, inner_tol=1e-14, max_inner=200, fourier_tol=1e-13)
    r0 = s.solve(s.opts(**base))
    r1 = s.solve(s.opts(inner_rtol=0.3, **base))
    assert r0["status"] == 0 and r1["status"] == 0
    assert r1["inner_iters"] < r0["inner_iters"]
    assert abs(r1["kappa"] - r0["kappa"]) <= 1e-10 * abs(r0["kappa"])
    assert rel(r1["T_L"].cpu().numpy(), r0["T_L"].cpu().numpy()) <= 1e-9
    assert r1["wrap_residual"] <= 2e-13
