"""Mode tables (Appendix A interpolation onto the vectorial-MFP grid) and the
mode-resolved conductivity: the HIP path through the C ABI against the FP64
oracle (oracle/modes.py) on the same seeded inputs."""
import functools

import numpy as np
import pytest

from inputs import gen
from oracle.bte import Problem, source_iteration
from oracle.modes import kappa_modes
from tests._lib import on_node_modes
from tests.gpu_common import gpu_solve, oracle_full, rel, require_gpu
from tests.test_gpu_parity import ragged_porous, small3d

pytestmark = pytest.mark.gpu

TIGHT = dict(outer_tol=1e-12, inner_tol=1e-14, fourier_tol=1e-14, max_inner=200)


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def test_on_node_modes_match_kernel_path(P):
    """One mode per grid node with the kernel's weights: the interpolation is
    the identity, so kappa matches the kappa_m path and kappa_mu is the
    per-system kappa (summed over directions: the per-MFP kappa)."""
    w0 = gen.small_2d(12, 10, solid=gen.square_block_mask(12, 10, 3, 7), n_dir=8, n_mfp=3)
    wn = on_node_modes(w0)
    r0 = gpu_solve(P, w0, **TIGHT)
    rn = gpu_solve(P, wn, **TIGHT)
    assert r0["status"] == 0 and rn["status"] == 0
    assert abs(rn["kappa"] - r0["kappa"]) <= 1e-11 * abs(r0["kappa"])
    assert rel(rn["T_L"], r0["T_L"]) < 1e-10
    s = rn["solver"]
    km = s.kappa_modes()
    assert km.shape == (len(w0.mfp) * len(w0.dir_w),)
    _, per_mfp = r0["solver"].kappa()
    assert np.allclose(km.reshape(len(w0.mfp), len(w0.dir_w)).sum(axis=1), per_mfp,
                       rtol=1e-10, atol=1e-12 * abs(r0["kappa"]))
    prob = Problem(wn)
    ref = source_iteration(prob, tol=1e-13)
    assert np.max(np.abs(km - kappa_modes(prob, ref["T"]))) <= 1e-10 * abs(ref["kappa_cc"])


CASES = {
    # 70 x 37 porous, rows over two wavefronts; 60 random modes, some beyond
    # the MFP grid (clamped to the end nodes)
    "ragged": lambda: gen.with_modes(ragged_porous(), 60, 7),
    # bulk: the closed form holds for any T_L weights
    "bulk": lambda: gen.with_modes(gen.small_2d(16, 12, n_dir=8, n_mfp=4), 40, 2),
    # 3D tensor direction grid: polar x azimuth interpolation
    "3d": lambda: gen.with_modes(small3d(), 48, 9),
    # 3D modes in a 2D domain (in-plane part) plus modes moving only along z
    "proj": lambda: gen.with_modes(gen.small_2d(14, 11, solid=gen.square_block_mask(14, 11, 4, 9), n_dir=12,
                                                n_mfp=4), 50, 17, dim3=True, n_static=6),
}


@functools.lru_cache(maxsize=None)
def oracle_case(name):
    w = CASES[name]()
    prob = Problem(w)
    return w, prob, source_iteration(prob, tol=1e-14, max_passes=40000)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("accel,lag", [(0, 0), (8, 0), (8, 1)])
def test_modes_vs_oracle(P, name, accel, lag):
    """Also with Anderson mixing and the lagged wrap, which need the
    re-centred pass map: the interpolated weights drift the plain iterates
    by a common constant every pass."""
    w, prob, ref = oracle_case(name)
    # both sides converged to a 1e-14 change: with contractions close to 1
    # a 1e-12 stop leaves ~1e-10 of fixed-point error in T_L
    r = gpu_solve(P, w, accel=accel, lag_wrap=lag, **dict(TIGHT, outer_tol=1e-14, max_outer=40000))
    assert r["status"] == 0
    kc = ref["kappa_cc"]
    assert abs(r["kappa"] - kc) <= 1e-10 * abs(kc)
    assert abs(r["kappa_face"] - ref["kappa_face"]) <= 1e-10 * abs(ref["kappa_face"])
    assert rel(r["T_L"], oracle_full(prob, ref["T_L"])) < 1e-10
    km = r["solver"].kappa_modes()
    km_ref = kappa_modes(prob, ref["T"])
    assert km.shape == km_ref.shape
    assert np.max(np.abs(km - km_ref)) <= 1e-10 * abs(kc)
    # sum rule: the modes' shares add up to kappa
    assert abs(km.sum() - r["kappa"]) <= 1e-11 * abs(r["kappa"])
    if name == "bulk":
        cf = float(np.sum(prob.mat.S[:, :, 0] * w.mfp[:, None] * w.dirs[None, :, 0]))
        assert abs(r["kappa"] - cf) <= 1e-11 * cf
    if name == "proj":
        assert np.all(km[-6:] == 0.0)       # the static modes carry nothing


def test_modes_fp32(P):
    w = CASES["ragged"]()
    r64 = gpu_solve(P, w, **TIGHT)
    r32 = gpu_solve(P, w, precision=1, outer_tol=1e-9, inner_tol=1e-6, fourier_tol=1e-12)
    assert r32["status"] == 0
    assert abs(r32["kappa"] - r64["kappa"]) <= 1e-4 * r64["kappa"]
    k32, k64 = r32["solver"].kappa_modes(), r64["solver"].kappa_modes()
    assert np.max(np.abs(k32 - k64)) <= 1e-4 * r64["kappa"]


def test_kappa_modes_state(P):
    """No solve yet (or no table): a state error, not stale values."""
    w = CASES["bulk"]()
    s = P.Solver.from_workload(w)
    with pytest.raises(P.obte.ObteError) as e:
        s.kappa_modes()
    assert e.value.status == P.obte.OBTE_ERR_STATE
    w0 = gen.small_2d(8, 6, n_dir=8, n_mfp=3)
    s0 = P.Solver.from_workload(w0)
    s0.solve(s0.opts(outer_tol=1e-6))
    with pytest.raises(P.obte.ObteError) as e:
        s0.kappa_modes()
    assert e.value.status == P.obte.OBTE_ERR_STATE


def test_modes_in_batch(P):
    """Mode tables inside a batched launch: each geometry's kappa_mu equals
    the single-geometry solve's."""
    ws = [CASES["ragged"](), CASES["bulk"](), gen.small_2d(12, 10, n_dir=8, n_mfp=4)]
    solvers = [P.Solver.from_workload(w) for w in ws]
    o = solvers[0].opts(**TIGHT)
    kb, st = P.solve_batch(solvers, o)
    assert all(x["status"] == 0 for x in st)
    for i in (0, 1):
        r = gpu_solve(P, ws[i], **TIGHT)
        assert abs(kb[i] - r["kappa"]) <= 1e-11 * abs(r["kappa"])
        ks, kr = solvers[i].kappa_modes(), r["solver"].kappa_modes()
        assert np.max(np.abs(ks - kr)) <= 1e-10 * abs(r["kappa"])
        assert abs(ks.sum() - kb[i]) <= 1e-11 * abs(kb[i])
    with pytest.raises(P.obte.ObteError):
        solvers[2].kappa_modes()


@pytest.mark.parametrize("accel", [0, 5])
def test_modes_adjoint_vs_oracle(P, accel):
    """The adjoint with a mode table: a wall's temperature takes every system
    whose S leaves through it, also against the system's direction, so the
    transposed coupling feeds those systems too."""
    from oracle.adjoint import adjoint_source_iteration
    rng = np.random.default_rng(21)
    s = gen.square_block_mask(10, 9, 3, 6)
    w = gen.with_modes(gen.small_2d(10, 9, solid=s, n_dir=8, n_mfp=3, sigma=rng.uniform(0.5, 2.0, 90)),
                       40, 11)
    prob = Problem(w)
    fwd = source_iteration(prob, tol=1e-14, max_passes=20000)
    ref = adjoint_source_iteration(prob, fwd["T"], tol=1e-14, max_passes=20000)
    gref = oracle_full(prob, ref["grad"])
    sv = P.Solver.from_workload(w)
    o = sv.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-14, keep_state=1, max_outer=20000,
                accel=accel)
    sv.solve(o, sigma=w.sigma, want_T_L=False)
    g, st = sv.adjoint(o)
    g = g.cpu().numpy()
    assert abs(st["kappa"] - fwd["kappa_cc"]) < 1e-10 * fwd["kappa_cc"]
    assert np.linalg.norm(g - gref) <= 1e-10 * np.linalg.norm(gref)


# ---------------------------------------------- no interpolation (Eq. iter3)

def _exact(w):
    import dataclasses
    return dataclasses.replace(w, modes_exact=True)


EXACT = {
    "ragged": lambda: _exact(CASES["ragged"]()),
    "proj": lambda: _exact(CASES["proj"]()),
    "3d": lambda: _exact(CASES["3d"]()),
}


@functools.lru_cache(maxsize=None)
def oracle_exact(name):
    w = EXACT[name]()
    prob = Problem(w)
    return w, prob, source_iteration(prob, tol=1e-14, max_passes=40000)


def test_exact_on_nodes_match_kernel_path(P):
    w0 = gen.small_2d(12, 10, solid=gen.square_block_mask(12, 10, 3, 7), n_dir=8, n_mfp=3)
    we = _exact(on_node_modes(w0))
    r0 = gpu_solve(P, w0, **TIGHT)
    re = gpu_solve(P, we, **TIGHT)
    assert re["solver"].n_systems == 24
    assert abs(re["kappa"] - r0["kappa"]) <= 1e-11 * abs(r0["kappa"])
    assert abs(re["kappa_face"] - r0["kappa_face"]) <= 1e-11 * abs(r0["kappa_face"])
    assert rel(re["T_L"], r0["T_L"]) < 1e-10


@pytest.mark.parametrize("name", list(EXACT))
@pytest.mark.parametrize("accel", [0, 8])
def test_exact_modes_vs_oracle(P, name, accel):
    w, prob, ref = oracle_exact(name)
    r = gpu_solve(P, w, accel=accel, **TIGHT)
    assert r["status"] == 0
    kc = ref["kappa_cc"]
    assert abs(r["kappa"] - kc) <= 1e-10 * abs(kc)
    assert abs(r["kappa_face"] - ref["kappa_face"]) <= 1e-10 * abs(ref["kappa_face"])
    assert rel(r["T_L"], oracle_full(prob, ref["T_L"])) < 1e-10
    km = r["solver"].kappa_modes()
    assert np.max(np.abs(km - kappa_modes(prob, ref["T"]))) <= 1e-10 * abs(kc)
    assert abs(km.sum() - r["kappa"]) <= 1e-11 * abs(r["kappa"])


def test_exact_modes_adjoint_vs_oracle(P):
    from oracle.adjoint import adjoint_source_iteration
    rng = np.random.default_rng(23)
    s = gen.square_block_mask(10, 9, 3, 6)
    w = _exact(gen.with_modes(gen.small_2d(10, 9, solid=s, n_dir=8, n_mfp=3, sigma=rng.uniform(0.5, 2.0, 90)),
                              30, 19))
    prob = Problem(w)
    fwd = source_iteration(prob, tol=1e-14, max_passes=20000)
    ref = adjoint_source_iteration(prob, fwd["T"], tol=1e-14, max_passes=20000)
    gref = oracle_full(prob, ref["grad"])
    sv = P.Solver.from_workload(w)
    o = sv.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-14, keep_state=1, max_outer=20000)
    sv.solve(o, sigma=w.sigma, want_T_L=False)
    g, st = sv.adjoint(o)
    g = g.cpu().numpy()
    assert abs(st["kappa"] - fwd["kappa_cc"]) < 1e-10 * fwd["kappa_cc"]
    assert np.linalg.norm(g - gref) <= 1e-10 * np.linalg.norm(gref)
