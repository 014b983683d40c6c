"""GPU adjoint, batched multi-geometry launch and checkpoint/resume, each
against the CPU oracle (or an unbatched / uninterrupted GPU run)."""
import os
import tempfile

import numpy as np
import pytest
import torch

from inputs import gen
from oracle.adjoint import adjoint_source_iteration
from oracle.bte import Problem, source_iteration
from tests.gpu_common import gpu_solve, oracle_full, rel, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def _adj_case():
    rng = np.random.default_rng(21)
    s = gen.square_block_mask(10, 9, 3, 6)
    return gen.small_2d(10, 9, solid=s, n_dir=8, n_mfp=3, sigma=rng.uniform(0.5, 2.0, 90))


@pytest.mark.parametrize("accel", [0, 5])
@pytest.mark.parametrize("prec", [0, 1])
def test_adjoint_vs_oracle(P, prec, accel):
    w = _adj_case()
    prob = Problem(w)
    fwd = source_iteration(prob, tol=1e-14, max_passes=20000)
    ref = adjoint_source_iteration(prob, fwd["T"], tol=1e-14, max_passes=20000)
    gref = oracle_full(prob, ref["grad"])
    s = P.Solver.from_workload(w)
    o = s.opts(precision=prec, outer_tol=1e-13 if prec == 0 else 1e-9,
               inner_tol=1e-14 if prec == 0 else 1e-7, fourier_tol=1e-14, keep_state=1,
               max_outer=20000, accel=accel)
    s.solve(o, sigma=w.sigma, want_T_L=False)
    g, st = s.adjoint(o)
    g = g.cpu().numpy()
    assert abs(st["kappa"] - fwd["kappa_cc"]) < (1e-10 if prec == 0 else 1e-4) * fwd["kappa_cc"]
    if prec == 0:
        assert np.linalg.norm(g - gref) <= 1e-10 * np.linalg.norm(gref)
    else:
        assert np.max(np.abs(g - gref)) <= 1e-3 * np.max(np.abs(gref))
        assert abs(g.sum() - gref.sum()) <= 1e-4 * abs(gref.sum())


def test_adjoint_bulk_closed_form(P):
    w = gen.small_2d(8, 6, n_dir=8, n_mfp=3, sigma=np.full(48, 1.3))
    s = P.Solver.from_workload(w)
    o = s.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-14, keep_state=1)
    s.solve(o, sigma=w.sigma, want_T_L=False)
    g, _ = s.adjoint(o)
    assert np.allclose(g.cpu().numpy(), -150.0 / (1.3 ** 2 * 48), rtol=1e-10)


def test_adjoint_autograd_function(P):
    w = _adj_case()
    s = P.Solver.from_workload(w)
    o = s.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-14)
    sig = torch.as_tensor(w.sigma, device="cuda").requires_grad_(True)
    k = P.KappaEff.apply(sig, s, o)
    k.backward()
    prob = Problem(w)
    fwd = source_iteration(prob, tol=1e-14, max_passes=20000)
    ref = adjoint_source_iteration(prob, fwd["T"], tol=1e-14, max_passes=20000)
    assert abs(k.item() - fwd["kappa_cc"]) < 1e-10 * fwd["kappa_cc"]
    assert np.linalg.norm(sig.grad.cpu().numpy() - oracle_full(prob, ref["grad"])) <= \
        1e-10 * np.linalg.norm(ref["grad"])


def test_autograd_two_forwards_then_first_backward(P):
    """Two graphs on one solver: the backward of the first (run after the
    second forward, and after its sigma tensor was changed in place) gives
    the gradient at the first sigma, not at the later one."""
    w = _adj_case()
    s = P.Solver.from_workload(w)
    o = s.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-14)
    sig1 = torch.as_tensor(w.sigma, device="cuda").requires_grad_(True)
    sig2 = torch.as_tensor(np.asarray(w.sigma)[::-1].copy(), device="cuda").requires_grad_(True)
    k1 = P.KappaEff.apply(sig1, s, o)
    k2 = P.KappaEff.apply(sig2, s, o)
    with torch.no_grad():
        sig1.mul_(1.5)                          # in place, after the forward
    k1.backward()
    k2.backward()
    # reference gradients from fresh solvers
    refs = []
    for sg in (w.sigma, np.asarray(w.sigma)[::-1].copy()):
        r = P.Solver.from_workload(w)
        ok = r.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-14, keep_state=1)
        r.solve(ok, sigma=sg, want_T_L=False)
        refs.append(r.adjoint(ok)[0].cpu().numpy())
    g1, g2 = sig1.grad.cpu().numpy(), sig2.grad.cpu().numpy()
    assert np.linalg.norm(g1 - refs[0]) <= 1e-12 * np.linalg.norm(refs[0])
    assert np.linalg.norm(g2 - refs[1]) <= 1e-12 * np.linalg.norm(refs[1])
    assert np.linalg.norm(refs[0] - refs[1]) > 1e-3 * np.linalg.norm(refs[0])


def test_adjoint_requires_state(P):
    w = _adj_case()
    s = P.Solver.from_workload(w)
    o = s.opts()
    s.solve(o, sigma=w.sigma, want_T_L=False)         # keep_state = 0
    with pytest.raises(P.ObteError) as e:
        s.adjoint(o)
    assert e.value.status == P.obte.OBTE_ERR_STATE


def test_batch_matches_single(P):
    ws = [gen.config1(), gen.small_2d(40, 40, solid=gen.circles_mask(40, 40, 1e-7, 1e-7, [(5e-8, 5e-8)], [2e-8]),
                                      n_dir=24, n_mfp=10, mfp_hi=10e-6),
          gen.small_2d(20, 20, solid=gen.square_block_mask(20, 20, 4, 9), n_dir=24, n_mfp=10, mfp_hi=10e-6)]
    solvers = [P.Solver.from_workload(w) for w in ws]
    o = P.default_opts(outer_tol=1e-10, inner_tol=1e-13, fourier_tol=1e-13)
    kb, stb = P.solve_batch(solvers, o)
    for w, k in zip(ws, kb):
        single = gpu_solve(P, w, want_J=False, outer_tol=1e-10, inner_tol=1e-13, fourier_tol=1e-13)
        assert abs(k - single["kappa"]) <= 1e-12 * abs(single["kappa"])
    ref = source_iteration(Problem(ws[2]), tol=1e-10)
    assert abs(kb[2] - ref["kappa_cc"]) <= 1e-9 * ref["kappa_cc"]


def test_checkpoint_resume_bitwise(P):
    w = gen.config1()
    full = gpu_solve(P, w, want_J=False, outer_tol=0.0, max_outer=12, passes_per_graph=1)
    s = P.Solver.from_workload(w)
    o = s.opts(outer_tol=0.0, max_outer=12, passes_per_graph=1)
    o5 = s.opts(outer_tol=0.0, max_outer=12, passes_per_graph=1)
    # run 5 passes by capping the pass count through a first call, then save
    o5.max_outer = 5
    s.solve(o5, want_T_L=False)
    path = os.path.join(tempfile.mkdtemp(), "ck.bin")
    s.checkpoint_save(path)
    # a fresh handle and workspace continue from the file
    s2 = P.Solver.from_workload(w)
    s2.ensure_workspace(o)
    s2.checkpoint_load(path)
    o.init = 1
    o.max_outer = 12
    out = s2.solve(o, want_T_L=True)
    assert out["outer_iters"] == 12
    assert out["kappa"] == full["kappa"]
    assert np.array_equal(out["T_L"].cpu().numpy(), full["T_L"])
