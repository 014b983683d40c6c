"""Full-size workloads on the GPU against the oracle's stored values
(tests/golden/*_oracle.json, written by tests/golden/make_golden.py from the
oracle only) and against properties that hold at any size."""
import json
import os

import numpy as np
import pytest
import torch

from inputs import gen
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def golden(name):
    return json.load(open(os.path.join(GOLD, f"{name}_oracle.json")))


def fields(name):
    """The oracle's full T_L and J fields (every cell, pores 0)."""
    with np.load(os.path.join(GOLD, f"{name}_fields.npz"), allow_pickle=False) as f:
        return f["T_L"], f["J"]


def solve(P, w, want_J=False, **opt):
    s = P.Solver.from_workload(w)
    out = s.solve(s.opts(**opt), sigma=w.sigma, want_T_L=True, want_J=want_J)
    out["T_L"] = out["T_L"].cpu().numpy()
    if want_J:
        out["J"] = out["J"].cpu().numpy()
    out["solver"] = s
    return out


def maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# both sides converged to a 1e-13 relative change (the GPU also to a 1e-13
# estimated iterate error): with contractions up to ~0.9 the fixed-point
# error of each is ~1e-12, far inside the 1e-10 bar
CONVERGED = dict(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-13, max_outer=5000, max_inner=64)


@pytest.mark.parametrize("name", ["cfg2", "cfg4"])
@pytest.mark.parametrize("accel", [0, 8])
def test_fp64_converged_vs_oracle(P, name, accel):
    """Every cell of T_L and J, kappa, kappa_face, kappa_F and the per-MFP
    kappa against the oracle's fields, to 1e-10 (Eq. (iter2), Eq. (keff))."""
    w = gen.config2() if name == "cfg2" else gen.config4()
    g = golden(name)
    T_ref, J_ref = fields(name)
    out = solve(P, w, want_J=True, accel=accel, **CONVERGED)
    assert out["status"] == 0
    assert abs(out["kappa"] - g["kappa_cc"]) <= 1e-10 * g["kappa_cc"]
    assert abs(out["kappa_face"] - g["kappa_face"]) <= 1e-10 * g["kappa_face"]
    assert abs(out["kappa_fourier"] - g["kappa_fourier"]) <= 1e-10 * g["kappa_fourier"]
    k, per = out["solver"].kappa()
    assert np.max(np.abs(per - np.asarray(g["kappa_per_mfp"]))) <= 1e-10 * g["kappa_cc"]
    assert maxrel(out["T_L"], T_ref) <= 1e-10
    assert maxrel(out["J"].reshape(J_ref.shape), J_ref) <= 1e-10
    if accel:
        assert out["outer_iters"] < g["passes"] // 2


@pytest.mark.parametrize("name", ["cfg2", "cfg4"])
@pytest.mark.parametrize("lag,rtol", [(0, 0.0), (1, 0.3), (1, 0.1), (0, 0.1)])
def test_fp32_form_vs_oracle(P, name, lag, rtol):
    """The FP32-sweep form at the bench's operating points reaches 1e-4."""
    w = gen.config2() if name == "cfg2" else gen.config4()
    g = golden(name)
    out = solve(P, w, precision=1, outer_tol=1e-6, inner_tol=1e-5, fourier_tol=1e-8,
                lag_wrap=lag, inner_rtol=rtol, max_outer=3000)
    assert out["status"] == 0
    assert abs(out["kappa"] - g["kappa_cc"]) <= 1e-4 * g["kappa_cc"]


@pytest.mark.parametrize("lag", [0, 1])
def test_fp64_lagged_wrap_same_fixed_point(P, lag):
    w = gen.config2()
    g = golden("cfg2")
    out = solve(P, w, lag_wrap=lag, inner_rtol=0.1, accel=8, **CONVERGED)
    assert out["status"] == 0
    assert abs(out["kappa"] - g["kappa_cc"]) <= 1e-10 * g["kappa_cc"]
    assert maxrel(out["T_L"], fields("cfg2")[0]) <= 1e-10


def test_cfg4_adjoint_vs_finite_differences(P):
    """The adjoint d kappa / d sigma (Eq. (iter2) transposed) against central
    differences of converged forward solves on all 32 seeded cells, at
    h = 1e-6 and h = 1e-4.  Each forward solve stops at a relative change
    and an estimated iterate error of 1e-13, so its kappa carries an error
    e <= ~1e-13 kappa; the difference quotient then errs by up to e / h
    (about 1e-5 absolute at h = 1e-6, 1e-7 at h = 1e-4), plus the O(h^2)
    truncation.  Entries are ~kappa / N_cells ~ 5e-3."""
    w = gen.config4()
    cells = gen.config4_fd_cells()
    assert len(cells) == 32
    s = P.Solver.from_workload(w)
    o = s.opts(accel=8, keep_state=1, passes_per_graph=8, **CONVERGED)
    base = s.solve(o, sigma=w.sigma, want_T_L=False)
    grad, st = s.adjoint(o)
    grad = grad.cpu().numpy()
    assert st["status"] == 0
    assert abs(st["kappa"] - base["kappa"]) <= 1e-10 * base["kappa"]      # p^T lambda = kappa
    o2 = s.opts(accel=8, passes_per_graph=8, **CONVERGED)
    kap = base["kappa"]
    for h, rel_tol in ((1e-6, 1e-3), (1e-4, 1e-5)):
        err = []
        for c in cells:
            k = []
            for d in (h, -h):
                sg = w.sigma.copy()
                sg[c] += d
                r = s.solve(o2, sigma=sg, want_T_L=False)
                assert r["status"] == 0
                k.append(r["kappa"])
            fd = (k[0] - k[1]) / (2 * h)
            # the forward error bound (2e-13 kappa / 2h) and the truncation
            bound = rel_tol * abs(grad[c]) + 2e-13 * kap / (2 * h)
            assert abs(fd - grad[c]) <= bound, (h, c, fd, grad[c])
            err.append(abs(fd - grad[c]) / abs(grad[c]))
        print(f"h={h:g}: max relative FD error over 32 cells {max(err):.2e}")
    # uniform scaling: d kappa(t sigma) / dt at t = 1 equals sigma . grad
    t = 1e-5
    kp = s.solve(o2, sigma=w.sigma * (1 + t), want_T_L=False)["kappa"]
    km = s.solve(o2, sigma=w.sigma * (1 - t), want_T_L=False)["kappa"]
    assert abs((kp - km) / (2 * t) - float(np.dot(w.sigma, grad))) <= 1e-7 * abs(kap)


def test_cfg4_fp32_adjoint_vs_fp64(P):
    """The FP32-sweep form of the adjoint at full size (128x128, 1440
    systems) against the FP64 adjoint: <= 1e-3 per entry (of the largest
    entry) and <= 1e-4 on sigma . grad."""
    w = gen.config4()
    s = P.Solver.from_workload(w)
    o64 = s.opts(accel=8, keep_state=1, **CONVERGED)
    s.solve(o64, sigma=w.sigma, want_T_L=False)
    g64, st64 = s.adjoint(o64)
    s32 = P.Solver.from_workload(w)
    o32 = s32.opts(precision=1, accel=8, keep_state=1, outer_tol=1e-7, inner_tol=1e-6, fourier_tol=1e-10,
                   max_outer=5000)
    s32.solve(o32, sigma=w.sigma, want_T_L=False)
    g32, st32 = s32.adjoint(o32)
    assert st64["status"] == 0 and st32["status"] == 0
    g64, g32 = g64.cpu().numpy(), g32.cpu().numpy()
    assert np.max(np.abs(g32 - g64)) <= 1e-3 * np.max(np.abs(g64))
    a, b = float(np.dot(w.sigma, g32)), float(np.dot(w.sigma, g64))
    assert abs(a - b) <= 1e-4 * abs(b)


@pytest.mark.parametrize("name", ["cfg2", "cfg4"])
@pytest.mark.parametrize("form", ["fp32", "fp64", "fp32_aa", "fp64_aa"])
def test_bench_operating_points_vs_oracle(P, name, form):
    """The operating points bench.py times (error-estimate stop rule at half
    the target) meet the 1e-4 target against the oracle."""
    import bench
    w = gen.config2() if name == "cfg2" else gen.config4()
    g = golden(name)
    out = solve(P, w, **bench.OP[form])
    assert out["status"] == 0
    assert abs(out["kappa"] - g["kappa_cc"]) <= 1e-4 * g["kappa_cc"]


def test_cfg4_adjoint_anderson_vs_plain(P):
    """The mixed adjoint iteration reaches the plain one's gradient."""
    w = gen.config4()
    s = P.Solver.from_workload(w)
    o = s.opts(keep_state=1, accel=6, **CONVERGED)
    s.solve(o, sigma=w.sigma, want_T_L=False)
    ga, sta = s.adjoint(o)
    o0 = s.opts(keep_state=1, **CONVERGED)
    s.solve(o0, sigma=w.sigma, want_T_L=False)
    gp, stp = s.adjoint(o0)
    assert sta["status"] == 0 and stp["status"] == 0
    assert sta["outer_iters"] < stp["outer_iters"]
    ga, gp = ga.cpu().numpy(), gp.cpu().numpy()
    assert np.linalg.norm(ga - gp) <= 1e-10 * np.linalg.norm(gp)
