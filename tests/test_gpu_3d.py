"""The 3D membrane (periodic in x and y, diffuse top and bottom, cylindrical
through-pore): the 16x16x4 replica with the full direction and MFP sets
against the oracle's stored values (tests/golden/cfg5r*_oracle.json), and
the full 64x64x16 case through properties that hold at any size (FP32 form
vs FP64 form, adjoint vs finite differences of the forward solve)."""
import json
import os

import numpy as np
import pytest

from inputs import gen
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def golden(name):
    return json.load(open(os.path.join(GOLD, f"{name}_oracle.json")))


def solve(P, w, **opt):
    s = P.Solver.from_workload(w)
    out = s.solve(s.opts(**opt), sigma=w.sigma, want_T_L=True, want_J=False)
    out["T_L"] = out["T_L"].cpu().numpy()
    out["solver"] = s
    return out


@pytest.mark.parametrize("accel", [0, 8])
def test_replica_fp64_vs_oracle(P, accel):
    """The 16x16x4 replica: kappa, kappa_face, kappa_F, per-MFP kappa and
    every cell of T_L and J against the oracle's fields, to 1e-10; both
    sides converged to a 1e-13 relative change (fixed-point error ~1e-12)."""
    w = gen.config5(nx=16, nz=4)
    g = golden("cfg5r")
    s = P.Solver.from_workload(w)
    out = s.solve(s.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-13, max_outer=8000, max_inner=64,
                         accel=accel), want_T_L=True, want_J=True)
    assert out["status"] == 0
    for key, gk in (("kappa", "kappa_cc"), ("kappa_face", "kappa_face"), ("kappa_fourier", "kappa_fourier")):
        assert abs(out[key] - g[gk]) <= 1e-10 * g[gk], (key, out[key], g[gk])
    k, per = s.kappa()
    assert np.max(np.abs(per - np.asarray(g["kappa_per_mfp"]))) <= 1e-10 * g["kappa_cc"]
    with np.load(os.path.join(GOLD, "cfg5r_fields.npz"), allow_pickle=False) as f:
        T_ref, J_ref = f["T_L"], f["J"]
    T = out["T_L"].cpu().numpy()
    J = out["J"].cpu().numpy().reshape(J_ref.shape)
    assert np.max(np.abs(T - T_ref)) <= 1e-10 * np.max(np.abs(T_ref))
    assert np.max(np.abs(J - J_ref)) <= 1e-10 * np.max(np.abs(J_ref))


@pytest.mark.parametrize("lag,rtol", [(0, 0.0), (1, 0.3)])
def test_replica_fp32_vs_oracle(P, lag, rtol):
    w = gen.config5(nx=16, nz=4)
    g = golden("cfg5r")
    out = solve(P, w, precision=1, outer_tol=5e-5, stop_rule=1, inner_tol=1e-5, lag_wrap=lag,
                inner_rtol=rtol, fourier_tol=1e-8, max_outer=5000)
    assert out["status"] == 0
    assert abs(out["kappa"] - g["kappa_cc"]) <= 1e-4 * g["kappa_cc"]


def test_replica_adjoint_vs_oracle(P):
    gpath = os.path.join(GOLD, "cfg5r_adjoint_oracle.json")
    if not os.path.exists(gpath):
        pytest.skip("cfg5r_adjoint_oracle.json has not been generated")
    g = json.load(open(gpath))
    w = gen.config5(nx=16, nz=4)
    s = P.Solver.from_workload(w)
    o = s.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-13, keep_state=1, max_outer=8000, accel=8,
               max_inner=64)
    s.solve(o, want_T_L=False)
    grad, st = s.adjoint(o)
    grad = grad.cpu().numpy()
    ref = np.asarray(g["grad"])
    assert st["status"] == 0
    assert np.linalg.norm(grad - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.all(grad[w.solid.ravel() == 0] == 0)


@pytest.fixture(scope="module")
def full(P):
    w = gen.config5()
    s = P.Solver.from_workload(w)
    r64 = s.solve(s.opts(outer_tol=1e-10, inner_tol=1e-12, fourier_tol=1e-11, max_outer=5000,
                         passes_per_graph=8), want_T_L=True)
    assert r64["status"] == 0
    r64["T_L"] = r64["T_L"].cpu().numpy()
    return w, s, r64


@pytest.mark.parametrize("lag,rtol", [(0, 0.0), (1, 0.3), (1, 0.1)])
def test_full_fp32_vs_fp64(P, full, lag, rtol):
    """The FP32-sweep form at the bench's operating points reaches 1e-4."""
    w, s, r64 = full
    r32 = s.solve(s.opts(precision=1, outer_tol=5e-5, stop_rule=1, inner_tol=1e-5, lag_wrap=lag,
                         inner_rtol=rtol, fourier_tol=1e-8, max_outer=5000), want_T_L=True)
    assert r32["status"] == 0
    assert abs(r32["kappa"] - r64["kappa"]) <= 1e-4 * r64["kappa"]
    T32 = r32["T_L"].cpu().numpy()
    assert np.max(np.abs(T32 - r64["T_L"])) <= 1e-3 * np.max(np.abs(r64["T_L"]))


def test_full_fp64_properties(P, full):
    """kappa_face exceeds kappa_cc by the upwind numerical diffusion only
    (O(h / Lambda), a few percent here) and T_L is odd under the x-mirror of
    this mirror-symmetric geometry (up to the additive gauge)."""
    w, s, r64 = full
    assert r64["kappa_face"] > r64["kappa"]
    assert (r64["kappa_face"] - r64["kappa"]) / r64["kappa"] < 0.15
    n = w.n
    T = r64["T_L"].reshape(n[2], n[1], n[0])
    sol = w.solid.reshape(n[2], n[1], n[0]).astype(bool)
    # cell ix <-> n-1-ix mirror about the pore centre; the periodic image
    # convention makes T + mirror(T) constant over the solid
    Tm = T[:, :, ::-1]
    ssum = (T + Tm)[sol]
    assert np.ptp(ssum) <= 1e-6 * np.abs(T[sol]).max()


def test_full_adjoint_scaling_identity(P, full):
    """sum_i sigma_i d kappa / d sigma_i at sigma = 1 against the derivative
    of kappa(t sigma) at t = 1 from two converged forward solves."""
    w, s, _ = full
    o = s.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-13, keep_state=1, max_outer=5000,
               passes_per_graph=8)
    base = s.solve(o, want_T_L=False)
    assert base["status"] == 0
    grad, st = s.adjoint(s.opts(outer_tol=1e-13, inner_tol=1e-14, keep_state=1, max_outer=5000))
    assert st["status"] == 0
    assert abs(st["kappa"] - base["kappa"]) <= 1e-9 * base["kappa"]
    grad = grad.cpu().numpy()
    sig = np.ones(w.n_cells)
    t = 1e-4
    o2 = s.opts(outer_tol=1e-13, inner_tol=1e-14, fourier_tol=1e-13, max_outer=5000, passes_per_graph=8)
    kp = s.solve(o2, sigma=sig * (1 + t), want_T_L=False)["kappa"]
    km = s.solve(o2, sigma=sig * (1 - t), want_T_L=False)["kappa"]
    fd = (kp - km) / (2 * t)
    assert abs(fd - float(np.dot(sig, grad))) <= 1e-6 * abs(base["kappa"]), (fd, float(np.dot(sig, grad)))


@pytest.mark.parametrize("form", ["fp32", "fp64", "fp32_aa", "fp64_aa"])
def test_bench_operating_points_replica(P, form):
    import bench
    w = gen.config5(nx=16, nz=4)
    g = golden("cfg5r")
    out = solve(P, w, **bench.OP[form])
    assert out["status"] == 0
    assert abs(out["kappa"] - g["kappa_cc"]) <= 1e-4 * g["kappa_cc"]
