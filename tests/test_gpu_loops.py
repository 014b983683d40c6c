"""The graph loops queue the next replay before the host reads the previous
one's flags (the outer pass loop and the Fourier CG loop).  Whatever runs
after the stop must exit at once: pass and iteration counts, kappa, T_L and
the adjoint gradient equal those of one pass per launch (no replay queued
ahead), bit for bit in FP64."""
import numpy as np
import pytest

from inputs import gen
from tests.gpu_common import gpu_solve, require_gpu

pytestmark = pytest.mark.gpu

TIGHT = dict(inner_tol=1e-13, fourier_tol=1e-12)


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def _w():
    return gen.small_2d(12, 10, solid=gen.square_block_mask(12, 10, 3, 7), n_dir=8, n_mfp=3)


@pytest.mark.parametrize("K", [3, 4, 8])
@pytest.mark.parametrize("max_outer", [5, 7, 13])
def test_pass_replays_stop_at_max_outer(P, K, max_outer):
    w = _w()
    r1 = gpu_solve(P, w, outer_tol=0.0, max_outer=max_outer, passes_per_graph=1, **TIGHT)
    rk = gpu_solve(P, w, outer_tol=0.0, max_outer=max_outer, passes_per_graph=K, **TIGHT)
    assert r1["outer_iters"] == max_outer and rk["outer_iters"] == max_outer
    assert rk["kappa"] == r1["kappa"]
    assert np.array_equal(rk["T_L"], r1["T_L"])


@pytest.mark.parametrize("K", [3, 4])
@pytest.mark.parametrize("accel", [0, 8])
def test_pass_replays_converged(P, K, accel):
    w = _w()
    r1 = gpu_solve(P, w, outer_tol=1e-9, accel=accel, passes_per_graph=1, **TIGHT)
    rk = gpu_solve(P, w, outer_tol=1e-9, accel=accel, passes_per_graph=K, **TIGHT)
    assert r1["status"] == 0 and rk["status"] == 0
    assert rk["outer_iters"] == r1["outer_iters"]
    assert rk["kappa"] == r1["kappa"]
    assert np.array_equal(rk["T_L"], r1["T_L"])


def test_adjoint_replays(P):
    rng = np.random.default_rng(3)
    w = gen.small_2d(10, 9, solid=gen.square_block_mask(10, 9, 3, 6), n_dir=8, n_mfp=3,
                     sigma=rng.uniform(0.5, 2.0, 90))
    out = []
    for K in (1, 4):
        s = P.Solver.from_workload(w)
        o = s.opts(outer_tol=1e-12, inner_tol=1e-14, fourier_tol=1e-14, keep_state=1, passes_per_graph=K,
                   max_outer=5000)
        s.solve(o, sigma=w.sigma, want_T_L=False)
        g, st = s.adjoint(o)
        out.append((g.cpu().numpy(), st["outer_iters"], st["status"]))
    assert out[0][2] == 0 and out[1][2] == 0
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


@pytest.mark.parametrize("max_fourier", [0, 3, 8, 11])
def test_fourier_replays_stop_at_max_fourier(P, max_fourier):
    """CG replays of 8 iterations: with a tolerance it cannot reach, the
    count stops at the bound whatever replays were queued past it."""
    w = _w()
    r = gpu_solve(P, w, outer_tol=1e-6, fourier_tol=1e-300, max_fourier=max_fourier, inner_tol=1e-12)
    assert r["fourier_iters"] == max_fourier
    assert r["status"] == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_waves_per_group_independent(P, dim):
    """The systems sharing a workgroup (and so the dispatch order of the work
    items) change nothing in the result: FP64 kappa and T_L bit for bit."""
    from tests.test_gpu_parity import ragged_porous, small3d
    w = ragged_porous() if dim == 2 else small3d()
    runs = [gpu_solve(P, w, outer_tol=1e-9, waves_per_group=W, **TIGHT) for W in (1, 2, 4)]
    for r in runs[1:]:
        assert r["outer_iters"] == runs[0]["outer_iters"]
        assert r["kappa"] == runs[0]["kappa"]
        assert np.array_equal(r["T_L"], runs[0]["T_L"])
