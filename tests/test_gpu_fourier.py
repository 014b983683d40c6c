"""The Fourier-only workload (only_fourier: the first guess alone, section
Results) over a batch of geometries in one launch sequence: kappa_F against
the oracle's sparse solve and against the Eucken-Maxwell model
r = (1 - phi) / (1 + phi) for circular pores in an infinitely thick
membrane."""
import math

import numpy as np
import pytest

from inputs import gen
from oracle.fourier import fourier_solve
from oracle.mesh import Mesh
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu
NM = 1e-9


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def porous(n, phi, L=100 * NM):
    r = math.sqrt(phi / math.pi) * L
    s = gen.circles_mask(n, n, L, L, [(L / 2, L / 2)], [r])
    return gen.small_2d(n, n, solid=s, n_dir=8, n_mfp=4, L=L, Ly=L)


def test_fourier_batch_eucken_maxwell(P):
    phis = [0.05, 0.1, 0.15, 0.2]
    ws = [porous(160, p) for p in phis] + [porous(96, 0.1), porous(200, 0.15)]
    solvers = [P.Solver.from_workload(w) for w in ws]
    o = P.default_opts(only_fourier=1, fourier_tol=1e-13)
    k, st = P.solve_batch(solvers, o)
    assert all(s["status"] == 0 for s in st)
    for w, kF, s in zip(ws, k, st):
        assert s["kappa_fourier"] == kF
        me = Mesh((w.n[0], w.n[1], 1), (w.L[0], w.L[1], 1.0), w.solid, (1, 1, 0), 0, w.dT, ndim=2)
        _, k_ref = fourier_solve(me, np.array([150.0, 150.0]))
        assert abs(kF - k_ref) <= 1e-10 * k_ref
        por = 1.0 - w.solid.mean()
        em = (1 - por) / (1 + por)
        assert abs(kF / 150.0 - em) < 0.01 * em     # the paper reports < 1%


def test_fourier_batch_matches_single(P):
    """The 64 geometries of the multi-geometry workload, Fourier only: the
    batched launches give each geometry's single-geometry kappa_F."""
    ws = gen.config3()
    solvers = [P.Solver.from_workload(w) for w in ws]
    o = P.default_opts(only_fourier=1, fourier_tol=1e-12)
    k, st = P.solve_batch(solvers, o)
    assert all(s["status"] == 0 for s in st)
    for i in (0, 17, 40, 63):
        r = solvers[i].solve(o, want_T_L=False)
        assert abs(r["kappa_fourier"] - k[i]) <= 1e-11 * abs(k[i])
