"""GPU: obte_solve_noalloc (workspace in the library's per-device static
array) against obte_solve with a caller workspace, through the C ABI: two
calls in a row, the second on a smaller mesh, FP64 (bitwise: same kernels
in the same order) and FP32."""
import numpy as np
import pytest
import torch

from inputs import gen
from tests.gpu_common import require_gpu
from tests.test_gpu_parity import ragged_porous

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def _both(P, w, **opt):
    s = P.Solver.from_workload(w)
    o = s.opts(**opt)
    n, nd = s.n_cells, s.ndim
    out = {}
    for label in ("ws", "noalloc"):
        T = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
        J = torch.full((n * nd,), 7.0, dtype=torch.float64, device="cuda")
        if label == "ws":
            ws = s.ensure_workspace(o)
            st = P.obte.obte_solve(s.mesh, o, None, ws, stream=s.stream, T_L=T, J=J)
        else:
            st = P.obte.obte_solve_noalloc(s.mesh, o, None, stream=s.stream, T_L=T, J=J)
        torch.cuda.synchronize()
        out[label] = (st.as_dict(), T.cpu().numpy(), J.cpu().numpy())
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_workspace_solve(P, prec):
    assert P.obte.obte_noalloc_scratch_bytes() == 32 << 20
    tol = dict(outer_tol=1e-12, inner_tol=1e-14, fourier_tol=1e-14, max_inner=200) if prec == 0 else \
        dict(outer_tol=1e-7, inner_tol=1e-6, fourier_tol=1e-10)
    # first call on the larger mesh, then a smaller one in the same array
    for w in (ragged_porous(), gen.small_2d(12, 10, solid=gen.square_block_mask(12, 10, 3, 7), n_dir=8,
                                            n_mfp=3)):
        r = _both(P, w, precision=prec, passes_per_graph=4, accel=4, **tol)
        (sa, Ta, Ja), (sb, Tb, Jb) = r["ws"], r["noalloc"]
        assert sa["status"] == 0 and sb["status"] == 0
        assert sa["outer_iters"] == sb["outer_iters"]
        if prec == 0:
            assert sa["kappa"] == sb["kappa"] and sa["kappa_face"] == sb["kappa_face"]
            assert np.array_equal(Ta, Tb) and np.array_equal(Ja, Jb)
        else:
            assert abs(sa["kappa"] - sb["kappa"]) <= 1e-10 * abs(sa["kappa"])
            assert np.max(np.abs(Ta - Tb)) <= 1e-10 * np.max(np.abs(Ta))
        assert sb["energy_residual"] == sa["energy_residual"] or prec == 1


def test_noalloc_rejects(P):
    w = gen.config2()                      # 1440 systems x 10136 solid cells: beyond 32 MiB
    s = P.Solver.from_workload(w)
    with pytest.raises(P.ObteError) as e:
        P.obte.obte_solve_noalloc(s.mesh, s.opts(), None, stream=s.stream)
    assert e.value.status == P.obte.OBTE_ERR_NOMEM
    small = P.Solver.from_workload(gen.small_2d(8, 6))
    for bad in (dict(init=1), dict(keep_state=1), dict(timing=1)):
        with pytest.raises(P.ObteError) as e:
            P.obte.obte_solve_noalloc(small.mesh, small.opts(**bad), None, stream=small.stream)
        assert e.value.status == P.obte.OBTE_ERR_ARG
