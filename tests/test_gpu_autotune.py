"""GPU: the launch-shape autotuner (systems per workgroup per launch class,
dispatch order, one persistent launch with a device-side item queue) on a batch that spans three launch classes: the choice is
cached and reused, and it leaves FP64 results bitwise unchanged."""
import numpy as np
import pytest

from inputs import gen
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return require_gpu()


def _batch():
    # widths 40, 100 and 150 (one, two and three cells per lane), each with a
    # square pore
    return [gen.small_2d(n, 16, solid=gen.square_block_mask(n, 16, 4, 10), n_dir=8, n_mfp=6,
                         L=n * 1e-9, Ly=16e-9) for n in (40, 100, 150)]


def test_tuned_shape_cached_and_bitwise_neutral(P, tmp_path, monkeypatch):
    ws = _batch()
    solvers = [P.Solver.from_workload(w) for w in ws]
    o = P.default_opts(outer_tol=1e-10, inner_tol=1e-13, fourier_tol=1e-12, max_outer=3000, accel=4)
    cache = str(tmp_path / "tune.json")
    calls = []
    real = P.autotune.measure
    monkeypatch.setattr(P.autotune, "measure", lambda *a, **k: calls.append(1) or real(*a, **k))
    choice = P.autotune.tune(solvers, o, cache_path=cache)
    assert len(calls) >= 1 + 3 * 4          # baseline, 3 classes x 4 candidates (+ dispatch)
    assert len(choice["waves_by_class"]) == 4 and choice["dispatch"] in (0, 1, 2)
    assert all(0 <= w <= 8 for w in choice["waves_by_class"])
    n = len(calls)
    again = P.autotune.tune(solvers, o, cache_path=cache)
    assert len(calls) == n                    # served from the cache, nothing timed
    assert again["from_cache"] and not choice["from_cache"]
    assert again["waves_by_class"] == choice["waves_by_class"] and again["dispatch"] == choice["dispatch"]
    k0, st0 = P.solve_batch(solvers, o)
    ot = P.autotune.apply(P.default_opts(**{f: getattr(o, f) for f, _ in o._fields_}), choice)
    k1, st1 = P.solve_batch(solvers, ot)
    assert [s["status"] for s in st0] == [0, 0, 0] and [s["status"] for s in st1] == [0, 0, 0]
    assert k0 == k1                            # bitwise
    # every other shape too: one system per workgroup everywhere, the
    # batch-wide longest-MFP-first order
    ox = P.autotune.apply(P.default_opts(**{f: getattr(o, f) for f, _ in o._fields_}),
                          {"waves_by_class": [1, 8, 4, 0], "dispatch": 1})
    k2, _ = P.solve_batch(solvers, ox)
    assert k2 == k0
    # one persistent launch over the three classes (device-side item queue),
    # with equal and with mixed systems per workgroup
    for wc in ([1, 1, 1, 0], [2, 1, 4, 0]):
        oq = P.autotune.apply(P.default_opts(**{f: getattr(o, f) for f, _ in o._fields_}),
                              {"waves_by_class": wc, "dispatch": 2})
        kq, stq = P.solve_batch(solvers, oq)
        assert [x["status"] for x in stq] == [0, 0, 0]
        assert kq == k0


@pytest.mark.parametrize("precision", [0, 1])
def test_queue_launch_four_classes(P, precision):
    """dispatch = 2 runs the items of all four cells-per-lane classes in one
    persistent launch (workgroups taking items from a device-side queue):
    the same kappa, kappa_face and pass count as one launch per class, and
    the adjoint of a queued forward solve equals the per-class one."""
    ws = [gen.small_2d(n, 12, solid=gen.square_block_mask(n, 12, 3, 8), n_dir=8, n_mfp=5,
                       L=n * 1e-9, Ly=12e-9) for n in (40, 100, 150, 220)]
    solvers = [P.Solver.from_workload(w) for w in ws]
    base = dict(precision=precision, outer_tol=1e-9, inner_tol=1e-12 if precision == 0 else 1e-6,
                fourier_tol=1e-12, max_outer=3000, accel=4)
    res = {}
    for d in (0, 2):
        k, st = P.solve_batch(solvers, P.default_opts(**base, dispatch=d))
        assert [x["status"] for x in st] == [0, 0, 0, 0]
        res[d] = (k, [x["kappa_face"] for x in st], [x["outer_iters"] for x in st])
    assert res[2] == res[0]                       # bitwise: the order of items changes no sum
    if precision == 0:
        s = P.Solver.from_workload(ws[3])
        grads = []
        for d in (0, 2):
            o = s.opts(**base, keep_state=1, dispatch=d)
            out = s.solve(o, want_T_L=False)
            assert out["status"] == 0
            g, _ = s.adjoint(o)
            grads.append(g.cpu().numpy())
        assert np.array_equal(grads[0], grads[1])


def test_fp64_wide_rows_cap_systems_per_workgroup(P):
    """FP64 sweeps of 3 or 4 cells per lane run at most 4 systems per
    workgroup (their kernels' register budget): 8 is refused on the host
    for those classes, accepted in FP32 and for narrower rows; the automatic
    choice stays within the cap."""
    w = gen.small_2d(150, 8, n_dir=8, n_mfp=9, L=150e-9, Ly=8e-9)
    s = P.Solver.from_workload(w)
    O = P.obte
    with pytest.raises(P.ObteError) as e:
        O.obte_workspace_size(s.mesh, P.default_opts(precision=0, waves_by_class=[0, 0, 8, 0]))
    assert e.value.status == O.OBTE_ERR_ARG
    assert O.obte_workspace_size(s.mesh, P.default_opts(precision=1, waves_by_class=[0, 0, 8, 0])) > 0
    assert O.obte_workspace_size(s.mesh, P.default_opts(precision=0, waves_by_class=[8, 8, 4, 4])) > 0
    out = s.solve(s.opts(precision=0, outer_tol=1e-8, waves_per_group=0), want_T_L=False)
    assert out["status"] == 0
