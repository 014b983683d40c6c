"""GPU: the launch-shape autotuner (systems per workgroup per launch class,
dispatch order) on a batch that spans three launch classes: the choice is
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
    assert len(choice["waves_by_class"]) == 4 and choice["dispatch"] in (0, 1)
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
                          {"waves_by_class": [1, 2, 8, 0], "dispatch": 1})
    k2, _ = P.solve_batch(solvers, ox)
    assert k2 == k0
