"""CPU: the autotuner's candidate loop, with the timing replaced by a fake
(no device): a candidate the library rejects is skipped, in every stage."""
import types

import pytest

from tests._lib import ensure_built


@pytest.fixture(scope="module")
def A():
    ensure_built()
    from paper_2106_02764_amd import autotune, obte
    return types.SimpleNamespace(autotune=autotune, obte=obte)


def test_rejected_candidates_are_skipped(A, monkeypatch, tmp_path):
    """Wide workgroups win under dispatch 0, and the queue rejects them (as
    the library does for FP64 with more than 4 systems per workgroup): the
    tuner keeps the best accepted shape instead of failing."""
    tried = []

    def fake_measure(solvers, opts, passes=4):
        w, d = list(opts.waves_by_class), int(opts.dispatch)
        tried.append((tuple(w), d))
        if w[1] == 2:
            raise A.obte.ObteError(A.obte.OBTE_ERR_ARG, "rejected candidate")
        if d == 2 and max(w) > 4:
            raise A.obte.ObteError(A.obte.OBTE_ERR_ARG, "queue cap")
        return 1.0 - 0.1 * w[1] - 0.05 * d

    monkeypatch.setattr(A.autotune, "measure", fake_measure)
    monkeypatch.setattr(A.autotune, "_key", lambda solvers, opts, device=None: "fake|shapes")
    solvers = [types.SimpleNamespace(n=(100, 40, 1), n_systems=8) for _ in range(2)]
    o = A.obte.default_opts(precision=A.obte.OBTE_FP64)
    choice = A.autotune.tune(solvers, o, cache_path=str(tmp_path / "cache.json"))
    # rows of 100 cells: launch class 2 (two cells per lane)
    assert choice["waves_by_class"] == [0, 8, 0, 0]
    assert choice["dispatch"] == 1
    assert "class2_w2" not in choice["timings"] and "class2_w4" in choice["timings"]
    assert "dispatch2" not in choice["timings"] and "dispatch1" in choice["timings"]
    assert ((0, 8, 0, 0), 2) in tried
    again = A.autotune.tune(solvers, o, cache_path=str(tmp_path / "cache.json"))
    assert again["from_cache"] and again["waves_by_class"] == choice["waves_by_class"]
