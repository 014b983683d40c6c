"""Launch-shape autotuner: picks the systems-per-workgroup (waves_per_group)
of the pass kernel by timing a few passes of each candidate with the
library's own HIP-event timers, and caches the winner per (mesh shape,
systems, precision, device) in a small JSON file."""
from __future__ import annotations

import json
import os

import torch

from . import obte as _o

CACHE = os.environ.get("OBTE_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "obte_autotune.json"))


def _key(solvers, opts):
    dev = torch.cuda.get_device_name()
    shapes = sorted({(s.n, s.n_systems) for s in solvers})
    return f"{dev}|{shapes}|prec{opts.precision}|rtol{opts.inner_rtol}|lag{opts.lag_wrap}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(solvers, opts, candidates=(2, 4, 6, 8), passes=3, use_cache=True):
    """Returns the best waves_per_group for `solvers` (one Solver or a list)
    under `opts`; `opts` is not modified."""
    if not isinstance(solvers, (list, tuple)):
        solvers = [solvers]
    key = _key(solvers, opts)
    cache = _load() if use_cache else {}
    if key in cache:
        return int(cache[key]["waves"])
    from .solver import solve_batch
    best, times = None, {}
    for w in candidates:
        o = _o.default_opts(**{f: getattr(opts, f) for f, _ in opts._fields_})
        o.waves_per_group = w
        o.outer_tol = 0.0
        o.max_outer = passes
        o.timing = 1
        o.only_fourier = 0
        try:
            if len(solvers) == 1:
                st = solvers[0].solve(o, want_T_L=False)
                ms = st["sweep_ms"] / max(st["sweep_launches"], 1)
            else:
                _, sts = solve_batch(solvers, o)
                ms = sts[0]["sweep_ms"] / max(sts[0]["sweep_launches"], 1)
        except _o.ObteError:
            continue        # e.g. the candidate needs more LDS than available
        times[w] = ms
        if best is None or ms < times[best]:
            best = w
    if best is None:
        return 0
    if use_cache:
        cache[key] = {"waves": best, "ms_per_pass": times}
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best
