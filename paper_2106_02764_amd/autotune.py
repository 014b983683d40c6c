"""Launch-shape autotuner of the pass kernel.

The knobs are the systems per workgroup of each cells-per-lane launch class
(``waves_by_class``) and how the work items are dispatched (``dispatch``:
one launch per class geometry by geometry, longest MFPs first over all
geometries, or one persistent launch whose workgroups take the items from a
device-side queue).  Neither changes a result (FP64 runs are bitwise the same),
only the time of a pass.  ``tune`` times a few passes per candidate with the
library's own HIP-event timers (coordinate descent: one class at a time,
then the dispatch order) and caches the winner per (device, mesh shapes,
systems, precision, operating point) in a small JSON file.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import obte as _o

CACHE = os.environ.get("OBTE_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "obte_autotune.json"))


def _copy(opts, **kw):
    o = _o.default_opts(**{f: getattr(opts, f) for f, _ in opts._fields_})
    for k, v in kw.items():
        if k == "waves_by_class":
            v = (type(o.waves_by_class))(*v)
        setattr(o, k, v)
    return o


def _key(solvers, opts, device=None):
    dev = torch.cuda.get_device_name() if device is None else device
    shapes = sorted({(tuple(s.n), s.n_systems) for s in solvers})
    return (f"{dev}|{shapes}|prec{opts.precision}|rtol{opts.inner_rtol}|lag{opts.lag_wrap}"
            f"|accel{opts.accel}")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(solvers, opts, cache_path=None):
    """A cached choice for these meshes and options taken on any device, or
    None (for processes that cannot read the device name, e.g. under a
    profiler's tool library)."""
    if not isinstance(solvers, (list, tuple)):
        solvers = [solvers]
    rest = _key(solvers, opts, device="").split("|", 1)[1]
    for k, v in _load(cache_path or CACHE).items():
        if k.split("|", 1)[1] == rest:
            return dict(v, from_cache=True)
    return None


def classes(solvers):
    """Launch classes (cells per lane) of these meshes."""
    return sorted({math.ceil(s.n[0] / 64) for s in solvers})


def measure(solvers, opts, passes=4):
    """Mean duration (ms) of the pass-kernel launches of `passes` passes."""
    from .solver import solve_batch
    o = _copy(opts, outer_tol=0.0, max_outer=passes, timing=1, only_fourier=0)
    if len(solvers) == 1:
        st = solvers[0].solve(o, want_T_L=False)
    else:
        st = solve_batch(solvers, o)[1][0]
    return st["sweep_ms"] / max(st["sweep_launches"], 1)


def apply(opts, choice):
    """Set a tuned choice on `opts` (in place) and return it."""
    opts.waves_by_class = (type(opts.waves_by_class))(*choice["waves_by_class"])
    opts.dispatch = int(choice["dispatch"])
    return opts


def tune(solvers, opts, candidates=(1, 2, 4, 8), passes=4, use_cache=True, cache_path=None):
    """The best launch shape for `solvers` (one Solver or a list) under
    `opts`: {"waves_by_class": [W1, W2, W3, W4], "dispatch": d, ...}; `opts`
    is not modified (use ``apply``)."""
    if not isinstance(solvers, (list, tuple)):
        solvers = [solvers]
    path = cache_path or CACHE
    key = _key(solvers, opts)
    cache = _load(path) if use_cache else {}
    if key in cache:
        return dict(cache[key], from_cache=True)
    wc = [0, 0, 0, 0]
    best = measure(solvers, _copy(opts, waves_by_class=wc, dispatch=0), passes)
    timings = {"auto": best}
    for c in classes(solvers):
        for w in candidates:
            trial = list(wc)
            trial[c - 1] = w
            try:
                ms = measure(solvers, _copy(opts, waves_by_class=trial, dispatch=0), passes)
            except _o.ObteError:
                continue        # e.g. the candidate needs more LDS than a workgroup has
            timings[f"class{c}_w{w}"] = ms
            if ms < best:
                best, wc = ms, trial
    disp = 0
    if len(solvers) > 1:
        for d in (1, 2):
            try:
                ms = measure(solvers, _copy(opts, waves_by_class=wc, dispatch=d), passes)
            except _o.ObteError:
                continue        # e.g. the queue's FP64 cap of 4 systems per workgroup
            timings[f"dispatch{d}"] = ms
            if ms < best:
                best, disp = ms, d
    choice = {"waves_by_class": wc, "dispatch": disp, "ms_per_pass_launch": best, "timings": timings,
              "from_cache": False}
    if use_cache:
        cache = _load(path)
        cache[key] = choice
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return choice
