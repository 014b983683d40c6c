"""Benchmark: converged kappa_eff solves/s (and cell*dir*MFP DoF/s) of the
aMFP-BTE hot path on one MI355X, FP32-sweep form and FP64 form, at 1e-4
relative kappa error, on the 128x128 porous-cell workload.

A step is one converged kappa_eff computation through the C ABI: the Fourier
first guess, then source-iteration passes (batched (m,l) solves + reductions)
until the relative kappa change meets the tolerance that gives <= 1e-4 error.
Inputs (mesh tables, material weights, sigma) are resident on the device
before the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("converged κ_eff solves/s and cell·dir·MFP DoF/s, FP32 vs FP64, "
          "at 1e-4 rel err")
PEAK = {"fp64_vector_tflops": 78.6, "fp32_vector_tflops": 157.3, "hbm_gbs": 8000.0}
# algorithmic flops of one upwind sweep per solid cell: the triangular update
# x = (b + c_x x_up,x + c_y x_up,y) / d  (2 FMA + 1 divide, counted as 5)
FLOPS_PER_CELL_SWEEP = {2: 5, 3: 7}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=20.0)
    p.add_argument("--workload", default="cfg2")
    p.add_argument("--copy-probe", type=int, default=0,
                   help="only run a plain device copy of this many bytes (scales rocprofv3 "
                        "FETCH_SIZE / WRITE_SIZE) and exit")
    return p.parse_args()


def copy_probe(nbytes):
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "launches": 3}), flush=True)


def make_workload(name):
    from inputs import gen
    if name == "cfg2":
        return gen.config2()
    if name == "cfg1":
        return gen.config1()
    if name == "cfg4":
        return gen.config4()
    if name == "cfg5":
        return gen.config5()
    raise SystemExit(f"unknown workload {name}")


def batch_bench(a):
    """64 geometries of uneven size in one launch per pass: geometry solves/s."""
    import torch
    import paper_2106_02764_amd as P
    from inputs import gen
    geoms = gen.config3()
    solvers = [P.Solver.from_workload(w) for w in geoms]
    dof = sum(w.dof for w in geoms)
    ref, _ = P.solve_batch(solvers, P.default_opts(outer_tol=1e-10, inner_tol=1e-12,
                                                   fourier_tol=1e-10, max_outer=4000))
    out = {}
    for name, prec, itol in (("fp32", 1, 1e-5), ("fp64", 0, 1e-8)):
        o = P.default_opts(precision=prec, outer_tol=3e-6, inner_tol=itol, inner_rtol=0.3,
                           lag_wrap=1, fourier_tol=1e-6, max_outer=4000, passes_per_graph=4)
        o.waves_per_group = P.autotune.tune(solvers, o)
        for _ in range(a.warmup):
            P.solve_batch(solvers, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            k, st = P.solve_batch(solvers, o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        err = max(abs(x - y) / y for x, y in zip(k, ref))
        out[name] = {"geometry_solves_per_s": len(geoms) / dt, "ms_per_batch": 1e3 * dt,
                     "dof_per_s": dof / dt, "max_kappa_rel_err_vs_fp64_ref": err,
                     "waves_per_group": o.waves_per_group,
                     "max_passes": max(x["outer_iters"] for x in st)}
    print(json.dumps({"workload": "64 periodic geometries (48^2..256^2, 1-4 circular pores, "
                      "L 50-500 nm), 48 directions x 30 MFPs, one launch per pass",
                      "dof": dof, **out}), flush=True)


def time_solves(P, solver, opts, steps, warmup):
    import torch
    for _ in range(warmup):
        solver.solve(opts, want_T_L=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweep_ms = red_ms = four_ms = 0.0
    launches = passes = sweeps = inner = 0
    k = None
    for _ in range(steps):
        out = solver.solve(opts, want_T_L=False)
        sweep_ms += out["sweep_ms"]
        red_ms += out["reduce_ms"]
        four_ms += out["fourier_ms"]
        launches += out["sweep_launches"]
        passes += out["outer_iters"]
        sweeps += out["sweeps"]
        inner += out["inner_iters"]
        k = out["kappa"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"seconds": dt, "kappa": k, "sweep_ms": sweep_ms, "reduce_ms": red_ms,
            "fourier_ms": four_ms, "launches": launches, "passes": passes, "sweeps": sweeps,
            "inner_iters": inner, "status": out["status"]}


def calibrate(P, solver, prec, kref, inner_tol):
    """Fastest configuration (inner-iteration cap per pass, loosest outer
    tolerance) whose kappa is within 1e-4 of the reference; Algorithm 1 stops
    on the relative change, which understates the error.  Untimed."""
    import torch
    best = None
    for lag, rtol in ((1, 0.3), (1, 0.1), (0, 0.1), (0, 0.0)):
        for tol in (3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7):
            o = solver.opts(precision=prec, outer_tol=tol, inner_tol=inner_tol, fourier_tol=1e-6,
                            passes_per_graph=4, inner_rtol=rtol, lag_wrap=lag)
            solver.solve(o, want_T_L=False)           # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = solver.solve(o, want_T_L=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = abs(out["kappa"] - kref) / abs(kref)
            if err <= 0.5e-4 and out["status"] == 0:
                if best is None or dt < best[2]:
                    best = (o, err, dt)
                break
    return best[0], best[1]


def cpu_baseline_measure(w, seconds):
    """Time the FP64 oracle on the same workload before the GPU is touched:
    every (m, l) system factored once (SuperLU, reused as in the paper) and a
    few source-iteration passes, with the directions spread over the host
    cores.  Bounded by `seconds` of passes."""
    from oracle.parallel import source_iteration_parallel
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    t0 = time.perf_counter()
    r = source_iteration_parallel(w, n_workers=cores, n_passes=3, time_limit=seconds)
    total = time.perf_counter() - t0
    return {"cores": cores, "t_factor": r["t_factor"], "pass_s": float(r["pass_times"].mean()),
            "passes_run": int(r["passes"]), "wall_s": total}


def cpu_baseline_value(m, passes, dof):
    per_solve = m["t_factor"] + passes * m["pass_s"]
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": m["cores"], "kind": "oracle",
            "sample": (f"full workload, all systems factored ({m['t_factor']:.1f}s) + "
                       f"{m['passes_run']} passes ({m['pass_s']:.3f}s each) on {m['cores']} worker "
                       f"processes; extrapolated to the {passes} passes of the FP64 GPU solve"),
            "dof_per_s": dof / per_solve, "seconds_per_solve_estimate": per_solve}


def main():
    a = parse()
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.workload == "cfg3":
        batch_bench(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is design-only)"}))
        sys.exit(2)
    w = make_workload(a.workload)
    cpu = None if a.no_cpu else cpu_baseline_measure(w, a.cpu_seconds)
    import torch
    import paper_2106_02764_amd as P

    solver = P.Solver.from_workload(w)
    dof = w.dof
    # reference: FP64 GPU form converged far below the target error (untimed)
    oref = solver.opts(outer_tol=1e-11, inner_tol=1e-12, fourier_tol=1e-12)
    ref = solver.solve(oref, want_T_L=False)
    kref = ref["kappa"]
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"{a.workload}_oracle.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))
    res = {}
    for name, prec, itol in (("fp32", 1, 1e-5), ("fp64", 0, 1e-8)):
        o, cal_err = calibrate(P, solver, prec, kref, itol)
        # leg 1: the throughput (pass kernels replayed as HIP graphs)
        r = time_solves(P, solver, o, a.steps, a.warmup)
        # leg 2: the same solves with HIP events around every kernel launch on
        # the library's stream (direct launches), for the per-kernel durations
        ot = solver.opts(**{f: getattr(o, f) for f, _ in o._fields_})
        ot.timing = 1
        rt = time_solves(P, solver, ot, a.steps, 0)
        for key in ("sweep_ms", "reduce_ms", "fourier_ms", "launches"):
            r[key] = rt[key]
        r["timed_leg_solves_per_s"] = a.steps / rt["seconds"]
        r["sweeps_timed_leg"] = rt["sweeps"]
        r["outer_tol"] = o.outer_tol
        r["inner_tol"] = o.inner_tol
        r["max_inner"] = o.max_inner
        r["inner_rtol"] = o.inner_rtol
        r["lag_wrap"] = o.lag_wrap
        r["kappa_rel_err_vs_fp64_ref"] = abs(r["kappa"] - kref) / abs(kref)
        if golden:
            r["kappa_rel_err_vs_oracle"] = abs(r["kappa"] - golden["kappa_cc"]) / golden["kappa_cc"]
        r["solves_per_s"] = a.steps / r["seconds"]
        r["dof_per_s"] = dof * a.steps / r["seconds"]
        r["ms_per_solve"] = 1e3 * r["seconds"] / a.steps
        res[name] = r
    main_r = res["fp32"]
    # roofline of the dominant kernel (the sweep pass): algorithmic flops per
    # launch = sweeps in that launch x solid cells x flops per cell-sweep
    sweeps_per_launch = main_r["sweeps_timed_leg"] / max(main_r["launches"], 1)
    flops_launch = sweeps_per_launch * w.n_solid * FLOPS_PER_CELL_SWEEP[w.ndim]
    avg_ms = main_r["sweep_ms"] / max(main_r["launches"], 1)
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK["fp32_vector_tflops"],
            "unit": "TFLOP/s", "frac": achieved / PEAK["fp32_vector_tflops"], "traffic": None,
            "kernel": "k_sweep_pass<float,2,1>", "avg_launch_ms": avg_ms,
            "sweeps_per_launch": sweeps_per_launch}
    line = {
        "metric": METRIC, "value": main_r["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": main_r["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("128x128 periodic cell, centred circular pore r=%.3f nm (seeded), "
                                "L=100 nm, 48 directions x 30 MFPs (1 nm..100 um), lognormal "
                                "kernel, 1e-4 rel kappa error" % (w.meta["pore_radius"] * 1e9)
                                if a.workload == "cfg2" else a.workload),
                   "solid_cells": w.n_solid, "systems": w.n_systems, "dof": dof},
        "dof_per_s": main_r["dof_per_s"],
        "kappa": main_r["kappa"], "kappa_ref_fp64": kref,
        "fp32": res["fp32"], "fp64": res["fp64"],
        "roofline": roof,
    }
    if golden:
        line["kappa_oracle"] = golden["kappa_cc"]
    if cpu is not None:
        line["cpu_baseline"] = cpu_baseline_value(cpu, int(round(res["fp64"]["passes"] / a.steps)), dof)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
