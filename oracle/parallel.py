"""Source iteration with the (m, l) systems spread over worker processes
(oracle; FP64).

Section "Implementation": within a pass the systems are independent, and the
paper assigns a set of directions to each core while the MFPs run serially
on it; all couplings (T_L, T_w) are lagged to the previous pass.  Here each
worker owns the directions l with l % n_workers == rank, keeps the LU factors
of its systems for the whole run, and returns its partial sums of T_L, T_w and
kappa every pass; the parent adds the partials in rank order.  Same
arithmetic as ``bte.source_iteration`` up to the order of the sums.
"""
from __future__ import annotations

import multiprocessing as mp
import time

import numpy as np

from .bte import Problem
from .fourier import fourier_solve


def _worker(work, rank, n_workers, conn):
    import os
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    prob = Problem(work)
    me, mat = prob.mesh, prob.mat
    mine = [l for l in range(mat.n_dir) if l % n_workers == rank]
    t0 = time.perf_counter()
    for l in mine:
        for m in range(mat.n_mfp):
            prob.lu(m, l, cache=True)
    conn.send(("ready", time.perf_counter() - t0))
    while True:
        msg = conn.recv()
        if msg[0] == "stop":
            break
        _, T_L, T_w = msg
        TLp = np.zeros(me.n_solid)
        Twp = np.zeros(me.n_walls)
        Jp = np.zeros((me.n_solid, mat.S.shape[2]))
        kml = {}
        for l in mine:
            for m in range(mat.n_mfp):
                x = prob.lu(m, l).solve(prob.rhs(m, l, T_L, T_w))
                TLp += mat.D[m, l] * x
                Jp += x[:, None] * mat.S[m, l][None, :]
                if me.n_walls:
                    Twp += prob.wout[:, m, l] * x[prob.wall_cell]
                kml[(m, l)] = (prob.kappa_cc_system(m, l, x), prob.kappa_face_system(m, l, x))
        conn.send((TLp, Twp, Jp, kml))


def source_iteration_parallel(work, n_workers=4, tol=1e-8, max_passes=2000, n_passes=None,
                              time_limit=None, verbose=False):
    """Returns kappa_cc, kappa_face, kappa_fourier, T_L (mean-subtracted), the
    flux map J of the last pass (section Model: J_i = sum_ml S_ml T_iml, per
    solid cell), history, passes, and the timings of the factorisation and of
    each pass."""
    ctx = mp.get_context("fork")
    prob = Problem(work)
    me, mat = prob.mesh, prob.mat
    T_F, kF = fourier_solve(me, mat.kappa_axis)
    pipes, procs = [], []
    t_start = time.perf_counter()
    for r in range(n_workers):
        a, b = ctx.Pipe()
        p = ctx.Process(target=_worker, args=(work, r, n_workers, b), daemon=True)
        p.start()
        pipes.append(a)
        procs.append(p)
    try:
        for a in pipes:
            a.recv()
        t_factor = time.perf_counter() - t_start
        T_L = T_F.copy()
        T_w = T_L[prob.wall_cell].copy() if me.n_walls else np.zeros(0)
        hist, histf, pass_times = [], [], []
        kprev = None
        converged = False
        while True:
            t0 = time.perf_counter()
            for a in pipes:
                a.send(("pass", T_L, T_w))
            TL = np.zeros(me.n_solid)
            Tw = np.zeros(me.n_walls)
            J = np.zeros((me.n_solid, mat.S.shape[2]))
            kml = np.zeros((mat.n_mfp, mat.n_dir))
            kfml = np.zeros((mat.n_mfp, mat.n_dir))
            for a in pipes:
                TLp, Twp, Jp, parts = a.recv()
                TL += TLp
                Tw += Twp
                J += Jp
                for (m, l), (kc, kf) in parts.items():
                    kml[m, l] = kc
                    kfml[m, l] = kf
            pass_times.append(time.perf_counter() - t0)
            k = float(kml.sum())
            hist.append(k)
            histf.append(float(kfml.sum()))
            T_L, T_w = TL, Tw
            if verbose:
                print(f"pass {len(hist)}: kappa_cc={k:.12g} ({pass_times[-1]:.2f}s)", flush=True)
            if n_passes is not None:
                if len(hist) >= n_passes:
                    break
            else:
                if kprev is not None and abs(k - kprev) <= tol * abs(k):
                    converged = True
                    break
                if len(hist) >= max_passes:
                    break
            if time_limit is not None and time.perf_counter() - t_start > time_limit:
                break
            kprev = k
    finally:
        for a in pipes:
            try:
                a.send(("stop",))
            except Exception:
                pass
        for p in procs:
            p.join(timeout=10)
    return {"kappa_cc": hist[-1], "kappa_face": histf[-1], "kappa_fourier": kF,
            "kappa_per_mfp": kml.sum(axis=1), "T_L": T_L - T_L.mean(), "J": J, "history": np.asarray(hist),
            "passes": len(hist), "converged": converged, "t_factor": t_factor,
            "pass_times": np.asarray(pass_times), "workers": n_workers}
