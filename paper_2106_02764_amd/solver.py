"""Convenience layer over the C ABI: one geometry + material + caller-owned
device workspace, and the autograd function for d kappa / d sigma.
Argument marshalling only; every step runs in libobte.so."""
from __future__ import annotations

import numpy as np
import torch

from . import obte as _o


class Solver:
    """Owns one obte_mesh handle and a device workspace (torch tensor)."""

    def __init__(self, ndim, n, L, solid, periodic, grad_axis, dT, mfp, dirs, dir_w, kappa_m,
                 device="cuda", modes=None, modes_exact=False):
        self.ndim = ndim
        self.n = tuple(int(v) for v in n)
        self.device = torch.device(device)
        self.mesh = _o.obte_mesh_create(ndim, n, L, solid, periodic, grad_axis, dT)
        _o.obte_material_set(self.mesh, mfp, dirs, dir_w, kappa_m, modes=modes, modes_exact=modes_exact)
        self.n_modes = 0 if modes is None else len(modes[1])
        c = _o.obte_mesh_counts(self.mesh)
        self.n_cells, self.n_solid, self.n_walls, self.n_systems = (
            c["n_cells"], c["n_solid"], c["n_walls"], c["n_systems"])
        self.n_mfp = 1 if (modes is not None and modes_exact) else len(mfp)
        self.n_dir = self.n_systems // self.n_mfp
        self.workspace = None
        self.last_stats = None
        self._sigma = None
        self.solve_count = 0      # completed solves on this mesh (state checks of KappaEff)
        # a stream of our own (default priority) so the outer loop can be
        # captured into HIP graphs; torch's legacy default stream cannot
        self.stream = torch.cuda.Stream(device=self.device) if self.device.type == "cuda" else None

    @classmethod
    def from_workload(cls, w, device="cuda"):
        return cls(w.ndim, w.n, w.L, w.solid, w.periodic, w.grad_axis, w.dT, w.mfp, w.dirs,
                   w.dir_w, w.kappa_m, device=device, modes=getattr(w, "modes", None),
                   modes_exact=getattr(w, "modes_exact", False))

    def opts(self, **kw):
        return _o.default_opts(**kw)

    def ensure_workspace(self, opts):
        nbytes = _o.obte_workspace_size(self.mesh, opts)
        if self.workspace is None or self.workspace.numel() < nbytes:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.workspace

    def sigma_tensor(self, sigma):
        if sigma is None:
            return None
        if isinstance(sigma, torch.Tensor):
            return sigma.to(device=self.device, dtype=torch.float64).contiguous()
        return torch.as_tensor(np.asarray(sigma, np.float64), device=self.device).contiguous()

    def _stream(self, stream):
        s = stream or self.stream
        s.wait_stream(torch.cuda.current_stream(self.device))
        return s

    def solve(self, opts=None, sigma=None, want_T_L=True, want_J=False, stream=None, **kw):
        opts = opts or self.opts(**kw)
        ws = self.ensure_workspace(opts)
        T_L = torch.empty(self.n_cells, dtype=torch.float64, device=self.device) if want_T_L else None
        J = torch.empty(self.n_cells * self.ndim, dtype=torch.float64, device=self.device) if want_J else None
        self._sigma = self.sigma_tensor(sigma)
        s = self._stream(stream)
        self.solve_count += 1
        st = _o.obte_solve(self.mesh, opts, self._sigma, ws, stream=s, T_L=T_L, J=J)
        torch.cuda.current_stream(self.device).wait_stream(s)
        self.last_stats = st
        out = st.as_dict()
        if want_T_L:
            out["T_L"] = T_L
        if want_J:
            out["J"] = J.view(self.n_cells, self.ndim)
        return out

    def kappa(self):
        return _o.obte_kappa(self.mesh, self.n_mfp)

    def system_counts(self):
        """Per-system (inner iterations, sweeps) of the last solve."""
        return _o.obte_system_counts(self.mesh)

    def kappa_modes(self):
        """Mode-resolved conductivity of the last solve (mode table only)."""
        return _o.obte_kappa_modes(self.mesh)

    def adjoint(self, opts, stream=None):
        g = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        s = self._stream(stream)
        st = _o.obte_adjoint(self.mesh, opts, self._sigma, self.workspace, g, stream=s)
        torch.cuda.current_stream(self.device).wait_stream(s)
        return g, st.as_dict()

    def apply(self, x, sys_ids, precision=0, transpose=False, sigma=None, stream=None):
        dt = torch.float64 if precision == 0 else torch.float32
        x = x.to(device=self.device, dtype=dt).contiguous()
        y = torch.empty_like(x)
        ids = torch.as_tensor(np.asarray(sys_ids, np.int32), device=self.device)
        sg = self.sigma_tensor(sigma)
        s = self._stream(stream)
        _o.obte_upwind_apply(self.mesh, precision, transpose, sg, ids, x, y, stream=s)
        torch.cuda.current_stream(self.device).wait_stream(s)
        return y

    def checkpoint_save(self, path):
        _o.obte_checkpoint_save(self.mesh, self.workspace, path)

    def checkpoint_load(self, path):
        _o.obte_checkpoint_load(self.mesh, self.workspace, path)

    def close(self):
        if self.mesh is not None:
            _o.obte_mesh_destroy(self.mesh)
            self.mesh = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class KappaEff(torch.autograd.Function):
    """kappa_eff(sigma) with the hand-written adjoint as its backward.

    The adjoint reads the converged forward state the solver keeps in its
    workspace.  forward() solves with its own copy of sigma and records the
    solver's solve count; when another solve ran on the same solver before
    backward() (another sigma, or this one changed in place), backward()
    first re-runs this graph's forward solve from the saved copy, so the
    gradient always belongs to the sigma of its own graph."""

    @staticmethod
    def forward(ctx, sigma, solver, opts):
        o = _o.default_opts(**{f: getattr(opts, f) for f, _ in opts._fields_})
        o.keep_state = 1
        sig = solver.sigma_tensor(sigma.detach()).clone()
        out = solver.solve(o, sigma=sig, want_T_L=False)
        ctx.solver = solver
        ctx.opts = o
        ctx.sigma = solver._sigma
        ctx.count = solver.solve_count
        return torch.tensor(out["kappa"], dtype=torch.float64, device=sigma.device)

    @staticmethod
    def backward(ctx, g):
        s = ctx.solver
        if s.solve_count != ctx.count or s._sigma is not ctx.sigma:
            s.solve(ctx.opts, sigma=ctx.sigma, want_T_L=False)
            s._sigma = ctx.sigma
            ctx.count = s.solve_count
        grad, _ = s.adjoint(ctx.opts)
        return g * grad, None, None


def solve_batch(solvers, opts, sigmas=None, device="cuda"):
    """All geometries in one launch per pass; returns (kappas, stats dicts)."""
    nbytes = _o.obte_workspace_size_batch([s.mesh for s in solvers], opts)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    sg = [None] * len(solvers) if sigmas is None else [s.sigma_tensor(x) for s, x in zip(solvers, sigmas)]
    stream = solvers[0].stream
    stream.wait_stream(torch.cuda.current_stream())
    k, st = _o.obte_solve_batch([s.mesh for s in solvers], opts, sg, ws, stream=stream)
    torch.cuda.current_stream().wait_stream(stream)
    return k, [x.as_dict() for x in st]


class UMeshSolver:
    """One unstructured 2D mesh (obte_umesh handle) with its material."""

    def __init__(self, nodes, cells, shifts, solid, L, grad_axis, dT, mfp, dirs, dir_w, kappa_m, device="cuda"):
        self.device = torch.device(device)
        self.n_cells = len(cells)
        self.mesh = _o.obte_umesh_create(nodes, cells, shifts, solid, L, grad_axis, dT)
        _o.obte_umesh_material_set(self.mesh, mfp, dirs, dir_w, kappa_m)
        L_ = _o.lib()
        self.n_solid = L_.obte_umesh_n_solid(self.mesh)
        self.n_faces = L_.obte_umesh_n_faces(self.mesh)
        self.n_walls = L_.obte_umesh_n_walls(self.mesh)
        self.n_dir = len(dir_w)
        self.n_systems = len(mfp) * self.n_dir
        self.stream = torch.cuda.Stream(device=self.device)

    @classmethod
    def from_workload(cls, w, device="cuda"):
        return cls(w.nodes, w.cells, w.shifts, w.solid, w.L, w.grad_axis, w.dT, w.mfp, w.dirs, w.dir_w,
                   w.kappa_m, device=device)

    def levels(self):
        return [_o.lib().obte_umesh_n_levels(self.mesh, l) for l in range(self.n_dir)]

    def opts(self, **kw):
        return _o.default_opts(**kw)

    def fourier(self, tol=1e-13, max_outer=1000, cg_tol=1e-14):
        T = torch.zeros(self.n_cells, dtype=torch.float64, device=self.device)
        kF, it, st = _o.obte_umesh_fourier(self.mesh, tol, max_outer, cg_tol, T, stream=self.stream)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return {"T": T, "kappa_fourier": kF, "outer_iters": it, "status": st}

    def solve(self, opts, sigma=None, want_T_L=True):
        sg = None
        if sigma is not None:
            sg = torch.as_tensor(np.asarray(sigma, np.float64), device=self.device).contiguous()
        T_L = torch.zeros(self.n_cells, dtype=torch.float64, device=self.device) if want_T_L else None
        st = _o.obte_umesh_solve(self.mesh, opts, sg, T_L, stream=self.stream)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        out = st.as_dict()
        out["T_L"] = T_L
        return out

    def close(self):
        if getattr(self, "mesh", None):
            _o.lib().obte_umesh_destroy(self.mesh)
            self.mesh = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
