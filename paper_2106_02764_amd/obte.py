"""ctypes binding of the C ABI in include/obte.h (argument marshalling only).

Every function here forwards to the gfx950 library ``libobte.so`` built in
this package directory; nothing is computed in Python.  torch is imported
before the library is loaded so that the process has a single HIP runtime
(torch's), whose device memory and streams the library then shares.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libobte.so")

OBTE_OK, OBTE_ERR_ARG, OBTE_ERR_HIP, OBTE_ERR_STATE = 0, -1, -2, -3
OBTE_ERR_NOT_CONVERGED, OBTE_ERR_NUMERIC, OBTE_ERR_NOMEM = -4, -5, -6
OBTE_FP64, OBTE_FP32 = 0, 1
STATUS_NAMES = {0: "OK", -1: "ERR_ARG", -2: "ERR_HIP", -3: "ERR_STATE", -4: "ERR_NOT_CONVERGED",
                -5: "ERR_NUMERIC", -6: "ERR_NOMEM"}


class ObteError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class obte_mesh_desc(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3),
                ("periodic", C.c_int * 3), ("grad_axis", C.c_int), ("dT_ext", C.c_double),
                ("solid", C.POINTER(C.c_uint8))]


class obte_material_desc(C.Structure):
    _fields_ = [("n_mfp", C.c_int), ("mfp", C.POINTER(C.c_double)), ("n_dir", C.c_int),
                ("dirs", C.POINTER(C.c_double)), ("dir_w", C.POINTER(C.c_double)),
                ("kappa_m", C.POINTER(C.c_double)), ("n_modes", C.c_int),
                ("mode_F", C.POINTER(C.c_double)), ("mode_alpha", C.POINTER(C.c_double)),
                ("mode_dim", C.c_int), ("modes_exact", C.c_int)]


class obte_solve_opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("outer_tol", C.c_double), ("max_outer", C.c_int),
                ("inner_tol", C.c_double), ("max_inner", C.c_int), ("init", C.c_int),
                ("only_fourier", C.c_int), ("passes_per_graph", C.c_int),
                ("waves_per_group", C.c_int), ("fourier_tol", C.c_double),
                ("max_fourier", C.c_int), ("keep_state", C.c_int),
                ("lag_wrap", C.c_int), ("inner_rtol", C.c_double), ("wrap_tol", C.c_double),
                ("timing", C.c_int), ("stop_rule", C.c_int), ("accel", C.c_int),
                ("waves_by_class", C.c_int * 4), ("dispatch", C.c_int)]


class obte_stats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_iters", C.c_longlong), ("sweeps", C.c_longlong),
                ("fourier_iters", C.c_int), ("kappa", C.c_double), ("kappa_face", C.c_double),
                ("kappa_fourier", C.c_double), ("last_rel_change", C.c_double),
                ("wrap_residual", C.c_double), ("status", C.c_int),
                ("sweep_launches", C.c_int), ("sweep_ms", C.c_double), ("reduce_ms", C.c_double),
                ("fourier_ms", C.c_double), ("energy_residual", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = {
    "obte_default_opts": (None, [C.POINTER(obte_solve_opts)]),
    "obte_mesh_create": (C.c_int, [C.POINTER(obte_mesh_desc), C.POINTER(C.c_void_p)]),
    "obte_material_set": (C.c_int, [C.c_void_p, C.POINTER(obte_material_desc)]),
    "obte_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(obte_solve_opts), C.POINTER(C.c_size_t)]),
    "obte_workspace_size_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(obte_solve_opts),
                                            C.POINTER(C.c_size_t)]),
    "obte_solve": (C.c_int, [C.c_void_p, C.POINTER(obte_solve_opts), C.c_void_p, C.c_void_p,
                             C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(obte_stats)]),
    "obte_solve_noalloc": (C.c_int, [C.c_void_p, C.POINTER(obte_solve_opts), C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.POINTER(obte_stats)]),
    "obte_noalloc_scratch_bytes": (C.c_size_t, []),
    "obte_solve_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(obte_solve_opts),
                                   C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t, C.c_void_p,
                                   C.POINTER(C.c_double), C.POINTER(obte_stats)]),
    "obte_kappa": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "obte_kappa_modes": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "obte_system_counts": (C.c_int, [C.c_void_p, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]),
    "obte_adjoint": (C.c_int, [C.c_void_p, C.POINTER(obte_solve_opts), C.c_void_p, C.c_void_p,
                               C.c_size_t, C.c_void_p, C.c_void_p, C.POINTER(obte_stats)]),
    "obte_upwind_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "obte_checkpoint_save": (C.c_int, [C.c_void_p, C.c_void_p, C.c_char_p]),
    "obte_checkpoint_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_char_p]),
    "obte_last_error": (C.c_char_p, []),
    "obte_mesh_destroy": (None, [C.c_void_p]),
    "obte_mesh_n_cells": (C.c_int, [C.c_void_p]),
    "obte_mesh_n_solid": (C.c_int, [C.c_void_p]),
    "obte_mesh_n_walls": (C.c_int, [C.c_void_p]),
    "obte_mesh_n_systems": (C.c_int, [C.c_void_p]),
    "obte_mesh_n_modes": (C.c_int, [C.c_void_p]),
    # unstructured 2D meshes
    "obte_umesh_create": (C.c_int, [C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                    C.c_int, C.c_int, C.POINTER(C.c_uint8), C.c_double, C.c_double, C.c_int,
                                    C.c_double, C.POINTER(C.c_void_p)]),
    "obte_umesh_material_set": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double)]),
    "obte_umesh_fourier": (C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                     C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "obte_umesh_solve": (C.c_int, [C.c_void_p, C.POINTER(obte_solve_opts), C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(obte_stats)]),
    "obte_umesh_destroy": (None, [C.c_void_p]),
    "obte_umesh_n_solid": (C.c_int, [C.c_void_p]),
    "obte_umesh_n_faces": (C.c_int, [C.c_void_p]),
    "obte_umesh_n_walls": (C.c_int, [C.c_void_p]),
    "obte_umesh_n_levels": (C.c_int, [C.c_void_p, C.c_int]),
}

_lib = None


def lib():
    """Load libobte.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2106_02764_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != OBTE_OK:
        raise ObteError(st, lib().obte_last_error().decode())


def _dptr(t):
    """Device pointer of a CUDA/HIP tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_opts(**kw):
    o = obte_solve_opts()
    lib().obte_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "waves_by_class":
            v = (C.c_int * 4)(*[int(x) for x in v])
        setattr(o, k, v)
    return o


def obte_mesh_create(ndim, n, L, solid, periodic, grad_axis=0, dT_ext=1.0):
    solid = np.ascontiguousarray(solid, dtype=np.uint8).ravel()
    d = obte_mesh_desc()
    d.ndim = ndim
    for a in range(3):
        d.n[a] = int(n[a]) if a < len(n) else 1
        d.L[a] = float(L[a]) if a < len(L) else 1.0
        d.periodic[a] = int(periodic[a]) if a < len(periodic) else 0
    d.grad_axis = grad_axis
    d.dT_ext = dT_ext
    d.solid = solid.ctypes.data_as(C.POINTER(C.c_uint8))
    h = C.c_void_p()
    _check(lib().obte_mesh_create(C.byref(d), C.byref(h)))
    return h


def obte_material_set(mesh, mfp, dirs, dir_w, kappa_m, modes=None, modes_exact=False):
    """modes = (F (n_modes, ndim), alpha (n_modes,)) or None; F may have 3
    columns for a 2D mesh (its in-plane part is used).  With a mode table
    kappa_m is ignored (may be None).  modes_exact: one system per mode, no
    interpolation (the grid arguments are then ignored)."""
    d = obte_material_desc()
    P = C.POINTER(C.c_double)
    keep = []
    if mfp is not None:
        mfp, dirs, dir_w = _f64(mfp), _f64(dirs), _f64(dir_w)
        d.n_mfp = len(mfp)
        d.mfp = mfp.ctypes.data_as(P)
        d.n_dir = len(dir_w)
        d.dirs = dirs.ctypes.data_as(P)
        d.dir_w = dir_w.ctypes.data_as(P)
    if kappa_m is not None:
        kappa_m = _f64(kappa_m)
        d.kappa_m = kappa_m.ctypes.data_as(P)
    if modes is not None:
        F, alpha = _f64(modes[0]), _f64(modes[1])
        keep = [F, alpha]
        d.n_modes = len(alpha)
        d.mode_dim = F.shape[1] if F.ndim == 2 else 0
        d.mode_F = F.ctypes.data_as(P)
        d.mode_alpha = alpha.ctypes.data_as(P)
        d.modes_exact = 1 if modes_exact else 0
    _check(lib().obte_material_set(mesh, C.byref(d)))
    del keep


def obte_kappa_modes(mesh):
    n = lib().obte_mesh_n_modes(mesh)
    out = np.zeros(max(n, 0))
    _check(lib().obte_kappa_modes(mesh, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def obte_system_counts(mesh):
    n = lib().obte_mesh_n_systems(mesh)
    its = np.zeros(max(n, 0), np.int64)
    sws = np.zeros(max(n, 0), np.int64)
    P = C.POINTER(C.c_longlong)
    _check(lib().obte_system_counts(mesh, its.ctypes.data_as(P), sws.ctypes.data_as(P)))
    return its, sws


def obte_workspace_size(mesh, opts):
    n = C.c_size_t()
    _check(lib().obte_workspace_size(mesh, C.byref(opts), C.byref(n)))
    return n.value


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def obte_workspace_size_batch(meshes, opts):
    n = C.c_size_t()
    arr = (C.c_void_p * len(meshes))(*[m.value for m in meshes])
    _check(lib().obte_workspace_size_batch(arr, len(meshes), C.byref(opts), C.byref(n)))
    return n.value


def obte_solve(mesh, opts, sigma, workspace, stream=None, T_L=None, J=None, raise_not_converged=False):
    st = obte_stats()
    rc = lib().obte_solve(mesh, C.byref(opts), _dptr(sigma), _dptr(workspace),
                          workspace.numel() * workspace.element_size(), _stream(stream),
                          _dptr(T_L), _dptr(J), C.byref(st))
    if rc != OBTE_OK and not (rc == OBTE_ERR_NOT_CONVERGED and not raise_not_converged):
        _check(rc)
    return st


def obte_solve_noalloc(mesh, opts, sigma, stream=None, T_L=None, J=None, raise_not_converged=False):
    st = obte_stats()
    rc = lib().obte_solve_noalloc(mesh, C.byref(opts), _dptr(sigma), _stream(stream), _dptr(T_L), _dptr(J),
                                  C.byref(st))
    if rc != OBTE_OK and not (rc == OBTE_ERR_NOT_CONVERGED and not raise_not_converged):
        _check(rc)
    return st


def obte_noalloc_scratch_bytes():
    return int(lib().obte_noalloc_scratch_bytes())


def obte_solve_batch(meshes, opts, sigmas, workspace, stream=None):
    n = len(meshes)
    arr = (C.c_void_p * n)(*[m.value for m in meshes])
    sg = (C.c_void_p * n)(*[(s.data_ptr() if s is not None else None) for s in sigmas])
    kap = (C.c_double * n)()
    stats = (obte_stats * n)()
    rc = lib().obte_solve_batch(arr, n, C.byref(opts), sg, _dptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream),
                                kap, stats)
    if rc not in (OBTE_OK, OBTE_ERR_NOT_CONVERGED):
        _check(rc)
    return list(kap), [stats[i] for i in range(n)]


def obte_kappa(mesh, n_mfp):
    k = C.c_double()
    per = (C.c_double * n_mfp)()
    _check(lib().obte_kappa(mesh, C.byref(k), per))
    return k.value, np.array(per[:])


def obte_adjoint(mesh, opts, sigma, workspace, grad, stream=None):
    st = obte_stats()
    _check(lib().obte_adjoint(mesh, C.byref(opts), _dptr(sigma), _dptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream(stream),
                              _dptr(grad), C.byref(st)))
    return st


def obte_upwind_apply(mesh, precision, transpose, sigma, sys_ids, x, y, stream=None):
    _check(lib().obte_upwind_apply(mesh, precision, int(transpose), _dptr(sigma), _dptr(sys_ids),
                                   int(sys_ids.numel()), _dptr(x), _dptr(y), _stream(stream)))


def obte_checkpoint_save(mesh, workspace, path):
    _check(lib().obte_checkpoint_save(mesh, _dptr(workspace), path.encode()))


def obte_checkpoint_load(mesh, workspace, path):
    _check(lib().obte_checkpoint_load(mesh, _dptr(workspace), path.encode()))


def obte_mesh_destroy(mesh):
    lib().obte_mesh_destroy(mesh)


def obte_mesh_counts(mesh):
    L = lib()
    return {"n_cells": L.obte_mesh_n_cells(mesh), "n_solid": L.obte_mesh_n_solid(mesh),
            "n_walls": L.obte_mesh_n_walls(mesh), "n_systems": L.obte_mesh_n_systems(mesh)}


# ---------------------------------------------------------------------------
# unstructured 2D meshes
# ---------------------------------------------------------------------------

def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.POINTER(np.ctypeslib.as_ctypes_type(dtype)))


def obte_umesh_create(nodes, cells, shifts, solid, L, grad_axis, dT):
    nodes_a, pn = _host(nodes, np.float64)
    cells_a, pc = _host(cells, np.int32)
    shifts_a, ps = _host(shifts, np.int32)
    solid_a, pso = _host(solid, np.uint8)
    n_cells, nv = cells_a.shape
    h = C.c_void_p()
    _check(lib().obte_umesh_create(pn, len(nodes_a), pc, ps, n_cells, nv, pso, float(L[0]), float(L[1]),
                                   int(grad_axis), float(dT), C.byref(h)))
    return h


def obte_umesh_material_set(mesh, mfp, dirs, dir_w, kappa_m):
    mfp_a, pm = _host(mfp, np.float64)
    dirs_a, pd = _host(np.asarray(dirs, float)[:, :2], np.float64)
    w_a, pw = _host(dir_w, np.float64)
    k_a, pk = _host(kappa_m, np.float64)
    _check(lib().obte_umesh_material_set(mesh, pm, len(mfp_a), pd, pw, len(w_a), pk))


def obte_umesh_fourier(mesh, tol, max_outer, cg_tol, T, stream=None, raise_not_converged=True):
    kF = C.c_double()
    it = C.c_int()
    st = lib().obte_umesh_fourier(mesh, float(tol), int(max_outer), float(cg_tol), _stream(stream), _dptr(T),
                                  C.byref(kF), C.byref(it))
    if st != OBTE_OK and (raise_not_converged or st != OBTE_ERR_NOT_CONVERGED):
        _check(st)
    return kF.value, it.value, st


def obte_umesh_solve(mesh, opts, sigma, T_L, stream=None, raise_not_converged=False):
    stats = obte_stats()
    st = lib().obte_umesh_solve(mesh, C.byref(opts), _dptr(sigma), _stream(stream), _dptr(T_L), C.byref(stats))
    if st != OBTE_OK and (raise_not_converged or st != OBTE_ERR_NOT_CONVERGED):
        _check(st)
    return stats
