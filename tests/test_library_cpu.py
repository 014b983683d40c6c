"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects bad arguments on the host (no device work)."""
import ctypes as C

import numpy as np
import pytest

from tests._lib import ensure_built, header_functions
from inputs import gen


@pytest.fixture(scope="module")
def L():
    ensure_built()
    from paper_2106_02764_amd import obte
    return obte


def test_exports_every_header_symbol(L):
    lib = L.lib()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(L.EXPORTS), set(names) - set(L.EXPORTS)


def test_default_opts(L):
    o = L.default_opts()
    assert o.precision == L.OBTE_FP64 and o.max_outer > 0 and o.inner_tol > 0
    assert o.keep_state == 0 and o.stop_rule == 0 and o.timing == 0 and o.accel == 0
    assert list(o.waves_by_class) == [0, 0, 0, 0] and o.dispatch == 0


def _desc_ok(**kw):
    base = dict(ndim=2, n=(8, 6, 1), L=(1e-7, 1e-7, 1.0), solid=np.ones(48, np.uint8),
                periodic=(1, 1, 0), grad_axis=0, dT_ext=1.0)
    base.update(kw)
    return base


@pytest.mark.parametrize("bad", [
    dict(ndim=4), dict(n=(1, 6, 1)), dict(L=(0.0, 1e-7, 1.0)), dict(periodic=(0, 1, 0)),
    dict(grad_axis=2), dict(solid=np.zeros(48, np.uint8)), dict(solid=np.full(48, 2, np.uint8)),
    dict(n=(300, 2, 1), solid=np.ones(600, np.uint8)), dict(dT_ext=0.0),
    dict(ndim=3, n=(4, 4, 130), solid=np.ones(2080, np.uint8)),
    dict(ndim=3, n=(4, 4, 2), periodic=(1, 1, 1), solid=np.ones(32, np.uint8)),
])
def test_mesh_create_rejects(L, bad):
    d = _desc_ok(**bad)
    with pytest.raises(L.ObteError) as e:
        L.obte_mesh_create(d["ndim"], d["n"], d["L"], d["solid"], d["periodic"], d["grad_axis"], d["dT_ext"])
    assert e.value.status == L.OBTE_ERR_ARG


@pytest.mark.parametrize("w", [gen.config1(), gen.small_3d(5, 4, 3, solid=None),
                               gen.small_2d(7, 5, solid=gen.stripe_mask(7, 5, 3))])
def test_mesh_counts_match_face_classes(L, w):
    from oracle.mesh import Mesh
    h = L.obte_mesh_create(w.ndim, w.n, w.L, w.solid, w.periodic, w.grad_axis, w.dT)
    c = L.obte_mesh_counts(h)
    me = Mesh(w.n, w.L, w.solid, w.periodic, w.grad_axis, w.dT, ndim=w.ndim)
    assert c["n_cells"] == me.n_cells and c["n_solid"] == me.n_solid and c["n_walls"] == me.n_walls
    L.obte_mesh_destroy(h)


@pytest.mark.parametrize("bad", ["norm", "weights", "asym", "mfp", "kappa"])
def test_material_set_rejects_on_host(L, bad):
    w = gen.small_2d(8, 6, n_dir=8, n_mfp=3)
    h = L.obte_mesh_create(w.ndim, w.n, w.L, w.solid, w.periodic, w.grad_axis, w.dT)
    mfp, dirs, dw, km = w.mfp.copy(), w.dirs.copy(), w.dir_w.copy(), w.kappa_m.copy()
    if bad == "norm":
        dirs[0] *= 1.1
    elif bad == "weights":
        dw[0] *= 2
    elif bad == "asym":
        dirs = np.array([[1.0, 0.0]] * 8)
    elif bad == "mfp":
        mfp[1] = -1.0
    else:
        km[0] = np.nan
    with pytest.raises(L.ObteError) as e:
        L.obte_material_set(h, mfp, dirs, dw, km)
    assert e.value.status == L.OBTE_ERR_ARG
    L.obte_mesh_destroy(h)


@pytest.mark.parametrize("bad", ["netflux", "alpha", "all_static", "dup_nodes", "nan", "dim"])
def test_mode_table_rejects_on_host(L, bad):
    """Mode-table validation happens before any device call."""
    w = gen.with_modes(gen.small_2d(8, 6, n_dir=8, n_mfp=3), 20, 5)
    h = L.obte_mesh_create(w.ndim, w.n, w.L, w.solid, w.periodic, w.grad_axis, w.dT)
    assert L.lib().obte_mesh_n_modes(h) == 0
    F, alpha = w.modes[0].copy(), w.modes[1].copy()
    mfp = w.mfp.copy()
    if bad == "netflux":
        F, alpha = F[1:], alpha[1:]          # drop one of a mirrored pair
    elif bad == "alpha":
        alpha[3] = -1.0
    elif bad == "all_static":
        F[:] = 0.0                           # no mode moves in the plane
    elif bad == "dim":
        F = np.concatenate([F, F[:, :1]], axis=1)[:, :1]   # one column in a 2D domain
    elif bad == "dup_nodes":
        mfp[1] = mfp[0]
    else:
        F[4, 0] = np.nan
    with pytest.raises(L.ObteError) as e:
        L.obte_material_set(h, mfp, w.dirs, w.dir_w, None, modes=(F, alpha))
    assert e.value.status == L.OBTE_ERR_ARG
    out = np.zeros(4)
    assert L.lib().obte_kappa_modes(h, out.ctypes.data_as(C.POINTER(C.c_double))) == L.OBTE_ERR_STATE
    L.obte_mesh_destroy(h)


@pytest.mark.parametrize("bad", ["netflux", "all_static", "no_gradient", "dim"])
def test_exact_modes_reject_on_host(L, bad):
    """The mode-resolved material (no interpolation) checks its table before
    any device call; the grid arguments may be absent."""
    w = gen.with_modes(gen.small_2d(8, 6, n_dir=8, n_mfp=3), 20, 5)
    h = L.obte_mesh_create(w.ndim, w.n, w.L, w.solid, w.periodic, w.grad_axis, w.dT)
    F, alpha = w.modes[0].copy(), w.modes[1].copy()
    if bad == "netflux":
        F, alpha = F[1:], alpha[1:]
    elif bad == "all_static":
        F[:] = 0.0
    elif bad == "no_gradient":
        F[:, 0] = 0.0                        # nothing moves along x
    else:
        F = F[:, :1]
    with pytest.raises(L.ObteError) as e:
        L.obte_material_set(h, None, None, None, None, modes=(F, alpha), modes_exact=True)
    assert e.value.status == L.OBTE_ERR_ARG
    L.obte_mesh_destroy(h)


def test_solve_state_errors_on_host(L):
    w = gen.small_2d(8, 6)
    h = L.obte_mesh_create(w.ndim, w.n, w.L, w.solid, w.periodic, w.grad_axis, w.dT)
    o = L.default_opts()
    st = L.obte_stats()
    lib = L.lib()
    # no material yet -> state error before any device access
    rc = lib.obte_solve(h, C.byref(o), None, C.c_void_p(4096), 1 << 20, None, None, None, C.byref(st))
    assert rc == L.OBTE_ERR_STATE
    o.precision = 7
    rc = lib.obte_solve(h, C.byref(o), None, C.c_void_p(4096), 1 << 20, None, None, None, C.byref(st))
    assert rc == L.OBTE_ERR_ARG
    o = L.default_opts()
    rc = lib.obte_solve(h, C.byref(o), None, None, 0, None, None, None, C.byref(st))
    assert rc == L.OBTE_ERR_ARG
    k = C.c_double()
    assert lib.obte_kappa(h, C.byref(k), None) == L.OBTE_ERR_STATE
    L.obte_mesh_destroy(h)


@pytest.mark.parametrize("field,value", [
    ("precision", 2), ("outer_tol", -1.0), ("max_outer", 0), ("max_outer", 65536),
    ("inner_tol", 0.0), ("max_inner", -1), ("waves_per_group", 9), ("passes_per_graph", -1),
    ("fourier_tol", 0.0), ("init", 2), ("lag_wrap", 2), ("wrap_tol", -1.0),
    ("inner_rtol", 1.0), ("stop_rule", 2), ("accel", -1), ("accel", 9), ("dispatch", -1), ("dispatch", 3)])
def test_options_rejected_on_host(L, field, value):
    w = gen.small_2d(8, 6)
    h = L.obte_mesh_create(w.ndim, w.n, w.L, w.solid, w.periodic, w.grad_axis, w.dT)
    # options are checked before anything else (no material, no device needed)
    with pytest.raises(L.ObteError) as e:
        L.obte_workspace_size(h, L.default_opts())
    assert e.value.status == L.OBTE_ERR_STATE
    with pytest.raises(L.ObteError) as e:
        L.obte_workspace_size(h, L.default_opts(**{field: value}))
    assert e.value.status == L.OBTE_ERR_ARG
    L.obte_mesh_destroy(h)


# ---- unstructured meshes: host-side construction (no device work before
# the material is set)

def _umesh(L, w):
    return L.obte_umesh_create(w.nodes, w.cells, w.shifts, w.solid, w.L, w.grad_axis, w.dT)


@pytest.mark.parametrize("tri", [False, True])
def test_umesh_counts_match_oracle(L, tri):
    from oracle.umesh import UMesh
    w = gen.unstructured_2d(9, 7, amp=0.3, tri=tri, seed=3, pores=[((40e-9, 55e-9), 22e-9)])
    h = _umesh(L, w)
    try:
        um = UMesh(w.L, w.nodes, w.cells, w.shifts, w.solid, w.grad_axis, w.dT)
        lib = L.lib()
        assert lib.obte_umesh_n_solid(h) == um.n_solid
        assert lib.obte_umesh_n_faces(h) == um.n_faces
        assert lib.obte_umesh_n_walls(h) == um.n_walls
        assert lib.obte_umesh_n_levels(h, 0) == -1          # no material yet
    finally:
        L.lib().obte_umesh_destroy(h)


def test_umesh_create_rejects(L):
    w = gen.unstructured_2d(6, 5, amp=0.2, tri=True, seed=1)
    bad = []
    cw, cws = w.cells.copy(), w.shifts.copy()
    cw[3], cws[3] = cw[3][::-1], cws[3][::-1]                # one clockwise cell
    bad.append(dict(cells=cw, shifts=cws))
    gone = np.delete(w.cells, 7, axis=0)                     # a hole: unmatched edges
    bad.append(dict(cells=gone, shifts=np.delete(w.shifts, 7, axis=0), solid=np.delete(w.solid, 7)))
    bad.append(dict(solid=np.zeros_like(w.solid)))
    oob = w.cells.copy()
    oob[0, 0] = len(w.nodes)
    bad.append(dict(cells=oob))
    for b in bad:
        args = dict(nodes=w.nodes, cells=w.cells, shifts=w.shifts, solid=w.solid)
        args.update(b)
        with pytest.raises(L.ObteError) as e:
            L.obte_umesh_create(args["nodes"], args["cells"], args["shifts"], args["solid"], w.L, 0, 1.0)
        assert e.value.status == L.OBTE_ERR_ARG
    for Lx, ga, dT in ((0.0, 0, 1.0), (1e-7, 2, 1.0), (1e-7, 0, 0.0)):
        with pytest.raises(L.ObteError) as e:
            L.obte_umesh_create(w.nodes, w.cells, w.shifts, w.solid, (Lx, 1e-7), ga, dT)
        assert e.value.status == L.OBTE_ERR_ARG
