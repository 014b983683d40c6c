/*
 * obte.h - C ABI of the MI355X (gfx950) aMFP-BTE hot-path library.
 *
 * The library solves the steady-state RTA phonon BTE with temperatures
 * interpolated onto vectorial mean-free-paths F_ml = Lambda_m s_l (the
 * anisotropic-MFP BTE of the OpenBTE paper, arXiv:2106.02764) on a structured
 * periodic finite-volume cell with diffuse pore walls, by the source iteration
 * of the paper's Eq. (iter) / Algorithm 1, starting from the Fourier first
 * guess of Eq. (fourier_iter).
 *
 * Conventions shared by every entry point
 *  - Units are SI: lengths in metres, conductivities in W/m/K, dT in K.
 *  - Cells are numbered x fastest: c = ix + nx (iy + ny iz).  2D meshes use
 *    nz = 1 and ndim = 2.
 *  - "host" pointers are read during the call only and may be freed after it;
 *    "device" pointers must stay valid until the work enqueued on `stream`
 *    has completed.  `stream` is a hipStream_t passed as void* (NULL = the
 *    legacy default stream).
 *  - Functions return an obte_status and never throw; obte_last_error()
 *    returns a thread-local description of the last failure.
 *  - Device memory larger than the small per-mesh tables is owned by the
 *    caller (workspace, sigma, outputs); the handle owns only its tables.
 */
#ifndef OBTE_H
#define OBTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct obte_mesh obte_mesh;     /* opaque handle */

typedef enum {
    OBTE_OK = 0,
    OBTE_ERR_ARG = -1,            /* invalid argument (checked on the host) */
    OBTE_ERR_HIP = -2,            /* a HIP runtime call failed */
    OBTE_ERR_STATE = -3,          /* call order violated (e.g. no material) */
    OBTE_ERR_NOT_CONVERGED = -4,  /* results written, tolerance not reached */
    OBTE_ERR_NUMERIC = -5,        /* non-finite value detected */
    OBTE_ERR_NOMEM = -6           /* workspace too small / host allocation */
} obte_status;

/* Geometry (paper: section "Geometry module"; Appendix A mesh terms).
 * solid: host, n[0]*n[1]*n[2] bytes, 1 = material, 0 = pore.  Faces between a
 * solid and a pore cell, and outer faces of non-periodic axes, are diffuse
 * thermalising walls.  grad_axis must be periodic; the image across its
 * periodic plane obeys T(x + L) = T(x) - dT_ext.
 * GPU-path limits: ndim 2 or 3; periodic[0] and periodic[1] may be 0 or 1,
 * periodic[2] must be 0 in 3D; n[0] <= 256; in 3D n[2] <= 128, and a solve
 * rejects meshes whose per-wave LDS rows (2 (1 + 2 ndim) reduction rows of ceil(n[0]/64) * 64
 * doubles plus, in 3D, n[2] rows in the compute type) exceed 64 KiB; grad_axis 0/1. */
typedef struct {
    int ndim;
    int n[3];
    double L[3];
    int periodic[3];
    int grad_axis;
    double dT_ext;
    const uint8_t* solid;
} obte_mesh_desc;

/* Material on the vectorial-MFP grid (paper: section "Material", Appendix A).
 * mfp: n_mfp MFP magnitudes Lambda_m (> 0); dirs: n_dir x ndim unit vectors
 * s_l (row-major), the set must be centrally symmetric; dir_w: quadrature
 * weights (> 0, sum 1); kappa_m: per-MFP bulk conductivity kernel (>= 0).
 * The library derives alpha_ml = kappa_m w_l / (Lambda_m^2 mu_g) with
 * mu_g = sum_l w_l s_{l,g}^2, the T_L weights D_ml = alpha / sum alpha, the flux
 * weights S_ml = alpha Lambda_m s_l and the outgoing wall weights per wall
 * orientation ReLu(S.n)/sum ReLu(S.n) (Appendix A, B_{lm'l'j}: the wall
 * temperature takes every system whose S leaves through the wall, which with
 * a mode table can include a system whose direction enters through it).
 * All pointers are host pointers. */
typedef struct {
    int n_mfp;
    const double* mfp;
    int n_dir;
    const double* dirs;
    const double* dir_w;
    const double* kappa_m;
    /* Optional mode table (Appendix A, aMFP interpolation): n_modes > 0
     * replaces kappa_m.  mode_F: n_modes x ndim vectorial MFPs F_mu (metres,
     * row-major); mode_alpha: n_modes weights alpha_mu = C/tau >= 0.  The
     * table must carry no net flux (sum alpha_mu F_mu = 0, e.g. every mode
     * with its reverse).  Each mode is spread over the grid with weights
     * c^mu_ml: linear in Lambda between the bracketing MFP nodes times linear
     * in angle between the bracketing directions (2D: azimuth, cyclic; 3D: a
     * tensor grid of polar bins x azimuths, polar angle clamped at the
     * outermost bins); beyond the MFP range the weight goes to the end node.
     * Then D_ml = sum_mu c D_mu, S_ml = sum_mu c alpha_mu F_mu, and the Fourier
     * conductivity per axis is sum_mu alpha_mu F_mu,a^2. */
    int n_modes;
    const double* mode_F;
    const double* mode_alpha;
    /* Components per row of mode_F: 0 or ndim, or 3 with a 2D mesh (section
     * Material, rta2DSym: the domain is uniform along z and each mode acts
     * through its in-plane part).  A mode whose (in-plane) F is zero keeps
     * T_mu = T_L and drops out: D is normalised over the moving modes and
     * its kappa_mu is 0. */
    int mode_dim;
    /* 1: no interpolation (Eq. iter3, the mode-resolved iteration): every
     * moving mode is its own system, transported along its own F_mu, with
     * D_mu = alpha_mu / sum alpha and S_mu = alpha_mu F_mu.  n_mfp, mfp, dirs,
     * dir_w and kappa_m are then ignored (may be 0 / NULL); the mesh has one
     * system per moving mode. */
    int modes_exact;
} obte_material_desc;

enum { OBTE_FP64 = 0, OBTE_FP32 = 1 };

/* Solver options.  precision OBTE_FP64: every sweep and Krylov vector in
 * double.  OBTE_FP32: sweeps and Krylov vectors in float, while T_L, T_w,
 * kappa and the convergence test accumulate in double.
 * outer_tol: stop when |kappa_n - kappa_{n-1}| <= outer_tol |kappa_n|
 * (Algorithm 1); 1 <= max_outer < 65536.  inner_tol: relative residual of the periodic-wrap Krylov
 * solve inside each (m,l) system; inner_rtol (0 = off) lets a pass stop
 * once the wrap residual it started from fell by that factor, and max_inner
 * caps the iterations per pass (either carries the rest of the wrap solve
 * into later passes).
 * The stop test also requires every relative wrap residual <= wrap_tol
 * (0 = max(inner_tol, 0.2 outer_tol)).  lag_wrap = 1 applies a pass's wrap
 * correction in the next pass instead of a correction sweep (the wrap
 * inflow is then lagged like T_L; the fixed point is unchanged).  init: 0 = Fourier first guess, 1 = resume
 * from the state left in the workspace by the previous call.
 * passes_per_graph: outer passes captured per HIP-graph replay (>= 1); the
 * host reads the done flags back once per replay, with the next replay of a
 * single-mesh solve already queued (passes after the stop exit at once, so
 * the pass count and results do not depend on it).  waves_per_group: systems that share
 * one workgroup's lockstep reduction (1..8, 0 = auto: 4 in 2D, 1 in 3D).  fourier_tol /
 * max_fourier: CG tolerance (relative residual) and iteration cap of the
 * Fourier first guess.  only_fourier: stop after the first guess.
 * keep_state: store the converged per-system solutions in the workspace (the
 * forward checkpoint obte_adjoint needs; n_systems * n_solid doubles).
 * timing: record HIP events on `stream` around every sweep, reduction and
 * Fourier launch and report their summed durations in obte_stats (the pass
 * kernels are then launched directly instead of through a HIP graph).
 * stop_rule: 0 = the relative change test above (Algorithm 1); 1 = the
 * estimated remaining error |kappa_n - kappa_{n-1}| rho/(1 - rho) <=
 * outer_tol |kappa_n| (from the 12th pass on), with the contraction rho the
 * largest of the last two ratios of successive changes and the mean ratio
 * over the last ten passes (clamped to [0, 0.995]); a slowly
 * contracting geometry then runs longer and a fast one stops earlier, so
 * outer_tol bounds the error of kappa rather than its last change.
 * accel: 0 = the plain source iteration of Algorithm 1 (each pass's T_L and
 * T_w are the next pass's inputs); 1..8 = Anderson mixing of depth accel on
 * the pair (T_L, T_w) (the adjoint: on (sum lambda, Phi)): the next inputs are
 * the combination of the last accel+1 iterates that minimises the linearised
 * residual.  Same fixed point, far fewer passes when the iteration contracts
 * slowly.  With accel > 0 the stop test also requires the estimated
 * relative error of the iterate, |G(x) - x| / (s |x|), <= outer_tol, where s
 * (>= 1e-3) estimates the smallest singular value of I - G' by the smallest
 * |dF_j| / |dX_j| over the mixing history.  An adjoint's accel may not exceed the depth of the forward solve
 * that sized the workspace. */
typedef struct {
    int precision;
    double outer_tol;
    int max_outer;
    double inner_tol;
    int max_inner;
    int init;
    int only_fourier;
    int passes_per_graph;
    int waves_per_group;
    double fourier_tol;
    int max_fourier;
    int keep_state;
    int lag_wrap;
    double inner_rtol;
    double wrap_tol;
    int timing;
    int stop_rule;
    int accel;
    /* Launch shape of the pass kernel (results do not depend on it; FP64 runs
     * are bitwise the same).  waves_by_class[c - 1]: systems per workgroup of
     * the launch over meshes with c = ceil(n[0] / 64) cells per lane (0..8,
     * 0 = waves_per_group; FP64 2D launches with c >= 3, and FP64 launches with
     * dispatch = 2, take at most 4: larger explicit values are OBTE_ERR_ARG).  dispatch: 0 = each geometry's work items longest
     * MFPs first (geometry by geometry), one launch per class; 1 = the
     * longest-MFP items of every geometry of a launch first; 2 (2D meshes;
     * 3D takes 1) = one persistent launch over the items of every class,
     * longest MFPs first over all geometries: each workgroup takes the next
     * item from a device-side queue until none is left (the workgroups have
     * as many waves as the widest class asks for). */
    int waves_by_class[4];
    int dispatch;
} obte_solve_opts;

typedef struct {
    int outer_iters;          /* passes executed */
    long long inner_iters;    /* BiCGSTAB iterations summed over systems/passes */
    long long sweeps;         /* upwind sweeps summed over systems/passes */
    int fourier_iters;
    double kappa;             /* kappa_cc: volume-averaged flux * L / dT */
    double kappa_face;        /* upwind flux through the hot contact plane */
    double kappa_fourier;
    double last_rel_change;
    double wrap_residual;     /* max relative wrap-row residual of the last pass */
    int status;
    int sweep_launches;       /* with opts.timing: pass-kernel launches timed */
    double sweep_ms;          /* summed duration of the sweep kernel launches */
    double reduce_ms;         /* summed duration of the per-pass reduction kernels */
    double fourier_ms;        /* duration of the Fourier first guess */
    /* Energy balance of the last pass (section Model: T_L is the temperature
     * that conserves energy, sum_ml alpha_ml sigma_i (T_iml - T_L,i) = 0):
     * max_i |sum_ml alpha_ml sigma_i (T_iml - T_L,i)| over the mean of
     * sum_ml alpha_ml |T_iml| per solid cell, with T the last pass's solutions
     * and T_L the lattice temperature they were solved with.  It vanishes at
     * the fixed point and measures how far the last pass is from it (forward
     * solves; 0 for an adjoint or without passes). */
    double energy_residual;
} obte_stats;

/* Fill opts with defaults (FP64, outer_tol 1e-8, ...). */
void obte_default_opts(obte_solve_opts* opts);

/* Create a mesh handle from a host description (validates, builds the face
 * classes on the host).  No device work. */
obte_status obte_mesh_create(const obte_mesh_desc* desc, obte_mesh** out);

/* Attach the material (computes the weights above on the host and uploads the
 * small tables to the current device).  Must precede obte_solve. */
obte_status obte_material_set(obte_mesh* mesh, const obte_material_desc* mat);

/* Bytes of device workspace obte_solve / obte_adjoint need for `opts`.  The
 * workspace holds every per-solve array, including the launch state (the
 * geometry views and the work-item list): a solve allocates no device
 * memory.  Each mesh keeps a small pinned host buffer for the flags and
 * results read back during its solves (taken at its first solve, grown when a
 * solve needs more, freed by obte_mesh_destroy). */
obte_status obte_workspace_size(const obte_mesh* mesh, const obte_solve_opts* opts,
                                size_t* bytes);

/* Bytes of device workspace obte_solve_batch needs for these meshes under
 * `opts` (the systems per workgroup of a batch follow its widest mesh, so this
 * can exceed the sum of the single-mesh sizes).  meshes: host array of n
 * handles with their material set. */
obte_status obte_workspace_size_batch(const obte_mesh* const* meshes, int n,
                                      const obte_solve_opts* opts, size_t* bytes);

/* Source iteration to convergence (paper Algorithm 1).
 * sigma_dev: device, n_cells doubles (pore entries ignored), NULL => 1.
 * workspace_dev: device, 256-byte aligned, workspace_bytes >= obte_workspace_size
 * (checked: a smaller workspace returns OBTE_ERR_NOMEM before any launch).
 * T_L_dev (nullable): device, n_cells doubles, receives the lattice
 * temperature with the solid-cell mean subtracted (0 in pores).
 * J_dev (nullable): device, n_cells*ndim doubles, receives the flux map
 * J_i = sum_ml S_ml T_iml (cell-major, component fastest).
 * stats: host.  Returns OBTE_ERR_NOT_CONVERGED (results written) when
 * max_outer passes did not reach outer_tol. */
obte_status obte_solve(obte_mesh* mesh, const obte_solve_opts* opts, const double* sigma_dev,
                       void* workspace_dev, size_t workspace_bytes, void* stream, double* T_L_dev,
                       double* J_dev, obte_stats* stats);

/* obte_solve for callers that cannot allocate device or pinned host memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  The workspace is a file-scope device array of
 * obte_noalloc_scratch_bytes() bytes (32 MiB) that the library holds on
 * every device it runs on until the process ends; the call takes the copy
 * of the current device (which must hold the mesh tables).  Arguments and
 * results as obte_solve, with: init = 0 (every call starts from the Fourier
 * guess), keep_state = 0 and timing = 0 (OBTE_ERR_ARG otherwise); a mesh
 * whose workspace (obte_workspace_size) exceeds the array returns
 * OBTE_ERR_NOMEM before any device work.  The call launches every kernel
 * directly on `stream` (no graph capture, no events, no pinned staging) and
 * allocates nothing; it synchronizes `stream` to read the results back.
 * All calls on one device share its array, which keeps the last call's
 * contents: calls that overlap on one device (other host threads, other
 * streams) race and must be serialised by the caller. */
obte_status obte_solve_noalloc(obte_mesh* mesh, const obte_solve_opts* opts, const double* sigma_dev,
                               void* stream, double* T_L_dev, double* J_dev, obte_stats* stats);
/* Bytes of the per-device array obte_solve_noalloc works in. */
size_t obte_noalloc_scratch_bytes(void);

/* Many independent geometries in one launch per pass (one per row-width
 * class: ceil(nx / 64) cells per lane).  meshes[i]
 * and sigma_dev[i] (nullable entries) as above; one workspace holds all, of
 * at least obte_workspace_size_batch bytes (OBTE_ERR_NOMEM otherwise); all
 * meshes must share the number of MFPs unless waves_per_group is set.  kappa_out: host, n doubles (kappa_cc).  stats: host,
 * n entries. */
obte_status obte_solve_batch(obte_mesh* const* meshes, int n, const obte_solve_opts* opts,
                             const double* const* sigma_dev, void* workspace_dev,
                             size_t workspace_bytes, void* stream, double* kappa_out,
                             obte_stats* stats);

/* Effective conductivity of the last solve (paper Eq. (keff): kappa_eff =
 * -(L/dT) times the heat flux through the cell's cross-section), in the
 * cell-centred form kappa_cc = L / (dT N_cells) sum_i sum_ml S_ml,g T_iml:
 * the volume-averaged flux J of section Model along the gradient axis g,
 * with N_cells counting pores (they carry no flux).  kappa_eff: host, one
 * double.  kappa_per_mfp (nullable): host, n_mfp doubles, the same sum split
 * over the MFPs.  OBTE_ERR_ARG for a NULL mesh, OBTE_ERR_STATE before the
 * first completed solve on it; the values are those the last obte_solve /
 * obte_solve_batch member wrote, also when it returned
 * OBTE_ERR_NOT_CONVERGED. */
obte_status obte_kappa(const obte_mesh* mesh, double* kappa_eff, double* kappa_per_mfp);

/* Per-system work of the last obte_solve / obte_solve_batch member on this
 * mesh, summed over its passes (Appendix A, Eq. (iter2): one (m,l) system is
 * one upwind solve per pass): inner_iters, the wrap-row BiCGSTAB iterations;
 * sweeps, the upwind sweeps (one per pass plus two per iteration, plus the
 * correction sweep without lag_wrap).  Host arrays of obte_mesh_n_systems()
 * entries in system order sys = m * n_dir + l; either may be NULL.
 * OBTE_ERR_STATE before a solve that ran passes. */
obte_status obte_system_counts(const obte_mesh* mesh, long long* inner_iters, long long* sweeps);

/* Mode-resolved conductivity of the last solve (paper Eq. mode-resolved, in
 * the cell-centred form of kappa_cc): kappa_mu = L S_mu,g / (dT N_cells)
 * sum_ml c^mu_ml sum_i (T_iml - <T_L>), which sums to kappa_cc over the
 * modes.  The periodic problem fixes the temperatures only up to a common
 * constant, which kappa_cc does not see but a single mode's share does; the
 * shares are taken relative to the mean lattice temperature <T_L> over the
 * solid cells (so they do not depend on that constant).  With a mode table
 * the per-MFP split of obte_kappa does depend on it.
 * kappa_mode: host, n_modes doubles.  OBTE_ERR_STATE without a mode table or
 * a completed solve. */
obte_status obte_kappa_modes(const obte_mesh* mesh, double* kappa_mode);

/* Adjoint gradient d kappa_cc / d sigma_i (derived from Appendix A,
 * Eq. (iter2)): M^T lambda = k by the transposed source iteration, then
 * d kappa / d sigma_i = -sum_ml lambda_iml (T_iml - T_L,i).  Requires a
 * converged obte_solve with keep_state = 1 on the same mesh, sigma pointer,
 * precision and workspace (else OBTE_ERR_STATE).  stats->kappa receives p^T lambda, which equals kappa_cc at
 * convergence.  dkappa_dsigma_dev: device, n_cells doubles, 0 in pores. */
obte_status obte_adjoint(obte_mesh* mesh, const obte_solve_opts* opts, const double* sigma_dev,
                         void* workspace_dev, size_t workspace_bytes, void* stream,
                         double* dkappa_dsigma_dev, obte_stats* stats);

/* Matrix-free upwind apply of one (m,l) system, y = (sigma + Lambda_m A_l) x
 * (transpose = 1: sigma + Lambda_m A_l^T), for n_sys systems at once.
 * x, y: device, n_sys * n_cells values of the precision (0 = double,
 * 1 = float), system-major; sys_ids: device int32 (n_sys) of m * n_dir + l.
 * Pore entries of y are written 0.  Used for the outer residual and by the
 * tests; paper Appendix A, Eq. (iter2) left-hand side. */
obte_status obte_upwind_apply(const obte_mesh* mesh, int precision, int transpose,
                              const double* sigma_dev, const int* sys_ids_dev, int n_sys,
                              const void* x_dev, void* y_dev, void* stream);

/* Save / restore the outer-loop state (pass count, kappa history, T_L, T_w
 * and the wrap inflow vectors) of the last solve to a host file.  Save checks
 * its arguments before it opens the file (a rejected call leaves the file
 * untouched) and closes it on every path; OBTE_ERR_HIP if a read-back or a
 * write fails, OBTE_ERR_ARG if the file cannot be opened or does not match.  Loading
 * needs a mesh with the same geometry and material; a following obte_solve
 * with init = 1 and the same precision, waves_per_group and keep_state
 * continues the iteration exactly where the saved run stopped. */
obte_status obte_checkpoint_save(const obte_mesh* mesh, const void* workspace_dev,
                                 const char* path);
obte_status obte_checkpoint_load(obte_mesh* mesh, void* workspace_dev, const char* path);

const char* obte_last_error(void);
void obte_mesh_destroy(obte_mesh* mesh);

/* Mesh/material queries (host). */
int obte_mesh_n_cells(const obte_mesh* mesh);
int obte_mesh_n_solid(const obte_mesh* mesh);
int obte_mesh_n_walls(const obte_mesh* mesh);
int obte_mesh_n_systems(const obte_mesh* mesh);
int obte_mesh_n_modes(const obte_mesh* mesh);

/* ---------------------------------------------------------------------
 * Unstructured 2D meshes (paper: section Geometry module, which meshes the
 * cell with unstructured polygons; Appendix A, where the mesh enters only
 * through the face vectors R_ij = A_ij n_ij / V_i; Appendix B, Eqs. (grad)
 * to (final2), the heat-conduction first guess with the non-orthogonal
 * secondary flux treated explicitly and least-squares cell gradients).
 * The cell is periodic along both axes; pore cells are removed and their
 * faces become diffuse walls.  FP64 throughout; the library owns the solve
 * buffers (taken at obte_umesh_material_set, freed by obte_umesh_destroy).
 * ------------------------------------------------------------------- */
typedef struct obte_umesh obte_umesh;   /* opaque handle */

/* Build the face lists and geometry on the host and upload them to the
 * current device.
 * nodes:  host, n_nodes x 2 doubles (metres);
 * cells:  host int32, n_cells x nv node ids (nv = 3 or 4), counter-clockwise;
 * shifts: host int32, n_cells x nv x 2: corner k of cell c lies at
 *         nodes[cells[c][k]] + shifts[c][k] * (Lx, Ly) (periodic images);
 * solid:  host uint8, n_cells (0 = pore).
 * Every edge must be shared by exactly two cells (OBTE_ERR_ARG otherwise,
 * and for clockwise or degenerate cells, sizes out of range or no solid
 * cell).  The applied difference dT > 0 is along grad_axis (0 = x, 1 = y),
 * with T(x + L) = T(x) - dT across the periodic plane.  Limits: at most
 * 8192 solid cells (a system's solution lives in one workgroup's LDS). */
obte_status obte_umesh_create(const double* nodes, int n_nodes, const int* cells, const int* shifts,
                              int n_cells, int nv, const unsigned char* solid, double Lx, double Ly,
                              int grad_axis, double dT, obte_umesh** out);

/* Material weights on the vectorial-MFP grid (section Model, Appendix A):
 * mfp (n_mfp), in-plane unit directions dirs (n_dir x 2), weights dir_w
 * (summing to 1), per-MFP conductivity kappa_m; all host.  Builds the
 * per-direction sweep order: the cells sorted into upwind levels with the
 * periodic faces cut (OBTE_ERR_ARG if the upwind graph of some direction has
 * a cycle, which convex cells do not produce). */
obte_status obte_umesh_material_set(obte_umesh* mesh, const double* mfp, int n_mfp, const double* dirs,
                                    const double* dir_w, int n_dir, const double* kappa_m);

/* Heat-conduction first guess, Eq. (final2): outer iterations of
 * A T^(n) = S T^(n-1) + P until max|T^(n) - T^(n-1)| <= tol max|T^(n)|
 * (at most max_outer), each solved by conjugate gradients to a relative
 * residual of cg_tol.  T_dev: device, n_cells doubles (mean zero over the
 * solid cells, 0 in pores); kappa_F: host, the face flux across the
 * periodic plane times L / (dT A_perp); outer_iters: host, may be NULL.
 * OBTE_ERR_NOT_CONVERGED if max_outer was reached (results written). */
obte_status obte_umesh_fourier(obte_umesh* mesh, double tol, int max_outer, double cg_tol, void* stream,
                               double* T_dev, double* kappa_F, int* outer_iters);

/* Algorithm 1 on the unstructured mesh: the Fourier first guess (to
 * opts->fourier_tol), then passes until |kappa_n - kappa_{n-1}| <=
 * opts->outer_tol |kappa_n| or opts->max_outer passes.  Each pass solves
 * every (m, l) system exactly up to its periodic-face coupling, which
 * BiCGSTAB solves to opts->inner_tol (at most opts->max_inner iterations),
 * or, with opts->inner_rtol > 0, until its residual fell by that factor (the
 * rest carries into the next pass; the stop test then also requires every
 * relative wrap residual <= wrap_tol, as for obte_solve).
 * Only precision = OBTE_FP64, init = 0 and accel = 0 are accepted.
 * sigma_dev: device, n_cells relaxation multipliers, or NULL for 1.
 * T_L_dev: device, n_cells doubles (mean zero over solid cells) or NULL.
 * stats: kappa (kappa_cc), kappa_face, kappa_fourier, outer_iters,
 * inner_iters, wrap_residual, last_rel_change, status. */
obte_status obte_umesh_solve(obte_umesh* mesh, const obte_solve_opts* opts, const double* sigma_dev,
                             void* stream, double* T_L_dev, obte_stats* stats);

void obte_umesh_destroy(obte_umesh* mesh);
int obte_umesh_n_solid(const obte_umesh* mesh);
int obte_umesh_n_faces(const obte_umesh* mesh);   /* interior faces between solid cells */
int obte_umesh_n_walls(const obte_umesh* mesh);
int obte_umesh_n_levels(const obte_umesh* mesh, int direction);  /* upwind levels of a direction */

#ifdef __cplusplus
}
#endif
#endif /* OBTE_H */
