// Internal types shared by the host driver and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Face classes, two bits per face, face index f = 2 * axis + side
// (side 0 = '-' face, 1 = '+' face); bit 0 of the cell word = solid.
#define FC_INTERIOR 0   // solid neighbour (with periodic wrap), no jump
#define FC_WALL 1       // pore neighbour or outer face of a non-periodic axis
#define FC_JUMP_P 2     // solid neighbour across the periodic plane, image hotter by dT
#define FC_JUMP_M 3     // solid neighbour across the periodic plane, image colder by dT

__host__ __device__ inline int fc_solid(uint16_t w) { return w & 1; }
__host__ __device__ inline int fc_class(uint16_t w, int f) { return (w >> (1 + 2 * f)) & 3; }

enum { CTRL_DONE = 0, CTRL_PASS = 1, CTRL_CONVERGED = 2, CTRL_NONFINITE = 3, CTRL_N = 8 };

// wrap-plane vectors per system kept in the workspace by the 3D pass kernel
constexpr int KRY3_VECS = 11;

// Per-geometry view used by every kernel: static tables (library-owned) plus
// the per-solve workspace carve (caller-owned).
struct GeomDev {
    int nx, ny, nz, ndim, nf, ncells, nwalls, nwrap;
    int nsolid;                  // solid cells: the length of one system's stored solution
    int xs;                      // stride of one system's row in X and Tstore: nsolid rounded up
                                 // to 64 values, so the reductions' 64-cell strips start on lines
    int periodic[3];
    int grad_axis;
    double h[3], L[3], dT;
    int n_mfp, n_dir, n_sys;
    int n_perp;                  // ncells / n[grad_axis]
    // ---- static tables
    const uint16_t* fc;          // ncells
    const int* sidx;             // ncells: solid index of the cell (cells in order), -1 in pores
    const int* scell;            // nsolid: cell of each solid index
    const int* wall_cell;        // nwalls
    const int* wall_face;        // nwalls: face index 2a+side of the owning cell
    const int* wall_idx;         // ncells * nf: wall index of (cell, face), -1 if not a wall
    const double* mfp;           // n_mfp
    const double* dirs;          // n_dir * 3 (z = 0 in 2D)
    const double* Dw;            // n_sys: T_L weights D_ml
    const double* S;             // n_sys * 3: flux weights S_ml
    const double* wout;          // nf * n_sys: outgoing wall weights per face orientation
    const double* kappa_axis;    // 3
    // ---- workspace
    double* sigma;               // ncells (1 in pores)
    float* sigma_f;              // ncells
    double* sT;                  // 2 * ncells: sigma * T_L of the pass input (double buffered)
    double* Tw;                  // 2 * nwalls: wall temperatures (double buffered)
    double* T_L;                 // ncells: latest lattice temperature
    void* U;                     // n_sys * nwrap (compute precision): wrap inflow vectors
    void* kry;                   // 3D: n_sys * 11 * nwrap (compute precision): wrap-plane Krylov vectors
    void* X;                     // n_sys * xs (compute precision): each system's solution of
                                 // the pass (forward T, adjoint lambda) on the solid cells
    double* ksys;                // n_sys: kappa_cc contribution of each system
    double* kfsys;               // n_sys: kappa_face contribution
    long long* iters;            // n_sys: accumulated BiCGSTAB iterations
    long long* sweeps;           // n_sys: accumulated sweeps
    double* hist;                // max_outer
    double* hist_face;           // max_outer
    int* ctrl;                   // CTRL_N ints
    double* fx;                  // Fourier CG vectors: 8 * ncells, partials and scalars
    double* fscal;               // scalars: [0] kappa_F, [1] CG iterations, [2] CG residual,
                                 // [3] mixing error estimate, [4] energy residual of the last pass,
                                 // [5] smallest sigma over the solid cells
    double* Tstore;              // n_sys * xs (adjoint forward state) or null
    double* lam_psi;             // adjoint: 2 * ncells (double buffered Psi)
    double* lam_phi;             // adjoint: 2 * nwalls (double buffered Phi)
    double* gradient;            // adjoint: ncells
    double* bnd;                 // 4 * nf * ncells: inflow boundary value per (face, cell);
                                 // forward buffers 0/1, adjoint buffers 2/3 (double buffered)
    double* wres;                // n_sys: relative wrap-row residual after this pass's solve
    double* wres_hist;           // max_outer: max over systems per pass
    // ---- the outer fixed point x = (cell field, wall values), n_aa = ncells + nwalls:
    // forward (T_L, T_w), adjoint (sum_ml lambda, Phi)
    int n_aa;
    double* ax;                  // n_aa: the iterate the next pass consumes
    // Anderson mixing (aa_m > 0 only)
    int aa_m;                    // history depth
    double* ag;                  // n_aa: G(x) of this pass
    double* axp;                 // n_aa: previous iterate
    double* afp;                 // n_aa: previous residual G(x) - x
    double* adX;                 // aa_m * n_aa: iterate differences (ring)
    double* adF;                 // aa_m * n_aa: residual differences (ring)
    double* agram;               // aa_m * aa_m Gram matrix of the adF columns, then aa_m |adX_j|^2
    double* apart;               // per-block partial sums of the mixing kernels
    double* kraw;                // n_sys: sum over cells of each system's last solution
    // 1 with a mode table: the outer iterates are re-centred every pass
    // (ax[n_aa] holds the shift between the two gauge kernels)
    int gauge;
    int* actl;                   // 2 x 4 (by pass parity): stored columns, ring head, previous pass valid
    // ---- 2D sweep inputs of the pass in each sweep orientation's order,
    // written by the pack kernel before the pass's sweeps.  Quadrant
    // q = [s_x < 0] + 2 [s_y < 0]; entry q * ncells + r * nx + p is the cell
    // at row r (y-upwind order) and position p (x-upwind order).
    void* qrec;                  // 4 * ncells records {sb, bx, by, meta} of 4 compute-type words
                                 // (meta: byte 0 x inflow open, 1 y inflow open, 2 kappa_face
                                 // plane cell, 3 solid).  3D: the pass's sources (ncells) and
                                 // inflow tables (nf * ncells) in the compute type
    uint32_t* qoff;              // 4 * ncells: byte offset of the cell's stored value, QOFF_NONE in pores
    void* qsg;                   // 4 * ncells: sigma in the compute type
    void* qalt;                  // adjoint passes: 4 * ncells pairs {bx, by} of the outflow faces
                                 // (with a mode table S may leave against the sweep direction)
    int qnk[4];                  // per quadrant: cells flagged as kappa_face plane cells
};

// Store offset of a pore cell: past any stored array, also when doubled for
// the FP64 copy of an FP32 solution (raw buffer stores there are dropped).
constexpr uint32_t QOFF_NONE = 0x7FFFFFF0u;

constexpr int AA_MAX = 8;

struct Item {
    int geom;    // index into the geometry array
    int l;       // direction
    int m0;      // first MFP of the group
    int nm;      // MFPs in the group (<= waves per group)
};

struct PassParams {
    double inner_tol;
    int max_inner;
    int mode;          // 0 = full pass, 1 = replay the last pass's final sweep only (J / store)
    int store_T;       // write the final x of every system to Tstore
    int adjoint;       // 1 = transposed system with adjoint sources
    int max_outer;
    double outer_tol;
    int lag_wrap;      // 1 = apply this pass's wrap correction in the next pass
    double inner_rtol; // per-pass wrap solve stops once the residual fell by this factor
    double wrap_tol;   // stop test: every relative wrap residual <= wrap_tol
    int stop_rule;     // 0 = relative change, 1 = change * rho / (1 - rho)
    int sigma1;        // 1 when no geometry of the launch has a sigma field (sigma = 1)
};

// kernel launchers (kernels.hip)
// Fourier CG: init (x = 0, r = p = b), per iteration (parity = iteration & 1)
// the direction / A p kernel and the x, r update, the count of geometries
// still iterating, and the epilogue (mean-free T_F, pass inputs, kappa_F).
// fx must hold fourier_scratch_doubles(ncells) doubles.
constexpr size_t fourier_scratch_doubles(size_t ncells) { return 8 * ncells + 4 * 256 + 16; }
hipError_t launch_fourier_init(const GeomDev* geoms_dev, int n_geoms, int max_cells, hipStream_t st);
hipError_t launch_fourier_iter(const GeomDev* geoms_dev, int n_geoms, int max_cells, int parity, double tol,
                               int max_iter, hipStream_t st);
hipError_t launch_fourier_pending(const GeomDev* geoms_dev, int n_geoms, int* pending_dev, hipStream_t st);
hipError_t launch_fourier_finish(const GeomDev* geoms_dev, int n_geoms, int max_cells, hipStream_t st);
hipError_t launch_sweep_pass(int precision, int cpl, int nz, const GeomDev* geoms_dev,
                             const Item* items_dev, int n_items, int waves, PassParams pp,
                             size_t lds_bytes, hipStream_t st, int full);
// 2D: every item of a batch in one persistent launch; the groups take items
// from the device counter *queue, which launch_pack_rows sets to 0.
hipError_t launch_sweep_queue(int precision, const GeomDev* geoms_dev, const Item* items_dev, int n_items,
                              int waves, PassParams pp, hipStream_t st, int* queue);
// 2D: the pass inputs in the quadrant layout (GeomDev::qrec, qoff, qsg) of
// every geometry, read from the buffers the pass's sweeps consume; a non-null
// queue (the persistent launch's item counter) is set to 0.
hipError_t launch_pack_rows(int precision, const GeomDev* geoms_dev, int n_geoms, int max_cells, PassParams pp,
                            hipStream_t st, int* queue);
// 3D: the pass's sources and inflow tables in the compute type (GeomDev::qrec).
hipError_t launch_pack3(int precision, const GeomDev* geoms_dev, int n_geoms, int max_cells, PassParams pp,
                        hipStream_t st);
hipError_t launch_reduce_pass(int precision, const GeomDev* geoms_dev, int n_geoms, int max_solid,
                              PassParams pp, hipStream_t st);
// Energy balance of the last pass of one geometry (forward solve):
// max_i |sigma_i T_L,i - sigma_i T_L^in_i| / (sum_i sum_ml D_ml |T_iml| / N_solid) into
// fscal[4], with T_L = sum_ml D_ml T_iml of the stored solutions.  Scratch:
// energy_scratch_doubles(nsolid) doubles in the Fourier CG region.
// row stride of the per-system stores X and Tstore
constexpr size_t x_stride(size_t nsolid) { return (nsolid + 63) / 64 * 64; }
constexpr size_t energy_scratch_doubles(size_t nsolid) { return 2 * ((nsolid + 63) / 64); }
hipError_t launch_energy(const GeomDev* geom_dev, int precision, int nsolid, hipStream_t st);
// Anderson mixing: per-block partials (up to 256 blocks of 256 threads per
// geometry, 2 * AA_MAX + 3 sums each), then the combination.
constexpr size_t aa_partial_doubles() { return 256 * (2 * AA_MAX + 3); }
// kappa_mu = pref * Sg_mu * (sum_k w_k kraw[sys_k] - sum_s D_s kraw[s]) for
// every mode (terms per mode fixed, unused terms carry weight 0).
hipError_t launch_kappa_modes(const int* sys, const double* w, const double* Sg, int n_modes, int terms,
                              const double* D, int n_sys, const double* kraw, double pref, double* out,
                              hipStream_t st);
// re-centre T_L / T_w of the geometries with gauge = 1 (forward passes)
hipError_t launch_gauge(const GeomDev* geoms_dev, int n_geoms, int max_aa, hipStream_t st);
hipError_t launch_anderson(const GeomDev* geoms_dev, int n_geoms, int max_naa, PassParams pp, hipStream_t st);
hipError_t launch_finalize(const GeomDev* geoms_dev, int n_geoms, PassParams pp, hipStream_t st);
// outputs of one geometry (T_L centred, the flux map, the adjoint gradient;
// each skipped when its pointer is null)
hipError_t launch_output(const GeomDev* geom_dev, int precision, int ncells, double* T_L_out, double* J_out,
                         double* grad_out, hipStream_t st);
hipError_t launch_prep_sigma(const GeomDev* g_dev, int ncells, const double* sig, hipStream_t st);
hipError_t launch_apply(int precision, int transpose, const GeomDev* g_dev, const GeomDev& g_host,
                        const double* sigma, const int* sys_ids, int n_sys, const void* x, void* y,
                        hipStream_t st);

// Set the message obte_last_error returns (host, per thread).
void obte_set_error(const char* msg);
