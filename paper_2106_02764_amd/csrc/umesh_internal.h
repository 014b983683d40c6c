// Internal types of the unstructured-mesh path, shared by its host driver
// (umesh.cpp) and its gfx950 kernels (ukernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// At most four faces per cell (triangles and quadrilaterals).
constexpr int UFACES = 4;
// Code of an inflow slot in the sweep tables: >= n_solid: a periodic face
// (wrap slot code - n_solid); >= 0: the upwind solid cell; UWALL0 - code: a
// wall face; UNONE: unused.
constexpr int UNONE = -1;
constexpr int UWALL0 = -2;
// Wrap slots per wave lane the pass kernel keeps in registers.
constexpr int UWPL_MAX = 8;

struct UGeomDev {
    int ns, nwalls, n_sys, n_dir, n_mfp, grad_axis;
    int wmax;                 // wrap slots of the direction with the most
    int ncut;                 // interior faces across the periodic plane of the gradient axis
    double dT, Lg, Vbox, Aperp;
    // ---- static tables
    const double* V;          // ns: cell areas
    const double* mfp;        // n_mfp
    const double* Dw;         // n_sys: T_L weights
    const double* S;          // 2 * n_sys: flux weights
    const double* wout;       // nwalls * n_sys: outgoing weights of each wall face
    const int* wcell;         // nwalls: solid cell of each wall face
    // sweep tables per direction l: cells in upwind (topological) order,
    // grouped in levels whose cells depend only on earlier levels
    const int* ord;           // n_dir * ns
    const int* lbase;         // n_dir: start of direction l's level pointers in lptr
    const int* nlev;          // n_dir
    const int* lptr;          // level boundaries (positions in ord), n_lev + 1 per direction
    const double* dout;       // n_dir * ns (by position): sum of the outflow |s.n| A / V
    const int* inc;           // n_dir * ns * UFACES (by position): inflow codes
    const double* inv;        // n_dir * ns * UFACES: inflow |s.n| A / V
    const int* nwrap;         // n_dir: wrap slots of direction l
    const int* wup;           // n_dir * wmax: upwind solid cell of each wrap slot
    const double* wdel;       // n_dir * wmax: jump of the value crossing (delta dT)
    const int* cut_i;         // ncut: cell on the + side of the cut
    const int* cut_j;         // ncut: its neighbour across the cut
    const double* cut_An;     // 2 * ncut: A_f n_f (n_f from cut_i to cut_j)
    // ---- solve state (library-owned buffers)
    const double* sigma;      // ns
    double* T_L;              // ns
    double* T_w;              // nwalls
    double* U;                // n_sys * wmax: wrap inflow values
    double* X;                // n_sys * ns: each system's solution of the pass
    double* ksys;             // n_sys: kappa_cc share
    double* kfsys;            // n_sys: kappa_face share
    long long* iters;         // n_sys: accumulated BiCGSTAB iterations
    double* kap;              // 4: kappa_cc, kappa_face of the pass, max relative wrap residual
    double* wres;             // n_sys: relative wrap residual after the pass
    // ---- per pass, in every direction's sweep order (k_upack): sigma of the
    // cell at each position, sigma T_L, and the sum over its inflow wall faces
    // of |s.n| A / V T_w (the wall part of the source before the factor Lambda)
    double* psg;              // n_dir * ns
    double* pb0;              // n_dir * ns
    double* pbw;              // n_dir * ns
};

struct UFourierDev {
    int ns, nfaces, grad_axis, ncut;
    double dT, Lg, Aperp;
    const int* nb_ptr;        // ns + 1: neighbour lists (both sides of every interior face)
    const int* nb_j;          // neighbour cell
    const double* nb_a;       // primary coefficient A_f n.K n / (n.d)
    const double* nb_del;     // jump of the neighbour's image seen from the cell
    const double* nb_w;       // 2 per entry: least-squares weight column of the entry
    const int* nb_f;          // face index * 2 + (1 if the cell is the face's second cell)
    const int* fi;            // nfaces
    const int* fj;
    const double* fw;         // interpolation weight of the second cell's gradient
    const double* fc;         // 2 * nfaces: the secondary-flux vector c_f (first cell's side)
    const double* P;          // ns: perturbation (volume-scaled)
    const int* cut_f;         // ncut: face index of each cut face
    const int* cut_s;         // ncut: +1 if the face's first cell is on the + side, else -1
    const double* cut_K;      // 3 * ncut: n.K n / (n.d), (K n)_x, (K n)_y of the + side orientation
    const double* cut_d;      // 2 * ncut: d from the + side cell
    const double* cut_A;      // ncut
    // scratch (ns each) and outputs
    double* T;                // ns: the solution (mean zero)
    double* r;
    double* p;
    double* q;
    double* b;
    double* g;                // 2 * ns: cell gradients
    double* bf;               // nfaces: secondary flux per face
    double* out;              // 4: kappa_F, outer iterations, CG iterations, last relative change
    // multi-block solve: the second direction buffer, the previous outer
    // iterate, the diagonal, per-block partial sums and loop scalars
    double* r1;               // ns: r, A M^-1 r (w) and A p (s) by CG iteration parity
    double* w0;
    double* w1;
    double* s0;
    double* s1;
    double* tp;               // ns
    double* dg;               // ns
    double* fpart;            // UF_SLOTS * UF_MAXB
    double* fsc;              // UF_SCALARS
};
constexpr int UF_MAXB = 64;   // blocks of the multi-block heat-conduction kernels (256 cells each)
constexpr int UF_SLOTS = 10;
constexpr int UF_SCALARS = 16;

// Heat conduction, Eq. (final2), over several blocks: the start of an outer
// iteration (gradients, secondary fluxes, right-hand side, first residual),
// `iters` CG iterations (one kernel each; they return at once once the CG
// has stopped, which fsc[0] says), and the end of an outer iteration (mean
// removed, the change against the previous iterate in fsc[4], fsc[5] = 1 when
// it is within tol); then kappa_F and the statistics into out.
hipError_t ulaunch_fourier_start(const UFourierDev* f_dev, int ns, int nfaces, hipStream_t st);
hipError_t ulaunch_fourier_cg(const UFourierDev* f_dev, int ns, int iters, double cg_tol, int max_cg,
                              hipStream_t st);
hipError_t ulaunch_fourier_end(const UFourierDev* f_dev, int ns, double tol, hipStream_t st);
hipError_t ulaunch_fourier_kappa(const UFourierDev* f_dev, int ns, hipStream_t st);
// the pass's sources packed in sweep order (n_pos = n_dir * n_solid
// positions), then every system's pass
hipError_t ulaunch_pass(const UGeomDev* g_dev, int n_sys, int n_pos, int wpl, size_t lds_bytes, double inner_tol,
                        double inner_rtol, int max_inner, hipStream_t st);
hipError_t ulaunch_reduce(const UGeomDev* g_dev, int ns, int nwalls, hipStream_t st);
