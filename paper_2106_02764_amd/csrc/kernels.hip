// gfx950 kernels of the aMFP-BTE hot path.
//
// One outer pass (paper: Eq. (iter), Algorithm 1) solves, for every
// direction l and MFP m,
//     (sigma + Lambda_m A_l) x = b,
//     b = sigma T_L + Lambda_m [wall inflow (T_w) + periodic-jump inflow]
// with the upwind finite-volume operator of Appendix A, Eq. (iter2), then
// reduces the solutions into T_L = sum D x, the diffuse-wall temperatures
// T_w and kappa.
//
// Inner solve.  Ordering the cells of a structured grid in upwind order makes
// A_l lower triangular except for the periodic wrap couplings.  One wavefront
// owns one (m,l) system and sweeps the grid row by row in y-upwind order
// (and plane by plane in z-upwind order in 3D); inside a row the x-recurrence
// x_i = a_i + q_i x_{i-1}, cyclic when x is periodic, is solved exactly with a
// wavefront-wide scan of affine maps.  The sweep M^{-1} is therefore exact up
// to the y-wrap coupling E (row 0 <- last row).  BiCGSTAB right-preconditioned
// by the sweep works on A M^{-1} = I - E M^{-1}: its Krylov vectors are
// supported on the wrap row only, so they are nx*nz values held in the
// wavefront's registers and every dot product is a wavefront reduction.
// Each matrix-vector product is one sweep whose only source is the wrap row.
// No per-(cell,system) vector is ever stored: b is formed on the fly from the
// per-cell T_L / T_w tables shared by all systems.
//
// Reductions.  The systems of one workgroup share a direction and run their
// final sweep in lockstep; per row they combine D x (T_L), the outgoing wall
// weights (T_w) and S x (flux) through LDS in a fixed order and write one
// partial per workgroup.  A second kernel sums the partials per cell / wall in
// a fixed order and a third reduces kappa, so FP64 results are bitwise
// reproducible (no floating-point atomics).
#include "obte_internal.h"
#include <type_traits>

namespace {

constexpr int WAVE = 64;

template <typename T>
__device__ __forceinline__ T shfl_up(T v, int d) { return __shfl_up(v, d, WAVE); }
template <typename T>
__device__ __forceinline__ T shfl_at(T v, int l) { return __shfl(v, l, WAVE); }
template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int m) { return __shfl_xor(v, m, WAVE); }

// Butterfly sum: every lane ends with the bitwise-same value.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
    return v;
}

// N butterfly sums at once, step by step, so the cross-lane reads of the N
// values are in flight together; each value is summed exactly as wave_sum does.
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        double t[N];
#pragma unroll
        for (int q = 0; q < N; ++q) t[q] = shfl_xor(v[q], m);
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] += t[q];
    }
}

// Deterministic block sum (blockDim.x multiple of 64, <= 1024).
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (wid == 0) {
        t = lane < nw ? red[lane] : 0.0;
        t = wave_sum(t);
        if (lane == 0) red[16] = t;
    }
    __syncthreads();
    return red[16];
}

// Two block sums in one pass (red: at least 34 doubles); each value is summed
// exactly as block_sum sums it.
__device__ void block_sum2(double& a, double& b, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double v[2] = {a, b};
    wave_sum_n(v);
    __syncthreads();
    if (lane == 0) {
        red[wid] = v[0];
        red[16 + wid] = v[1];
    }
    __syncthreads();
    if (wid == 0) {
        double t[2] = {lane < nw ? red[lane] : 0.0, lane < nw ? red[16 + lane] : 0.0};
        wave_sum_n(t);
        if (lane == 0) {
            red[32] = t[0];
            red[33] = t[1];
        }
    }
    __syncthreads();
    a = red[32];
    b = red[33];
}

// A cell's grid coordinates (one division chain per cell), and its
// neighbour across face f (2a: '-' side of axis a, 2a + 1: '+' side) with the
// periodic wrap taken by comparison, so the per-face lookups divide nothing.
struct CellPos {
    int ix, iy, iz;
};
__device__ __forceinline__ CellPos cell_pos(const GeomDev& g, int cell) {
    const int q = cell / g.nx, r = q / g.ny;
    return {cell - q * g.nx, q - r * g.ny, r};
}
__device__ __forceinline__ int nbr_cell(const GeomDev& g, int cell, const CellPos& cp, int f) {
    const int a = f >> 1;
    const bool up = f & 1;
    const int n = a == 0 ? g.nx : (a == 1 ? g.ny : g.nz);
    const int i = a == 0 ? cp.ix : (a == 1 ? cp.iy : cp.iz);
    const int st = a == 0 ? 1 : (a == 1 ? g.nx : g.nx * g.ny);
    if (up) return i == n - 1 ? cell - (n - 1) * st : cell + st;
    return i == 0 ? cell + (n - 1) * st : cell - st;
}

using rsrc_t = __amdgpu_buffer_rsrc_t;

// Wave-uniform copies of values the compiler cannot prove uniform (loaded
// after the kernel's first store, or derived from the wave index): scalar
// registers, so the buffer resources and row offsets built from them are too.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ double uni(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
template <typename P>
__device__ __forceinline__ P* uni(P* p) {
    const unsigned long long a = (unsigned long long)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
    return (P*)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(uni(p)), 0, (int)uni(bytes), 0x00020000);
}

// ---------------------------------------------------------------------------
// per-system constants
// ---------------------------------------------------------------------------
template <typename T>
struct SysC {
    int sys, m, l;
    int pos[3];          // 1 if the sweep runs towards + along the axis
    int fin[3], fout[3]; // inflow / outflow face index per axis
    double cd[3];        // Lambda |s_a| / h_a
    T c[3];
    double kw;           // adjoint source k_ml
    double Dml;
    double Sg;           // S_ml along the gradient axis
    double S[3];
};

template <typename T>
__device__ __forceinline__ SysC<T> make_sys(const GeomDev& g, int m, int l, int adjoint) {
    SysC<T> s;
    s.m = m;
    s.l = l;
    s.sys = m * g.n_dir + l;
    const double lam = g.mfp[m];
    for (int a = 0; a < 3; ++a) {
        double sa = (a < g.ndim) ? g.dirs[l * 3 + a] : 0.0;
        if (adjoint) sa = -sa;   // A_l^T = A_{-l} on a uniform grid
        s.pos[a] = sa > 0.0;
        s.fin[a] = 2 * a + (sa > 0.0 ? 0 : 1);
        s.fout[a] = 2 * a + (sa > 0.0 ? 1 : 0);
        s.cd[a] = (a < g.ndim) ? lam * fabs(sa) / g.h[a] : 0.0;
        s.c[a] = (T)s.cd[a];
        s.S[a] = g.S[s.sys * 3 + a];
    }
    s.Dml = g.Dw[s.sys];
    s.Sg = g.S[s.sys * 3 + g.grad_axis];
    s.kw = g.L[g.grad_axis] / (g.dT * (double)g.ncells) * s.Sg;
    // one system per wave: the indices and orientation flags are
    // wave-uniform (scalar registers; they address the row loads)
    s.sys = uni(s.sys);
    s.m = uni(s.m);
    s.l = uni(s.l);
    for (int a = 0; a < 3; ++a) {
        s.pos[a] = uni(s.pos[a]);
        s.fin[a] = uni(s.fin[a]);
        s.fout[a] = uni(s.fout[a]);
    }
    return s;
}

// Upper bound of the gain of a system's wrap map G (inflow of the first row
// -> mask * c_y * outflow of the last row, sources zero).  One row of the
// sweep solves (D - C_in) x = c_y y, where D = sigma + sum c and C_in holds
// the in-row (x, and z in 3D) upwind couplings: an M-matrix whose rows and
// columns both exceed their off-diagonal sums by at least sigma_min + c_y.
// So every row transfer has max- and 1-norm (hence 2-norm) at most
// q = c_y / (sigma_min + c_y), walls and pores only lower it, and
// |G r| <= q^ny |r| for the BiCGSTAB's 2-norm.  1 when sigma_min <= 0.
// The sweep-free step is taken only where it cuts the wrap residual at least
// tenfold: with a weaker cut (up to the forcing term 0.3) the mixed outer
// iteration needed more passes (22 -> 26 on the 128x128 cell), which cost
// more than the sweeps saved.
constexpr double RICH_MAX = 0.1;

template <typename T>
__device__ __forceinline__ double wrap_gain_bound(const GeomDev& g, const SysC<T>& s) {
    const double smin = g.fscal[5], cy = s.cd[1];
    if (!(smin > 0.0)) return 1.0;
    return pow(cy / (smin + cy), (double)g.ny);
}

template <typename T>
__device__ __forceinline__ const T* sigma_ptr(const GeomDev& g);
template <>
__device__ __forceinline__ const double* sigma_ptr<double>(const GeomDev& g) { return g.sigma; }
template <>
__device__ __forceinline__ const float* sigma_ptr<float>(const GeomDev& g) { return g.sigma_f; }


// ---------------------------------------------------------------------------
// cross-lane primitives: DPP row shifts / row broadcasts / wave shift and
// v_readlane.  `old` is what a lane receives when it has no source lane.
// ---------------------------------------------------------------------------
template <int CTRL, int RM>
__device__ __forceinline__ float dpp(float v, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, RM, 0xf, false));
}
template <int CTRL, int RM>
__device__ __forceinline__ double dpp(double v, double old) {
    const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, CTRL, RM, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, RM, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One Hillis-Steele step of the affine-map scan: this lane's map x -> A + Q x
// is composed after the map of the source lane (identity where none).  Only
// A and P = 1 - Q are carried: P keeps full relative accuracy where it is
// small (a nearly closed cyclic chain, the closure divides by it), and where
// 1 - P is inexact (Q tiny) it only scales terms it makes negligible.
// Full-mask row shifts read the source with bound_ctrl (a lane without
// source reads 0, the identity's A and P).
template <int CTRL, int RM>
__device__ __forceinline__ void scan_step(float& A, float& P) {
    const bool bc = RM == 0xf;
    const float A2 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(A), CTRL, RM, 0xf, bc));
    const float P2 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(P), CTRL, RM, 0xf, bc));
    const float t = 1.0f - P;
    A = A + t * A2;
    P = P + t * P2;
}
template <int CTRL, int RM>
__device__ __forceinline__ void scan_step(double& A, double& P) {
    const double A2 = dpp<CTRL, RM>(A, 0.0), P2 = dpp<CTRL, RM>(P, 0.0);
    const double t = 1.0 - P;
    A = A + t * A2;
    P = P + t * P2;
}

// Inclusive wavefront scan of the maps (A, P).
template <typename T>
__device__ __forceinline__ void wave_scan(T& A, T& P) {
    scan_step<0x111, 0xf>(A, P);   // row_shr:1
    scan_step<0x112, 0xf>(A, P);   // row_shr:2
    scan_step<0x114, 0xf>(A, P);   // row_shr:4
    scan_step<0x118, 0xf>(A, P);   // row_shr:8
    scan_step<0x142, 0xa>(A, P);   // row_bcast:15 into rows 1, 3
    scan_step<0x143, 0xc>(A, P);   // row_bcast:31 into rows 2, 3
}

// FP32: a step is t = 1 - P and two multiply-adds whose multiplicand is the
// accumulator itself read from the source lane (a DPP operand may name the
// destination: the source lanes are read before any is written; and the
// rows a row_bcast step writes never hold its source lane).  A lane with no
// source reads 0 (bound_ctrl), a row that a row_bcast step does not write
// keeps its map: both compose the identity.  The compiler does not fold its
// own DPP moves into v_fmac, so this saves two moves per step and the zero
// fills of the row_bcast steps.  Hazard: a DPP read needs two wait states
// after the VALU write of its register; within a step the v_sub and the
// other accumulator's update provide them, s_nop 1 covers the first step.
__device__ __forceinline__ void wave_scan(float& A, float& P) {
    float t;
    asm volatile(
        "s_nop 1\n\t"
        "v_sub_f32 %2, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %2 row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %1, %2 row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_sub_f32 %2, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %2 row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %1, %2 row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_sub_f32 %2, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %2 row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %1, %2 row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_sub_f32 %2, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %2 row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %1, %2 row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_sub_f32 %2, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %2 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %1, %2 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_sub_f32 %2, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %2 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %1, %2 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(A), "+v"(P), "=&v"(t));
}

// Loads through these views compile to global (not flat) loads, which keep
// only the vector-memory counter pending while the row computes.
template <typename T>
using gptr_t = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr_t<T> gview(const T* p) { return (gptr_t<T>)p; }
// Writable global views: stores through them are global (not flat) stores,
// which a barrier's wait on the LDS counter does not include.
template <typename T>
using gmut_t = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gmut_t<T> gmut(T* p) { return (gmut_t<T>)p; }

// Raw buffer access (gfx9 descriptors): a resource for the whole array, a
// per-lane byte offset fixed for the sweep and a scalar offset per row, so a
// row's loads need no per-lane address arithmetic.  A raw buffer access is
// range-checked on its per-lane offset: a store whose offset is at or past
// the array's size is dropped (used for pores and beyond-row lanes).
constexpr uint32_t BUF_OOB = 0x80000000u;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bld16(rsrc_t r, uint32_t vo, uint32_t so) {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ uint32_t bld32(rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ double bld64(rsrc_t r, uint32_t vo, uint32_t so) {
    const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0);
    return __longlong_as_double(((long long)v.y << 32) | (unsigned long long)v.x);
}
template <typename T>
__device__ __forceinline__ T bldT(rsrc_t r, uint32_t vo, uint32_t so);
template <>
__device__ __forceinline__ float bldT<float>(rsrc_t r, uint32_t vo, uint32_t so) {
    return __uint_as_float(bld32(r, vo, so));
}
template <>
__device__ __forceinline__ double bldT<double>(rsrc_t r, uint32_t vo, uint32_t so) {
    return bld64(r, vo, so);
}
__device__ __forceinline__ void bst(float v, rsrc_t r, uint32_t vo) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)vo, 0, 0);
}
__device__ __forceinline__ void bst(double v, rsrc_t r, uint32_t vo) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    u32x2_t w;
    w.x = (unsigned int)b;
    w.y = (unsigned int)(b >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)vo, 0, 0);
}

// Per-wave state of a sweep that keeps its result: the kappa sums in
// registers, and the solution stored on the solid cells (the sums over
// systems per cell and per wall are taken afterwards by the reduction kernel).
template <typename T>
struct Red {
    int store_T;
    int on;                    // 0: inactive wave (nothing is stored)
    double kacc, kface;
    T kt, kft;                 // per-lane partials of kacc / kface in the compute type (2D)
    rsrc_t X;                  // this system's solution by solid index
    rsrc_t Tstore;             // this system's stored state (store_T only)
};

// 1/d: hardware reciprocal (float), refined by two Newton steps (double).
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = r * (2.0 - d * r);
    return r * (2.0 - d * r);
}

// per-row inputs of one lane (prefetched ahead of use; the 3D-only fields
// have one dummy entry in 2D, so the rotation buffers stay in registers)
template <typename T, int CPL, bool D3>
struct RowIn {
    uint32_t w[CPL];
    T sg[CPL];
    T sb[CPL];          // base source (sigma T_L, or k + D Psi), compute type
    T bx[CPL], by[CPL];                 // inflow boundary values per axis
    T bz[D3 ? CPL : 1];
    int si[CPL];        // solid index of the cell (sweeps that store), -1 in pores
    T ui[D3 ? CPL : 1]; // 3D: the wrap-plane input of the row's plane (used on the first y-row)
};

// Row results of a storing sweep, kept in registers until a group of rows is
// stored together.  A wave's global loads and stores share one counter on
// gfx9, and with both kinds in flight every wait for a prefetched row must
// drain the whole counter; storing once per group keeps the row prefetch
// overlapped everywhere else.
template <typename T, int CPL>
struct RowOut {
    T x[CPL];
    int si[CPL];        // -1: nothing to store
};

// per-sweep constant views: buffer resources of the per-cell tables and of
// the 3D wrap-plane input, and this lane's byte offsets within a row
template <typename T, int CPL>
struct Views {
    rsrc_t fc, sidx, sg, u, src, bx, by, bz;
    uint32_t o2[CPL], o4[CPL], oT[CPL], ou[CPL];
    // geometry scalars read once per sweep: the row loop stores to global
    // memory, after which the compiler would reload them from the view
    int nx, ny, nz, ga;
    int lx, cx;                        // lane and register of a row's last cell (p = nx - 1)
    double dT;
};

template <typename T, int CPL, bool D3, bool WITH_B, bool S1, bool ST>
__device__ __forceinline__ void load_row(const GeomDev& g, const SysC<T>& s, const Views<T, CPL>& v, int lane,
                                         int jj, int kk, RowIn<T, CPL, D3>& r) {
    // every lane loads (beyond the row: the row's first cell, masked by the
    // row step), so no load sits in a branch or feeds a select here: the
    // compiler then counts the loads in flight exactly and waits only for
    // the row it is about to use
    const int iy = s.pos[1] ? jj : v.ny - 1 - jj;
    const int iz = D3 ? (s.pos[2] ? kk : v.nz - 1 - kk) : 0;
    const uint32_t rowbase = uni((uint32_t)(v.nx * (iy + v.ny * iz)));
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        r.w[c] = bld16(v.fc, v.o2[c], rowbase * 2u);
        if (ST) r.si[c] = (int)bld32(v.sidx, v.o4[c], rowbase * 4u);
        r.sg[c] = S1 ? T(1) : bldT<T>(v.sg, v.oT[c], rowbase * (uint32_t)sizeof(T));
        if (WITH_B) {
            const uint32_t rb = rowbase * (uint32_t)sizeof(T);
            r.sb[c] = bldT<T>(v.src, v.oT[c], rb);
            r.bx[c] = bldT<T>(v.bx, v.oT[c], rb);
            r.by[c] = bldT<T>(v.by, v.oT[c], rb);
            if (D3) r.bz[c] = bldT<T>(v.bz, v.oT[c], rb);
        }
        if (D3) r.ui[c] = bldT<T>(v.u, v.ou[c], uni((uint32_t)(kk * v.nx)) * (uint32_t)sizeof(T));
    }
}

// Row storage of the sweep.  2D: the previous row in registers.  3D: the
// previous y-row of every z-plane in this wave's LDS region (the plane index
// is a runtime value), and the row just below in z in registers.
template <typename T, int CPL, bool D3>
struct Rows {
    T xr[CPL];    // 2D: row jj-1; 3D: row (jj, kk-1)
    T* xz;        // 3D: nz * ROW values, plane kk holds row (jj-1, kk) until overwritten
    int ROW;
    __device__ __forceinline__ T prev_y(int kk, int c, int lane) const {
        return D3 ? xz[kk * ROW + lane * CPL + c] : xr[c];
    }
    __device__ __forceinline__ T prev_z(int c) const { return D3 ? xr[c] : T(0); }
    __device__ __forceinline__ void put(int kk, int c, int lane, T v) {
        if (D3) xz[kk * ROW + lane * CPL + c] = v;
        xr[c] = v;
    }
};

// Wrap-row input (inflow u of the first row) and output (the last row).
// 2D: register arrays of this lane.  3D: the system's nz x nx plane in
// global memory, element (kk, p) at kk * nx + p, always touched by the lane
// that owns column p, so no cross-lane ordering is needed.
template <typename T, int CPL>
struct RegIO {
    const T (&u)[CPL];
    T (&xl)[CPL];
    __device__ __forceinline__ T in(int, int c, int) const { return u[c]; }
    __device__ __forceinline__ const T* input() const { return nullptr; }
    __device__ __forceinline__ void out(int, int c, int, T v) { xl[c] = v; }
};
template <typename T, int CPL>
struct GlobIO {
    gptr_t<T> u;
    rsrc_t xl;           // size 0 when the last row is not needed (or the wave is inactive)
    int nx;
    __device__ __forceinline__ const T* input() const { return (const T*)u; }
    // the row loads prefetch the input (Views::u); nothing is read here
    __device__ __forceinline__ T in(int, int, int) const { return T(0); }
    // a buffer store in no per-lane branch (beyond the row: an offset past
    // the plane, dropped), so the compiler keeps counting the row prefetches
    // in flight exactly across it
    __device__ __forceinline__ void out(int kk, int c, int lane, T v) {
        const int p = lane * CPL + c;
        bst(v, xl, p < nx ? (uint32_t)(kk * nx + p) * (uint32_t)sizeof(T) : BUF_OOB);
    }
};
// out_plane: the nz x nx plane receiving the last row, or nullptr
template <typename T, int CPL>
__device__ __forceinline__ GlobIO<T, CPL> make_gio(gptr_t<T> u, gmut_t<T> out_plane, int nx, int nz, int active) {
    GlobIO<T, CPL> io;
    io.u = u;
    io.xl = make_rsrc((const T*)out_plane, (out_plane && active) ? (uint32_t)(nx * nz) * (uint32_t)sizeof(T) : 0u);
    io.nx = nx;
    return io;
}

// One row step of the sweep (cells of row (jj, kk) in upwind order).  FULL:
// the row fills every lane (nx = 64 CPL), so no lane holds cells beyond it.
template <typename T, int CPL, bool D3, bool WITH_B, bool RED, bool ADD, bool S1, int GA, bool FULL = false,
          class IO>
__device__ __forceinline__ void row_step(const GeomDev& g, const SysC<T>& s, const Views<T, CPL>& vw,
                                         int active, int lane, int adj, int jj, int kk,
                                         const RowIn<T, CPL, D3>& cur, Rows<T, CPL, D3>& rows, IO& io,
                                         const double (&mb)[3], Red<T>* rd, RowOut<T, CPL>& ro) {
    constexpr int ND = D3 ? 3 : 2;
    const int nx = vw.nx, ny = vw.ny;
    const T cz = D3 ? s.c[2] : T(0);
    // diagonal without sigma (2D: no z term, so no +0 is left in the chain)
    const T cdiag = D3 ? s.c[0] + s.c[1] + cz : s.c[0] + s.c[1];
    const T cyz = D3 ? s.c[1] + cz : s.c[1];
    // sigma = 1: the cell coefficients are this system's constants
    const T rdv1 = S1 ? recip(T(1) + cdiag) : T(0);
    const T q1 = s.c[0] * rdv1, pxs1 = (T(1) + cyz) * rdv1, pnx1 = (T(1) + cdiag) * rdv1;
    T a[CPL], q[CPL];
    T Al, Pl;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int p = lane * CPL + c;
        const uint32_t w = (FULL || p < nx) ? cur.w[c] : 0u;     // beyond the row: not solid
        const bool sol = active && fc_solid(w);
        const int clx = fc_class(w, s.fin[0]);
        const int cly = fc_class(w, s.fin[1]);
        const int clz = D3 ? fc_class(w, s.fin[2]) : FC_WALL;
        // sigma = 1 everywhere (no multiplier given): rdv is this system's constant
        const T sg = S1 ? T(1) : cur.sg[c];
        const T rdv = S1 ? rdv1 : recip(sg + cdiag);
        // kk and jj are wave-uniform: the wrap input is used on the first row
        // only (3D: prefetched with every row, so its load is in no branch)
        const T uin = D3 ? ((FULL || p < nx) ? cur.ui[c] : T(0)) : io.in(kk, c, lane);
        // the row below in y is read unconditionally (no branch around the
        // LDS load) and selected
        const T py = rows.prev_y(kk, c, lane);
        const T yin = cly != FC_WALL ? ((jj == 0) ? uin : s.c[1] * py) : T(0);
        T rhs = yin;
        if (WITH_B) {
            // in the compute type (the sources were converted once per pass)
            T sd = adj ? (T)s.kw + (T)s.Dml * cur.sb[c] : cur.sb[c];
            sd += (T)mb[0] * cur.bx[c] + (T)mb[1] * cur.by[c];
            if (D3) sd += (T)mb[2] * cur.bz[c];
            rhs = sd + yin;
        }
        if (D3) rhs += (clz != FC_WALL && kk > 0) ? cz * rows.prev_z(c) : T(0);
        const bool xs = (clx != FC_WALL);
        T av = rhs * rdv;
        T qv = xs ? (S1 ? q1 : s.c[0] * rdv) : T(0);
        T pv = S1 ? (xs ? pxs1 : pnx1) : (sg + (xs ? cyz : cdiag)) * rdv;
        // pore: (0, 0, 1) breaks the chain; beyond the row (face word 0, so
        // not solid either): the identity (0, 1, 0)
        const bool beyond = !FULL && p >= nx;
        av = sol ? av : T(0);
        qv = sol ? qv : (beyond ? T(1) : T(0));
        pv = sol ? pv : (beyond ? T(0) : T(1));
        a[c] = av;
        q[c] = qv;
        if (c == 0) {
            Al = av;
            Pl = pv;
        } else {
            Al = av + qv * Al;
            Pl = pv + qv * Pl;
        }
    }
    T A = Al, P = Pl;
    wave_scan(A, P);
    const T At = readlane(A, WAVE - 1), Pt = readlane(P, WAVE - 1);
    const T xin = (Pt > T(0)) ? At * recip(Pt) : T(0);   // cyclic closure x_{-1} = x_{nx-1}
    const T Ae = dpp<0x138, 0xf>(A, T(0)), Pe = dpp<0x138, 0xf>(P, T(0));   // wave_shr:1
    T xp = Ae + (T(1) - Pe) * xin;
    T xrow[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const T xv = a[c] + q[c] * xp;
        const int p = lane * CPL + c;
        xrow[c] = (FULL || p < nx) ? xv : T(0);
        rows.put(kk, c, lane, xrow[c]);
        xp = xv;
    }
    if (jj == ny - 1) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) io.out(kk, c, lane, xrow[c]);
    }
    if (RED) {
        // branch-free: cells that contribute nothing add an exact 0 (an
        // inactive wave's sums are dropped, its stores skipped)
        // the row's cells summed in the compute type, the rows in double
        T rsum = T(0);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int p = lane * CPL + c;
            const uint32_t wv = (FULL || p < nx) ? cur.w[c] : 0u;
            const bool sol = fc_solid(wv);
            ro.x[c] = xrow[c];
            ro.si[c] = sol ? cur.si[c] : -1;
            rsum += sol ? xrow[c] : T(0);
        }
        rd->kacc += (double)rsum;
        // Flux through the periodic plane of the gradient axis (kappa_face;
        // the adjoint: p^T lambda of the jump inflow, on the forward's jump
        // faces = this sweep's outflow faces).  The jump term belongs to the
        // b sweep only.
        if (GA == 0) {
            // the plane's cell of a row is its last cell in sweep order
            // (p = nx - 1): one lane's value, read into a scalar, added on
            // lane 0 (the wave sum then equals the sum over the rows)
            // (each register is read into a scalar and the scalars are
            // selected: selecting the registers first would let the compiler
            // index the row buffers at run time, which puts them in memory)
            T xl = readlane(xrow[0], vw.lx);
            uint32_t wl = (uint32_t)__builtin_amdgcn_readlane((int)cur.w[0], vw.lx);
#pragma unroll
            for (int c = 1; c < CPL; ++c) {
                const T xc = readlane(xrow[c], vw.lx);
                const uint32_t wc = (uint32_t)__builtin_amdgcn_readlane((int)cur.w[c], vw.lx);
                xl = (c == vw.cx) ? xc : xl;
                wl = (c == vw.cx) ? wc : wl;
            }
            double add = 0.0;
            if (fc_solid(wl)) {
                const int cl = fc_class(wl, s.fout[0]);
                const double xd = (double)xl;
                if (adj) {
                    const double cj = s.cd[0] * vw.dT;
                    add = cl == FC_JUMP_P ? cj * xd : (cl == FC_JUMP_M ? -cj * xd : 0.0);
                } else {
                    add = cl != FC_WALL ? xd + ((!ADD && s.pos[0]) ? vw.dT : 0.0) : 0.0;
                }
            }
            rd->kface += lane == 0 ? add : 0.0;
        } else if (GA == 1 && jj == ny - 1) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int p = lane * CPL + c;
                const uint32_t wv = (FULL || p < nx) ? cur.w[c] : 0u;
                // selects, not per-lane branches: a divergent region in the
                // row loop makes the compiler wait for every row prefetch
                const double xv = (double)xrow[c];
                const int cl = fc_class(wv, s.fout[1]);
                double add;
                if (adj) {
                    const double cj = s.cd[1] * vw.dT;
                    add = cl == FC_JUMP_P ? cj * xv : (cl == FC_JUMP_M ? -cj * xv : 0.0);
                } else {
                    add = cl != FC_WALL ? xv + ((!ADD && s.pos[1]) ? vw.dT : 0.0) : 0.0;
                }
                rd->kface += fc_solid(wv) ? add : 0.0;
            }
        }
    }
}

// Store a group of rows of a storing sweep (ADD: add to the stored values);
// cells with nothing to store get an out-of-range offset, so every lane
// issues the same stores and the hardware drops those.
template <typename T, int CPL, int NR, bool ADD>
__device__ __forceinline__ void store_rows(Red<T>* rd, const RowOut<T, CPL> (&ro)[NR]) {
    // no branch on rd->on: an inactive wave's resources have size 0
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int i = ro[r].si[c];
            const uint32_t vo = i >= 0 ? (uint32_t)i * (uint32_t)sizeof(T) : BUF_OOB;
            T v = ro[r].x[c];
            if (ADD) v += bldT<T>(rd->X, vo, 0);
            bst(v, rd->X, vo);
            if (rd->store_T) bst((double)ro[r].x[c], rd->Tstore, i >= 0 ? (uint32_t)i * 8u : BUF_OOB);
        }
}

// ---------------------------------------------------------------------------
// The upwind sweep x = M^{-1}(src + P u): rows in y-upwind order (planes in
// z-upwind order), each row's cyclic x-recurrence solved by a wavefront scan.
// WITH_B: the pass sources are included, otherwise the only source is the
// wrap inflow u.  RED: lockstep reductions (every wave of the block calls
// it); ADD: add to the partials written by an earlier RED sweep of the same
// block.  Returns the last row (jj = ny-1) in xl.  Row inputs are prefetched
// two rows ahead (2D) through a three-buffer rotation without copies.
// ---------------------------------------------------------------------------


template <typename T, int CPL, bool D3, bool WITH_B, bool RED, bool ADD, bool S1, int GA, bool FULL = false,
          class IO>
__device__ __forceinline__ void sweep(const GeomDev& g, const SysC<T>& s, int active, int lane, int adj,
                                      const T* __restrict__ srcbase, const T* __restrict__ bnd,
                                      IO& io, Red<T>* rd, T* zrows) {
    constexpr int ND = D3 ? 3 : 2;
    double mb[3];
    // boundary input face per axis: forward, the wall this direction enters
    // from; adjoint, the wall whose temperature takes this system, the one
    // that S leaves through (with kappa_m weights: the reversed inflow face)
    int fb[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        fb[ax] = adj ? 2 * ax + (s.S[ax] > 0.0 ? 1 : 0) : s.fin[ax];
        mb[ax] = adj ? (ax < ND ? g.wout[fb[ax] * g.n_sys + s.sys] : 0.0) : s.cd[ax];
    }
    Views<T, CPL> vw;
    const uint32_t nc = (uint32_t)g.ncells;
    vw.fc = make_rsrc(g.fc, nc * 2u);
    vw.sidx = make_rsrc(g.sidx, nc * 4u);
    vw.sg = make_rsrc(sigma_ptr<T>(g), nc * (uint32_t)sizeof(T));
    vw.u = make_rsrc(io.input(), (uint32_t)(g.nx * g.nz) * (uint32_t)sizeof(T));
    const uint32_t tb = nc * (uint32_t)sizeof(T);
    vw.src = make_rsrc(srcbase, tb);
    vw.bx = make_rsrc(bnd + (size_t)fb[0] * g.ncells, tb);
    vw.by = make_rsrc(bnd + (size_t)fb[1] * g.ncells, tb);
    vw.bz = make_rsrc(bnd + (size_t)(D3 ? fb[2] : 0) * g.ncells, tb);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        // cell of this lane within a row (beyond the row: the row's first cell)
        const int p = lane * CPL + c;
        const uint32_t lo = p < g.nx ? (uint32_t)(s.pos[0] ? p : g.nx - 1 - p) : 0u;
        vw.o2[c] = lo * 2u;
        vw.o4[c] = lo * 4u;
        vw.oT[c] = lo * (uint32_t)sizeof(T);
        vw.ou[c] = (uint32_t)min(p, g.nx - 1) * (uint32_t)sizeof(T);
    }
    vw.nx = uni(g.nx);
    vw.ny = uni(g.ny);
    vw.nz = uni(g.nz);
    vw.ga = uni(g.grad_axis);
    vw.lx = (vw.nx - 1) / CPL;
    vw.cx = (vw.nx - 1) % CPL;
    vw.dT = uni(g.dT);
    Rows<T, CPL, D3> rows;
#pragma unroll
    for (int c = 0; c < CPL; ++c) rows.xr[c] = T(0);
    rows.xz = zrows;
    rows.ROW = WAVE * CPL;
    const int ny = g.ny;
    // Rows (jj, kk) in order, kk inner (2D: kk = 0).  A three-buffer
    // rotation keeps the inputs two rows ahead; prefetches are never skipped
    // (past the last row they reload it): a load inside a branch would leave
    // the compiler unsure how many loads are in flight at the join, and it
    // would then wait for all.  A storing sweep stores each group of three
    // rows after the group's last row.
    const int nz = D3 ? g.nz : 1, nrows = ny * nz;
    // row r -> (r / nz, r % nz) by a multiply with mz = ceil(2^32 / nz), not a
    // division per row: r mz / 2^32 = r / nz + r e / (nz 2^32) with e = mz nz
    // - 2^32 < nz, so the floor is exact while r e < 2^32, i.e. for every
    // r < 2^25 (nz <= 128)
    const uint64_t mz = D3 ? ((1ull << 32) + (uint64_t)nz - 1) / (uint64_t)nz : 1ull;
    auto row_j = [&](int r) { return D3 ? (int)(((uint64_t)(uint32_t)r * mz) >> 32) : r; };
    auto pre = [&](int r, RowIn<T, CPL, D3>& b) {
        const int rr = min(r, nrows - 1);
        const int jr = row_j(rr);
        load_row<T, CPL, D3, WITH_B, S1, RED>(g, s, vw, lane, jr, D3 ? rr - jr * nz : 0, b);
    };
    auto step = [&](int r, const RowIn<T, CPL, D3>& b, RowOut<T, CPL>& ro) {
        const int jr = row_j(r);
        row_step<T, CPL, D3, WITH_B, RED, ADD, S1, GA, FULL>(g, s, vw, active, lane, adj, jr, D3 ? r - jr * nz : 0,
                                                       b, rows, io, mb, rd, ro);
    };
    RowIn<T, CPL, D3> b0, b1, b2;
    pre(0, b0);
    pre(1, b1);
    for (int r = 0; r < nrows; r += 3) {
        RowOut<T, CPL> ro[3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int c = 0; c < CPL; ++c) ro[q].si[c] = -1;
        pre(r + 2, b2);
        step(r, b0, ro[0]);
        pre(r + 3, b0);
        if (r + 1 < nrows) step(r + 1, b1, ro[1]);
        pre(r + 4, b1);
        if (r + 2 < nrows) step(r + 2, b2, ro[2]);
        if (RED) store_rows<T, CPL, 3, ADD>(rd, ro);
    }
}

// ---------------------------------------------------------------------------
// 2D sweeps in the quadrant layout.  Every system whose direction falls in
// quadrant q reads the same per-cell inputs in the same order, so the pack
// kernel writes them once per pass in that order (GeomDev::qrec, qoff, qsg):
// a sweep row is then contiguous records behind one scalar row offset, and a
// row step spends a few multiply-adds per cell (the face classes are
// decoded, the sources converted and the pores zeroed once per pass, not
// once per system).  x-upwind position p of a row and x-upwind lane order
// are the same, so a lane's CPL cells are consecutive records.
// ---------------------------------------------------------------------------
struct alignas(16) QRecF {
    float sb, bx, by;
    uint32_t meta;
};
struct alignas(16) QRecD {
    double sb, bx, by;
    uint32_t meta, pad;
};
template <typename T>
using QRec = typename std::conditional<sizeof(T) == 4, QRecF, QRecD>::type;
static_assert(sizeof(QRecF) == 16 && sizeof(QRecD) == 32, "record = four compute-type words");

template <typename T>
__global__ void __launch_bounds__(256) k_pack_rows(const GeomDev* __restrict__ geoms, PassParams pp,
                                                   int* __restrict__ queue) {
    // the pass's item queue (persistent launches) starts at the first item
    if (queue && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *queue = 0;
    const GeomDev& g = geoms[blockIdx.y];
    if (pp.mode == 0 && g.ctrl[CTRL_DONE]) return;
    // the buffers the pass's sweeps read (the same rule as the pass kernel)
    const int pass = g.ctrl[CTRL_PASS];
    const int buf = (pp.mode == 1) ? ((pass + 1) & 1) : (pass & 1);
    const int nx = g.nx, ny = g.ny, nc = g.ncells, ga = g.grad_axis;
    const double* src = (pp.adjoint ? g.lam_psi : g.sT) + (size_t)buf * nc;
    const double* bnd = g.bnd + ((size_t)(pp.adjoint ? 2 : 0) + buf) * g.nf * nc;
    const T* sig = sigma_ptr<T>(g);
    QRec<T>* rec = reinterpret_cast<QRec<T>*>(g.qrec);
    T* qsg = reinterpret_cast<T*>(g.qsg);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 4 * nc; i += gridDim.x * blockDim.x) {
        const int q = i / nc, k = i - q * nc;
        const int r = k / nx, p = k - r * nx;
        const int negx = q & 1, negy = q >> 1;          // 1: the sweep runs towards - along the axis
        const int cell = (negy ? ny - 1 - r : r) * nx + (negx ? nx - 1 - p : p);
        const uint16_t w = g.fc[cell];
        const bool sol = fc_solid(w);
        // inflow face per axis (face 2a + side, side 1 = '+'): the '-' face
        // of a sweep towards +; the same rule gives the adjoint's boundary
        // face (its sweep runs along -s, its values sit on the faces S leaves by)
        const int fix = negx, fiy = 2 + negy;
        const bool ox = sol && fc_class(w, fix) != FC_WALL;
        const bool oy = sol && fc_class(w, fiy) != FC_WALL;
        const bool plane = ga == 0 ? p == nx - 1 : r == ny - 1;
        const int fo = ga == 0 ? 1 - negx : 3 - negy;   // outflow face along the gradient axis
        const bool kf = sol && plane && fc_class(w, fo) != FC_WALL;
        QRec<T> e{};
        e.sb = sol ? (T)src[cell] : T(0);
        e.bx = sol ? (T)bnd[(size_t)fix * nc + cell] : T(0);
        e.by = sol ? (T)bnd[(size_t)fiy * nc + cell] : T(0);
        e.meta = (uint32_t)ox | ((uint32_t)oy << 8) | ((uint32_t)kf << 16) | ((uint32_t)sol << 24);
        rec[i] = e;
        g.qoff[i] = sol ? (uint32_t)g.sidx[cell] * (uint32_t)sizeof(T) : QOFF_NONE;
        qsg[i] = sig[cell];
        if (pp.adjoint) {
            T* alt = reinterpret_cast<T*>(g.qalt) + 2 * (size_t)i;
            alt[0] = sol ? (T)bnd[(size_t)(1 - negx) * nc + cell] : T(0);
            alt[1] = sol ? (T)bnd[(size_t)(3 - negy) * nc + cell] : T(0);
        }
    }
}

typedef unsigned int u32x3_t __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
// N consecutive dwords at one lane offset, in loads of at most four dwords
template <int N>
__device__ __forceinline__ void bld_dw(uint32_t (&d)[N], rsrc_t r, uint32_t vo, uint32_t so) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
        const int n = N - i < 4 ? N - i : 4;
        const uint32_t o = vo + 4u * (uint32_t)i;
        if (n == 4) {
            const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)o, (int)so, 0);
            d[i] = v.x; d[i + 1] = v.y; d[i + 2] = v.z; d[i + 3] = v.w;
        } else if (n == 3) {
            const u32x3_t v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)o, (int)so, 0);
            d[i] = v.x; d[i + 1] = v.y; d[i + 2] = v.z;
        } else if (n == 2) {
            const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)o, (int)so, 0);
            d[i] = v.x; d[i + 1] = v.y;
        } else {
            d[i] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)o, (int)so, 0);
        }
    }
}
template <typename T>
__device__ __forceinline__ T from_dw(const uint32_t* d);
template <>
__device__ __forceinline__ float from_dw<float>(const uint32_t* d) { return __uint_as_float(d[0]); }
template <>
__device__ __forceinline__ double from_dw<double>(const uint32_t* d) {
    return __longlong_as_double(((long long)d[1] << 32) | (unsigned long long)d[0]);
}
// a byte of a record's flag word as a compute-type 0 / 1
template <typename T, int B>
__device__ __forceinline__ T flag(uint32_t m) { return (T)(float)((m >> (8 * B)) & 0xffu); }

template <typename T, int CPL>
struct QViews {
    rsrc_t rec, off, sg, alt;
    uint32_t orec[CPL];    // byte offset of this lane's records within a row
    uint32_t ooff, osg;    // byte offset of this lane's first store offset / sigma within a row
    int nx, ny;
};

template <typename T, int CPL>
struct QRowIn {
    T sb[CPL], bx[CPL], by[CPL];
    T bxo[CPL], byo[CPL];      // adjoint: boundary values of the outflow faces
    uint32_t meta[CPL];
    uint32_t so[CPL];
    T sg[CPL];
};

template <typename T, int CPL>
struct QRowOut {
    T x[CPL];
    uint32_t so[CPL];
};

// Row inputs at record k0 (the row's first cell; at or past the end of the
// table, as for the prefetch beyond the last row, the range-checked loads
// return zeros that no row step uses).
template <typename T, int CPL, bool WITH_B, bool ADJ, bool S1, bool ST>
__device__ __forceinline__ void load_qrow(const QViews<T, CPL>& v, uint32_t k0, QRowIn<T, CPL>& b) {
    constexpr uint32_t RB = 4 * sizeof(T);
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        if (WITH_B) {
            uint32_t d[RB / 4];
            bld_dw<RB / 4>(d, v.rec, v.orec[c], k0 * RB);
            b.sb[c] = from_dw<T>(d);
            b.bx[c] = from_dw<T>(d + sizeof(T) / 4);
            b.by[c] = from_dw<T>(d + 2 * sizeof(T) / 4);
            b.meta[c] = d[3 * sizeof(T) / 4];
        } else {
            b.meta[c] = bld32(v.rec, v.orec[c] + 3u * (uint32_t)sizeof(T), k0 * RB);
        }
    }
    if (ST) bld_dw<CPL>(b.so, v.off, v.ooff, k0 * 4u);
    if (ADJ && WITH_B) {
        uint32_t d[CPL * 2 * sizeof(T) / 4];
        bld_dw<CPL * 2 * sizeof(T) / 4>(d, v.alt, v.ooff * 2u * (uint32_t)(sizeof(T) / 4), k0 * 2u * (uint32_t)sizeof(T));
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            b.bxo[c] = from_dw<T>(d + 2 * c * sizeof(T) / 4);
            b.byo[c] = from_dw<T>(d + (2 * c + 1) * sizeof(T) / 4);
        }
    }
    if (!S1) {
        uint32_t d[CPL * sizeof(T) / 4];
        bld_dw<CPL * sizeof(T) / 4>(d, v.sg, v.osg, k0 * (uint32_t)sizeof(T));
#pragma unroll
        for (int c = 0; c < CPL; ++c) b.sg[c] = from_dw<T>(d + c * sizeof(T) / 4);
    }
}

// The part of a row's maps that depends neither on the sources nor on the
// row below: Q of each cell, 1 / diagonal, the scan weights t_k = 1 - P of
// the lane's running map before step k, 1 - P of its inclusive map and 1 / P
// of the whole row.  A sweep computes it one row ahead, so the chain from one
// row's solution to the next holds only the A half of the scan.
template <typename T, int CPL>
struct QPart {
    T q[CPL];
    T rdv[CPL];
    T t[6];
    T omP;
    T rPt;
};

// Q, 1 / diagonal of each cell of a row and P of the lane's segment.
template <typename T, int CPL, bool S1, bool FULL>
__device__ __forceinline__ T qpart_cells(const SysC<T>& s, int nx, int lane, const QRowIn<T, CPL>& b,
                                         QPart<T, CPL>& o) {
    const T c0 = s.c[0], c1 = s.c[1], cdiag = s.c[0] + s.c[1];
    // sigma = 1: the cell coefficients are this system's constants
    const T rdv1 = S1 ? recip(T(1) + cdiag) : T(0);
    const T q1 = c0 * rdv1, px1 = (T(1) + c1) * rdv1;
    T Pl;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const T fx = flag<T, 0>(b.meta[c]);
        T rdv, qx, px;
        if (S1) {
            rdv = rdv1; qx = q1; px = px1;
        } else {
            rdv = recip(b.sg[c] + cdiag);
            qx = c0 * rdv;
            px = (b.sg[c] + c1) * rdv;
        }
        T qv = fx * qx;                  // x inflow closed (wall, pore): Q = 0, P = 1
        T pv = fx * px + (T(1) - fx);
        if (!FULL) {
            // beyond the row: the identity (Q, P) = (1, 0)
            const bool bey = lane * CPL + c >= nx;
            qv = bey ? T(1) : qv;
            pv = bey ? T(0) : pv;
        }
        o.q[c] = qv;
        o.rdv[c] = rdv;
        Pl = c == 0 ? pv : pv + qv * Pl;
    }
    return Pl;
}

// 1 - P of the lane's inclusive map and 1 / P of the row (cyclic closure
// x_{-1} = x_{nx-1}; with sigma = 1 every open cell has P > 0, so P_t > 0).
template <typename T, int CPL, bool S1>
__device__ __forceinline__ void qpart_close(T P, QPart<T, CPL>& o) {
    const T Pt = readlane(P, WAVE - 1);
    o.rPt = S1 ? recip(Pt) : (Pt > T(0) ? recip(Pt) : T(0));
    o.omP = T(1) - P;
}

// The P half of the scan alone (the first row of a sweep), recording t_k.
template <typename T>
__device__ __forceinline__ void pscan(T& P, T (&t)[6]) {
    t[0] = T(1) - P; P = P + t[0] * dpp<0x111, 0xf>(P, T(0));   // row_shr:1
    t[1] = T(1) - P; P = P + t[1] * dpp<0x112, 0xf>(P, T(0));   // row_shr:2
    t[2] = T(1) - P; P = P + t[2] * dpp<0x114, 0xf>(P, T(0));   // row_shr:4
    t[3] = T(1) - P; P = P + t[3] * dpp<0x118, 0xf>(P, T(0));   // row_shr:8
    t[4] = T(1) - P; P = P + t[4] * dpp<0x142, 0xa>(P, T(0));   // row_bcast:15 into rows 1, 3
    t[5] = T(1) - P; P = P + t[5] * dpp<0x143, 0xc>(P, T(0));   // row_bcast:31 into rows 2, 3
}

// This row's A scan with its recorded weights t, and the next row's P scan
// recording tn (the same steps as wave_scan; the two chains interleave).
template <typename T>
__device__ __forceinline__ void scan_pair(T& A, const T (&t)[6], T& P, T (&tn)[6]) {
    tn[0] = T(1) - P; A = A + t[0] * dpp<0x111, 0xf>(A, T(0)); P = P + tn[0] * dpp<0x111, 0xf>(P, T(0));
    tn[1] = T(1) - P; A = A + t[1] * dpp<0x112, 0xf>(A, T(0)); P = P + tn[1] * dpp<0x112, 0xf>(P, T(0));
    tn[2] = T(1) - P; A = A + t[2] * dpp<0x114, 0xf>(A, T(0)); P = P + tn[2] * dpp<0x114, 0xf>(P, T(0));
    tn[3] = T(1) - P; A = A + t[3] * dpp<0x118, 0xf>(A, T(0)); P = P + tn[3] * dpp<0x118, 0xf>(P, T(0));
    tn[4] = T(1) - P; A = A + t[4] * dpp<0x142, 0xa>(A, T(0)); P = P + tn[4] * dpp<0x142, 0xa>(P, T(0));
    tn[5] = T(1) - P; A = A + t[5] * dpp<0x143, 0xc>(A, T(0)); P = P + tn[5] * dpp<0x143, 0xc>(P, T(0));
}
// FP32: the same with the DPP read folded into v_fmac (see wave_scan); each
// accumulator's DPP read comes two instructions after its last write.
__device__ __forceinline__ void scan_pair(float& A, const float (&t)[6], float& P, float (&tn)[6]) {
    asm volatile(
        "s_nop 1\n\t"
        "v_sub_f32 %2, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %8 row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %1, %2 row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_sub_f32 %3, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %9 row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %1, %3 row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_sub_f32 %4, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %10 row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %1, %4 row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_sub_f32 %5, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %11 row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %1, %5 row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_sub_f32 %6, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %12 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %1, %6 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_sub_f32 %7, 1.0, %1\n\t"
        "v_fmac_f32_dpp %0, %0, %13 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %1, %7 row_bcast:31 row_mask:0xc bank_mask:0xf"
        : "+v"(A), "+v"(P), "=&v"(tn[0]), "=&v"(tn[1]), "=&v"(tn[2]), "=&v"(tn[3]), "=&v"(tn[4]), "=&v"(tn[5])
        : "v"(t[0]), "v"(t[1]), "v"(t[2]), "v"(t[3]), "v"(t[4]), "v"(t[5]));
}

// One row step of a 2D sweep in the quadrant layout (row jj in y-upwind
// order), with the source-free part qp of this row, and computing qn of the
// next row (inputs nxt).  yp holds the y inflow of each cell of the row: the
// wrap input on the first row, then c_y x of the row below.  mb: per-system
// weights of the boundary values of the inflow faces, mo: of the outflow
// faces (adjoint); sk, sdm: the adjoint's constant source and T_L weight.
template <typename T, int CPL, bool WITH_B, bool RED, bool ADJ, bool S1, int GA, bool FULL, class IO>
__device__ __forceinline__ void qrow_step(const SysC<T>& s, const QViews<T, CPL>& vw, int lane, int jj,
                                          const QRowIn<T, CPL>& cur, const QPart<T, CPL>& qp,
                                          const QRowIn<T, CPL>& nxt, QPart<T, CPL>& qn, T (&yp)[CPL], IO& io,
                                          const T (&mb)[2], const T (&mo)[2], T sk, T sdm, Red<T>* rd,
                                          QRowOut<T, CPL>& ro) {
    const int nx = vw.nx;
    const T c1 = s.c[1];
    T Pn = qpart_cells<T, CPL, S1, FULL>(s, nx, lane, nxt, qn);
    T a[CPL];
    T Al;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const uint32_t mt = cur.meta[c];
        const T fy = flag<T, 1>(mt);
        T rhs;
        if (WITH_B) {
            T base = ADJ ? sk + sdm * cur.sb[c] : cur.sb[c];
            if (ADJ) base += mo[0] * cur.bxo[c] + mo[1] * cur.byo[c];   // + 0 unless S leaves by an outflow face
            rhs = fy * yp[c] + (base + (mb[0] * cur.bx[c] + mb[1] * cur.by[c]));
        } else {
            rhs = fy * yp[c];
        }
        T av = rhs * qp.rdv[c];
        // pores: (A, Q, P) = (0, 0, 1) breaks the chain; their inputs are
        // zero, so only the adjoint's constant source needs the mask
        if (ADJ && WITH_B) av = (mt >> 24) ? av : T(0);
        if (!FULL) av = (lane * CPL + c >= nx) ? T(0) : av;    // beyond the row
        a[c] = av;
        Al = c == 0 ? av : av + qp.q[c] * Al;
    }
    T A = Al;
    scan_pair(A, qp.t, Pn, qn.t);
    qpart_close<T, CPL, S1>(Pn, qn);
    const T At = readlane(A, WAVE - 1);
    const T xin = At * qp.rPt;
    // this lane's last cell, handed to the next lane (lane 0 takes the closure)
    const T xe = A + qp.omP * xin;
    T xp = dpp<0x138, 0xf>(xe, xin);    // wave_shr:1
    T xrow[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const T xv = a[c] + qp.q[c] * xp;
        xrow[c] = (FULL || lane * CPL + c < nx) ? xv : T(0);
        xp = xv;
    }
    if (jj == vw.ny - 1) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) io.out(0, c, lane, xrow[c]);
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) yp[c] = c1 * xrow[c];
    if (RED) {
        // per-lane partials in the compute type (a lane holds at most
        // CPL cells of each row; the systems' sums are taken in double).
        // Pores hold an exact 0; kappa_face sums x over the plane cells (the
        // jump terms are added once per system at the end): with full rows
        // along x the plane cell of a row is its last register
        T rsum = xrow[0];
#pragma unroll
        for (int c = 1; c < CPL; ++c) rsum += xrow[c];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            ro.x[c] = xrow[c];
            ro.so[c] = (FULL || lane * CPL + c < nx) ? cur.so[c] : QOFF_NONE;
        }
        rd->kt += rsum;
        if (GA == 0 && FULL) {
            rd->kft += flag<T, 2>(cur.meta[CPL - 1]) * xrow[CPL - 1];
        } else if (GA == 0 || (GA == 1 && jj == vw.ny - 1)) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) rd->kft += flag<T, 2>(cur.meta[c]) * xrow[c];
        }
    }
}

// (an inactive wave's resources have size 0: its stores are dropped).
// STT: also store the FP64 copy of x (the adjoint's stored forward state).
template <typename T, int CPL, int NR, bool ADD, bool STT>
__device__ __forceinline__ void store_qrows(Red<T>* rd, const QRowOut<T, CPL> (&ro)[NR]) {
    if (STT) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                bst((double)ro[r].x[c], rd->Tstore, ro[r].so[c] * (uint32_t)(8 / sizeof(T)));
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const uint32_t vo = ro[r].so[c];
            T v = ro[r].x[c];
            if (ADD) v += bldT<T>(rd->X, vo, 0);
            bst(v, rd->X, vo);
        }
}

// The 2D upwind sweep in the quadrant layout (see sweep() for the phases'
// use of WITH_B / RED / ADD).
template <typename T, int CPL, bool WITH_B, bool RED, bool ADD, bool ADJ, bool S1, int GA, bool FULL,
          bool STT = false, class IO>
__device__ __forceinline__ void qsweep(const GeomDev& g, const SysC<T>& s, int lane, IO& io, Red<T>* rd) {
    constexpr uint32_t RB = 4 * sizeof(T);
    const int qd = (s.pos[0] ? 0 : 1) | (s.pos[1] ? 0 : 2);
    const uint32_t nc = (uint32_t)g.ncells;
    QViews<T, CPL> vw;
    vw.rec = make_rsrc(static_cast<const char*>(g.qrec) + (size_t)qd * nc * RB, nc * RB);
    vw.off = make_rsrc(g.qoff + (size_t)qd * nc, nc * 4u);
    vw.sg = make_rsrc(static_cast<const T*>(g.qsg) + (size_t)qd * nc, nc * (uint32_t)sizeof(T));
    vw.alt = make_rsrc(static_cast<const T*>(g.qalt) + 2 * (size_t)qd * nc, nc * 2u * (uint32_t)sizeof(T));
#pragma unroll
    for (int c = 0; c < CPL; ++c) vw.orec[c] = (uint32_t)(lane * CPL + c) * RB;
    vw.ooff = (uint32_t)(lane * CPL) * 4u;
    vw.osg = (uint32_t)(lane * CPL) * (uint32_t)sizeof(T);
    vw.nx = uni(g.nx);
    vw.ny = uni(g.ny);
    // per-system weights of the boundary values: forward Lambda |s_a| / h_a
    // on the inflow faces; adjoint the outgoing wall weight of the face S
    // leaves through (the sweep's inflow face, or with a mode table
    // possibly its outflow face)
    T mb[2], mo[2];
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        const int fb = 2 * ax + (s.S[ax] > 0.0 ? 1 : 0);
        const T wv = ADJ ? (T)g.wout[fb * g.n_sys + s.sys] : (T)s.cd[ax];
        const bool in = !ADJ || fb == s.fin[ax];
        mb[ax] = in ? wv : T(0);
        mo[ax] = in ? T(0) : wv;
    }
    const T sk = (T)s.kw, sdm = (T)s.Dml;
    T yp[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) yp[c] = io.in(0, c, lane);
    const int ny = vw.ny;
    // rows are prefetched in order: the first record of the next one is a
    // running scalar
    uint32_t knext = 0;
    const uint32_t nxu = (uint32_t)vw.nx;
    auto pre = [&](int, QRowIn<T, CPL>& b) {
        load_qrow<T, CPL, WITH_B, ADJ, S1, RED>(vw, knext, b);
        knext += nxu;
    };
    auto step = [&](int r, const QRowIn<T, CPL>& b, const QPart<T, CPL>& qp, const QRowIn<T, CPL>& bn,
                    QPart<T, CPL>& qn, QRowOut<T, CPL>& ro) {
        qrow_step<T, CPL, WITH_B, RED, ADJ, S1, GA, FULL>(s, vw, lane, r, b, qp, bn, qn, yp, io, mb, mo, sk, sdm,
                                                           rd, ro);
    };
    // four row buffers: a row's inputs arrive three rows ahead, the
    // source-free part of the next row is taken from them two rows after
    // their loads were issued
    QRowIn<T, CPL> b0, b1, b2, b3;
    QPart<T, CPL> p0, p1, p2, p3;
    if (RED && !ADD) {
        // Each row is stored right after its step, before the prefetch
        // reloads the buffer holding its store offsets.  Vector-memory ops
        // complete in order, so a wait for a prefetched row need not include
        // later stores; but at the loop header the compiler keeps, per
        // register, the most recent position any path gives its load.  So
        // the loop body has no branch (steps past the last row store
        // nothing) and the first group of rows is peeled: the loop is only
        // entered from a copy of its own body, and its waits stay partial.
        pre(0, b0);
        pre(1, b1);
        pre(2, b2);
        {
            T P = qpart_cells<T, CPL, S1, FULL>(s, vw.nx, lane, b0, p0);
            pscan(P, p0.t);
            qpart_close<T, CPL, S1>(P, p0);
        }
        auto sstep = [&](int r, const QRowIn<T, CPL>& b, const QPart<T, CPL>& qp, const QRowIn<T, CPL>& bn,
                         QPart<T, CPL>& qn) {
            QRowOut<T, CPL> ro[1];
            step(r, b, qp, bn, qn, ro[0]);
            // past the last row the inputs read as zeros (x = 0) and the
            // offsets are replaced (a zero offset would address a cell)
#pragma unroll
            for (int c = 0; c < CPL; ++c) ro[0].so[c] = r < ny ? ro[0].so[c] : QOFF_NONE;
            store_qrows<T, CPL, 1, false, STT>(rd, ro);
        };
        auto group = [&](int r) {
            pre(r + 3, b3);
            sstep(r, b0, p0, b1, p1);
            pre(r + 4, b0);
            sstep(r + 1, b1, p1, b2, p2);
            pre(r + 5, b1);
            sstep(r + 2, b2, p2, b3, p3);
            pre(r + 6, b2);
            sstep(r + 3, b3, p3, b0, p0);
        };
        group(0);
        for (int r = 4; r < ny; r += 4) group(r);
    } else {
        pre(0, b0);
        pre(1, b1);
        pre(2, b2);
        {
            T P = qpart_cells<T, CPL, S1, FULL>(s, vw.nx, lane, b0, p0);
            pscan(P, p0.t);
            qpart_close<T, CPL, S1>(P, p0);
        }
        // no stores, or an update of the stored values (four rows of
        // results are added to the stored ones together).  As above, the
        // body has no branch and the first group is peeled: a step past the
        // last row reads zero records, so its x is 0, it adds nothing and
        // stores nothing, and the waits for the prefetched rows stay partial.
        auto gstep = [&](int r, const QRowIn<T, CPL>& b, const QPart<T, CPL>& qp, const QRowIn<T, CPL>& bn,
                         QPart<T, CPL>& qn, QRowOut<T, CPL>& ro) {
            step(r, b, qp, bn, qn, ro);
#pragma unroll
            for (int c = 0; c < CPL; ++c) ro.so[c] = r < ny ? ro.so[c] : QOFF_NONE;
        };
        auto group = [&](int r) {
            QRowOut<T, CPL> ro[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < CPL; ++c) ro[u].so[c] = QOFF_NONE;
            pre(r + 3, b3);
            gstep(r, b0, p0, b1, p1, ro[0]);
            pre(r + 4, b0);
            gstep(r + 1, b1, p1, b2, p2, ro[1]);
            pre(r + 5, b1);
            gstep(r + 2, b2, p2, b3, p3, ro[2]);
            pre(r + 6, b2);
            gstep(r + 3, b3, p3, b0, p0, ro[3]);
            if (RED) store_qrows<T, CPL, 4, ADD, false>(rd, ro);
        };
        group(0);
        for (int r = 4; r < ny; r += 4) group(r);
    }
}

// E' x: inflow of the wrap row from the last row, c_y x_last where the pair
// across the y-wrap is solid.
template <typename T, int CPL, int NZ>
__device__ __forceinline__ void wrap_mask(const GeomDev& g, const SysC<T>& s, int active, int lane,
                                          T (&mk)[NZ][CPL]) {
    const int iy = s.pos[1] ? 0 : g.ny - 1;
#pragma unroll
    for (int k = 0; k < NZ; ++k)
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            mk[k][c] = T(0);
            const int p = lane * CPL + c;
            if (k < g.nz && p < g.nx && active && g.periodic[1]) {
                const int ix = s.pos[0] ? p : g.nx - 1 - p;
                const int iz = (NZ > 1) ? (s.pos[2] ? k : g.nz - 1 - k) : 0;
                const uint32_t w = g.fc[ix + g.nx * (iy + g.ny * iz)];
                if (fc_solid(w) && fc_class(w, s.fin[1]) != FC_WALL) mk[k][c] = s.c[1];
            }
        }
}

template <typename T, int CPL, int NZ>
__device__ __forceinline__ double vdot(const T (&a)[NZ][CPL], const T (&b)[NZ][CPL]) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < NZ; ++k)
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc += (double)a[k][c] * (double)b[k][c];
    return wave_sum(acc);
}

#define VLOOP(body)                                \
    _Pragma("unroll") for (int k = 0; k < NZ; ++k) \
    _Pragma("unroll") for (int c = 0; c < CPL; ++c) { body; }

// Per-system results of a pass: kappa partials and counters.
template <typename T>
__device__ __forceinline__ Red<T> make_red(const GeomDev& g, const SysC<T>& s, int active, const PassParams& pp) {
    Red<T> rd;
    rd.kacc = 0.0;
    rd.kface = 0.0;
    rd.kt = T(0);
    rd.kft = T(0);
    rd.on = active;
    // size 0 for an inactive wave: every store through it is dropped
    rd.X = make_rsrc(reinterpret_cast<T*>(g.X) + (size_t)s.sys * g.xs,
                     active ? (uint32_t)g.nsolid * (uint32_t)sizeof(T) : 0u);
    rd.Tstore = make_rsrc(g.Tstore ? g.Tstore + (size_t)s.sys * g.xs : nullptr,
                          (g.Tstore && active) ? (uint32_t)g.nsolid * 8u : 0u);
    rd.store_T = pp.store_T && g.Tstore != nullptr;
    return rd;
}

template <typename T>
__device__ __forceinline__ void finish_system(const GeomDev& g, const SysC<T>& s, int active, int lane,
                                              int adj, const PassParams& pp, const Red<T>& rd,
                                              long long n_it, long long n_sw) {
    const double ks = wave_sum(rd.kacc + (double)rd.kt), kf = wave_sum(rd.kface + (double)rd.kft);
    if (active && lane == 0) {
        if (adj) {
            g.ksys[s.sys] = kf;                 // this system's share of p^T lambda
            g.kfsys[s.sys] = 0.0;
        } else {
            g.kraw[s.sys] = ks;
            g.ksys[s.sys] = g.L[g.grad_axis] / (g.dT * (double)g.ncells) * s.Sg * ks;
            g.kfsys[s.sys] = g.L[g.grad_axis] / (g.dT * (double)g.n_perp) * s.Sg * kf;
        }
        if (pp.mode == 0) {
            g.iters[s.sys] += n_it;
            g.sweeps[s.sys] += n_sw;
        }
    }
}

// ---------------------------------------------------------------------------
// One outer pass for every work item (block = one item = W systems sharing a
// direction, so their table and source loads touch the same lines).  Phase
// A: each wave sweeps with the sources b and the previous wrap inflow u0 and
// stores its solution.  Phase B: each wave corrects its wrap inflow
// (BiCGSTAB on the wrap row).  Phase C: a wave that
// changed u sweeps the source P (u - u0) and adds the (linear) response to
// its stored solution.
// ---------------------------------------------------------------------------
// One system's pass (wave w of work item `item`; w is wave-uniform, so every
// per-system quantity and the buffer resources built from it are scalars).
template <typename T, int CPL, int ADJ, int SIG1, bool FULL>
__device__ __forceinline__ void pass_system(const GeomDev* __restrict__ geoms, const Item& item, int w,
                                            int lane, const PassParams& pp) {
    constexpr int NZ = 1;      // 2D: the wrap row is one x-row, held in registers
    const GeomDev& g = geoms[item.geom];
    if (pp.mode == 0 && g.ctrl[CTRL_DONE]) return;
    const int m = item.m0 + w;
    const int active = (w < item.nm) && (m < g.n_mfp);
    constexpr int adj = ADJ;     // the adjoint's branches fold at compile time
    const SysC<T> s = make_sys<T>(g, active ? m : item.m0, item.l, adj);
    const size_t half = adj ? (size_t)g.n_sys : 0;
    T* Uall = reinterpret_cast<T*>(g.U) + half * g.nwrap;

    T u[NZ][CPL], xl[NZ][CPL], mk[NZ][CPL];
    wrap_mask<T, CPL, NZ>(g, s, active, lane, mk);
    VLOOP({
        const int p = lane * CPL + c;
        u[k][c] = (active && k < g.nz && p < g.nx) ? Uall[(size_t)s.sys * g.nwrap + k * g.nx + p] : T(0);
    });
    Red<T> rd = make_red<T>(g, s, active, pp);
    // ---- phase A
    {
        RegIO<T, CPL> io{u[0], xl[0]};
        // the forward's replay that keeps its state stores an FP64 copy too
        const bool stt = ADJ == 0 && rd.store_T;
        if (g.grad_axis == 0) {
            if (stt) qsweep<T, CPL, true, true, false, ADJ != 0, SIG1 != 0, 0, FULL, ADJ == 0>(g, s, lane, io, &rd);
            else qsweep<T, CPL, true, true, false, ADJ != 0, SIG1 != 0, 0, FULL>(g, s, lane, io, &rd);
        } else {
            if (stt) qsweep<T, CPL, true, true, false, ADJ != 0, SIG1 != 0, 1, FULL, ADJ == 0>(g, s, lane, io, &rd);
            else qsweep<T, CPL, true, true, false, ADJ != 0, SIG1 != 0, 1, FULL>(g, s, lane, io, &rd);
        }
    }
    long long n_it = 0, n_sw = 1;
    int need = 0;
    T du[NZ][CPL];
    VLOOP(du[k][c] = T(0));
    const bool has_wrap = g.periodic[1] != 0;
    if (pp.mode == 0 && active && has_wrap) {
        // ---- phase B: residual of the wrap system for the inflow u0 just used
        T r[NZ][CPL], ez[NZ][CPL];
        VLOOP({ ez[k][c] = mk[k][c] * xl[k][c]; r[k][c] = ez[k][c] - u[k][c]; });
        const double scale = sqrt(vdot<T, CPL, NZ>(ez, ez));
        double rn = sqrt(vdot<T, CPL, NZ>(r, r));
        // target of this pass: inner_tol relative to the inflow, or (forcing)
        // a reduction by inner_rtol of the residual the pass started from
        const double thr = fmax(pp.inner_tol * scale, pp.inner_rtol * rn);
        const double thr_final = pp.inner_tol * scale;
        if (rn > thr_final && scale > 0.0) need = 1;
        const double rho_g = wrap_gain_bound(g, s);
        if (rn > thr && scale > 0.0 && rho_g * rn <= fmin(thr, fmax(thr_final, RICH_MAX * rn))) {
            // a weakly coupled wrap (short MFP along y): e = r leaves the
            // residual G r, at most rho_g |r|, within this pass's target and
            // below RICH_MAX |r| (or the final tolerance), with no sweep
            VLOOP(du[k][c] = r[k][c]);
            rn = rho_g * rn;
        } else if (rn > thr && scale > 0.0) {
            // BiCGSTAB for the remaining correction: (I - G) e = r.  A capped
            // BiCGSTAB is not monotone, so the iterate with the smallest
            // residual is kept: a pass never increases the wrap residual.
            T e[NZ][CPL], eb[NZ][CPL], rh[NZ][CPL], p[NZ][CPL], v[NZ][CPL], sv[NZ][CPL], t[NZ][CPL];
            VLOOP({ e[k][c] = T(0); eb[k][c] = T(0); rh[k][c] = r[k][c]; p[k][c] = T(0); v[k][c] = T(0); });
            double best = rn;
            int restarts = 0;
            double rho_old = 1.0, alpha = 1.0, omega = 1.0;
            for (int iter = 0; iter < pp.max_inner; ++iter) {
                double rho = vdot<T, CPL, NZ>(rh, r);
                if (fabs(rho) <= 1e-30 * rn * rn || !(omega != 0.0)) {
                    VLOOP({ rh[k][c] = r[k][c]; p[k][c] = T(0); v[k][c] = T(0); });
                    rho = vdot<T, CPL, NZ>(r, r);
                    rho_old = 1.0; alpha = 1.0; omega = 1.0;
                }
                const double beta = (rho / rho_old) * (alpha / omega);
                VLOOP(p[k][c] = r[k][c] + (T)beta * (p[k][c] - (T)omega * v[k][c]));
                {
                    RegIO<T, CPL> io{p[0], xl[0]};
                    qsweep<T, CPL, false, false, false, ADJ != 0, SIG1 != 0, -1, FULL>(g, s, lane, io, nullptr);
                }
                ++n_sw;
                VLOOP(v[k][c] = p[k][c] - mk[k][c] * xl[k][c]);
                const double rv = vdot<T, CPL, NZ>(rh, v);
                if (!isfinite(rv)) break;
                if (!(fabs(rv) > 1e-30 * fabs(rho))) {
                    // breakdown (shadow residual orthogonal to A p): restart
                    // from the current residual on the next iteration
                    if (restarts++ >= 4) break;
                    omega = 0.0;
                    continue;
                }
                alpha = rho / rv;
                VLOOP(sv[k][c] = r[k][c] - (T)alpha * v[k][c]);
                const double sn = sqrt(vdot<T, CPL, NZ>(sv, sv));
                ++n_it;
                if (sn <= thr) {
                    VLOOP(e[k][c] += (T)alpha * p[k][c]);
                    if (sn < best) { best = sn; VLOOP(eb[k][c] = e[k][c]); }
                    break;
                }
                {
                    RegIO<T, CPL> io{sv[0], xl[0]};
                    qsweep<T, CPL, false, false, false, ADJ != 0, SIG1 != 0, -1, FULL>(g, s, lane, io, nullptr);
                }
                ++n_sw;
                VLOOP(t[k][c] = sv[k][c] - mk[k][c] * xl[k][c]);
                const double tt = vdot<T, CPL, NZ>(t, t);
                omega = tt > 0.0 ? vdot<T, CPL, NZ>(t, sv) / tt : 0.0;
                VLOOP(e[k][c] += (T)alpha * p[k][c] + (T)omega * sv[k][c]);
                VLOOP(r[k][c] = sv[k][c] - (T)omega * t[k][c]);
                rn = sqrt(vdot<T, CPL, NZ>(r, r));
                rho_old = rho;
                if (!isfinite(rn)) break;
                if (rn < best) { best = rn; VLOOP(eb[k][c] = e[k][c]); }
                if (rn <= thr) break;
            }
            rn = best;
            VLOOP(du[k][c] += eb[k][c]);
        }
        if (lane == 0) g.wres[s.sys] = scale > 0.0 ? rn / scale : 0.0;
        if (need) {
            VLOOP({
                const int pp_ = lane * CPL + c;
                if (k < g.nz && pp_ < g.nx) Uall[(size_t)s.sys * g.nwrap + k * g.nx + pp_] = u[k][c] + du[k][c];
            });
        }
    }
    // ---- phase C: correction sweep of a wave that moved its inflow (skipped
    // when the correction is lagged into the next pass)
    if (!pp.lag_wrap && need) {
        RegIO<T, CPL> io{du[0], xl[0]};
        if (g.grad_axis == 0)
            qsweep<T, CPL, false, true, true, ADJ != 0, SIG1 != 0, 0, FULL>(g, s, lane, io, &rd);
        else
            qsweep<T, CPL, false, true, true, ADJ != 0, SIG1 != 0, 1, FULL>(g, s, lane, io, &rd);
        ++n_sw;
    }
    // kappa_face: the sweeps summed x over the plane cells.  The forward adds
    // the jump dT once per plane cell when it crosses the plane towards +
    // (the image there is hotter); the adjoint weighs its jump faces by
    // Lambda |s_a| / h_a dT, with the sign of the jump (the '+' face's image
    // is colder)
    {
        // (selects, not a run-time index: that would put s in scratch memory)
        const bool ga0 = g.grad_axis == 0;
        const int qd = (s.pos[0] ? 0 : 1) | (s.pos[1] ? 0 : 2);
        const bool pos = ga0 ? s.pos[0] : s.pos[1];
        const double cd = ga0 ? s.cd[0] : s.cd[1];
        rd.kface += (double)rd.kft;
        rd.kft = T(0);
        if (adj) rd.kface *= (pos ? -1.0 : 1.0) * cd * g.dT;
        else if (lane == 0 && pos) rd.kface += g.dT * (double)g.qnk[qd];
    }
    finish_system(g, s, active, lane, adj, pp, rd, n_it, n_sw);
}

// Threads per workgroup of a 2D pass kernel: FP64 rows of 3 or 4 cells per
// lane hold more registers than two waves per SIMD leave (they spilled to
// scratch), so those kernels take at most 4 waves per group (the host caps
// the systems per workgroup to match).
template <typename T, int CPL>
constexpr int pass_threads() { return (sizeof(T) == 8 && CPL >= 3) ? 256 : 512; }

// The 2D pass: one workgroup per work item, one of its systems per wave.
template <typename T, int CPL, int ADJ, int SIG1, bool FULL>
__global__ void __launch_bounds__((pass_threads<T, CPL>())) k_sweep_pass(const GeomDev* __restrict__ geoms,
                                                    const Item* __restrict__ items, int n_items,
                                                    PassParams pp) {
    const int it = blockIdx.x;
    if (it >= n_items) return;
    pass_system<T, CPL, ADJ, SIG1, FULL>(geoms, items[it], __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
                                         threadIdx.x & 63, pp);
}

// The 2D pass over every work item of a batch in one persistent launch: a
// workgroup takes the next item from a device-side queue (an atomic counter,
// set to 0 by the pack kernel before every pass) until none is left and runs
// it with its geometry's cells-per-lane body, so the items of every launch
// class share one grid (ordered longest MFPs first over all geometries).
// The waves of a group never wait for each other inside an item; the two
// barriers only order the group's read of the slot against its next write.
template <typename T, int ADJ, int SIG1>
__global__ void __launch_bounds__((pass_threads<T, 4>())) k_sweep_queue(const GeomDev* __restrict__ geoms,
                                                     const Item* __restrict__ items, int n_items,
                                                     PassParams pp, int* __restrict__ queue) {
    __shared__ int slot;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) slot = atomicAdd(queue, 1);
        __syncthreads();
        const int it = slot;
        if (it >= n_items) return;                     // every wave of the group leaves together
        const Item item = items[it];
        switch ((geoms[item.geom].nx + WAVE - 1) / WAVE) {
            case 1: pass_system<T, 1, ADJ, SIG1, false>(geoms, item, w, lane, pp); break;
            case 2: pass_system<T, 2, ADJ, SIG1, false>(geoms, item, w, lane, pp); break;
            case 3: pass_system<T, 3, ADJ, SIG1, false>(geoms, item, w, lane, pp); break;
            default: pass_system<T, 4, ADJ, SIG1, false>(geoms, item, w, lane, pp); break;
        }
    }
}

// ---------------------------------------------------------------------------
// The 3D pass.  Same phases as the 2D kernel; the wrap plane of a system
// (nx * nz values) is too large for registers, so its Krylov vectors live in
// a per-system slab of the workspace (KV_N planes).  Every element (k, p) is
// read and written only by the lane owning column p, as in the sweep.
// ---------------------------------------------------------------------------
enum { KV_XL, KV_MK, KV_DU, KV_R, KV_E, KV_EB, KV_RH, KV_P, KV_V, KV_S, KV_T, KV_N };
static_assert(KV_N == KRY3_VECS, "workspace carve and kernel disagree on the 3D slab");

#define PLOOP(body)                                     \
    for (int k = 0; k < nz; ++k)                        \
        _Pragma("unroll") for (int c = 0; c < CPL; ++c) { \
            const int p_ = lane * CPL + c;              \
            if (p_ < nx) {                              \
                const int i = k * nx + p_;              \
                body;                                   \
            }                                           \
        }

template <typename T, int CPL, int ADJ, int SIG1, bool FULL>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(CPL == 1 ? (sizeof(T) == 4 ? 5 : 4) : 1))) k_sweep_pass3(const GeomDev* __restrict__ geoms,
                                                     const Item* __restrict__ items, int n_items,
                                                     PassParams pp) {
    extern __shared__ double lds[];
    const int it = blockIdx.x;
    if (it >= n_items) return;
    const Item item = items[it];
    const GeomDev& g = geoms[item.geom];
    if (pp.mode == 0 && g.ctrl[CTRL_DONE]) return;
    // the wave index is wave-uniform: read it into a scalar so that every
    // per-system quantity (and the buffer resources built from it) is too
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = item.m0 + w;
    const int active = (w < item.nm) && (m < g.n_mfp);
    constexpr int adj = ADJ;
    const SysC<T> s = make_sys<T>(g, active ? m : item.m0, item.l, adj);
    // the pass's sources and inflow tables, converted to the compute type by
    // k_pack3 before the pass
    const T* srcbase = static_cast<const T*>(g.qrec);
    const T* bnd = srcbase + g.ncells;
    const int nx = g.nx, nz = g.nz, nw = g.nwrap;
    const size_t half = adj ? (size_t)g.n_sys : 0;
    const gmut_t<T> U = gmut(reinterpret_cast<T*>(g.U) + (half + s.sys) * (size_t)nw);
    const gmut_t<T> K = gmut(reinterpret_cast<T*>(g.kry) + (size_t)s.sys * KV_N * nw);
    const gmut_t<T> xl = K + (size_t)KV_XL * nw;
    const gmut_t<T> du = K + (size_t)KV_DU * nw;
    // per-wave LDS: nz rows of this wave
    T* zrows = reinterpret_cast<T*>(lds) + (size_t)w * nz * WAVE * CPL;
    Red<T> rd = make_red<T>(g, s, active, pp);
    // ---- phase A
    {
        GlobIO<T, CPL> io = make_gio<T, CPL>(U, xl, nx, nz, active);
        if (g.grad_axis == 0)
            sweep<T, CPL, true, true, true, false, SIG1 != 0, 0, FULL>(g, s, active, lane, adj, srcbase, bnd, io, &rd, zrows);
        else
            sweep<T, CPL, true, true, true, false, SIG1 != 0, 1, FULL>(g, s, active, lane, adj, srcbase, bnd, io, &rd, zrows);
    }
    long long n_it = 0, n_sw = 1;
    int need = 0;
    const bool has_wrap = g.periodic[1] != 0;
    if (pp.mode == 0 && active && has_wrap) {
        const gmut_t<T> mk = K + (size_t)KV_MK * nw;
        const gmut_t<T> r = K + (size_t)KV_R * nw;
        const gmut_t<T> e = K + (size_t)KV_E * nw;
        const gmut_t<T> eb = K + (size_t)KV_EB * nw;
        const gmut_t<T> rh = K + (size_t)KV_RH * nw;
        const gmut_t<T> p = K + (size_t)KV_P * nw;
        const gmut_t<T> v = K + (size_t)KV_V * nw;
        const gmut_t<T> sv = K + (size_t)KV_S * nw;
        const gmut_t<T> t = K + (size_t)KV_T * nw;
        // wrap mask E' (c_y where the pair across the y-wrap is solid), the
        // inflow produced by the sweep and the residual of the wrap system
        const int iy = s.pos[1] ? 0 : g.ny - 1;
        double ss = 0.0, rr = 0.0;
        PLOOP({
            const int ix = s.pos[0] ? p_ : nx - 1 - p_;
            const int iz = s.pos[2] ? k : nz - 1 - k;
            const uint32_t wv = g.fc[ix + nx * (iy + g.ny * iz)];
            const T mv = (fc_solid(wv) && fc_class(wv, s.fin[1]) != FC_WALL) ? s.c[1] : T(0);
            mk[i] = mv;
            const T ez = mv * xl[i];
            const T rv = ez - U[i];
            r[i] = rv;
            du[i] = T(0);
            ss += (double)ez * (double)ez;
            rr += (double)rv * (double)rv;
        });
        const double scale = sqrt(wave_sum(ss));
        double rn = sqrt(wave_sum(rr));
        const double thr = fmax(pp.inner_tol * scale, pp.inner_rtol * rn);
        const double thr_final = pp.inner_tol * scale;
        if (rn > thr_final && scale > 0.0) need = 1;
        const double rho_g = wrap_gain_bound(g, s);
        if (rn > thr && scale > 0.0 && rho_g * rn <= fmin(thr, fmax(thr_final, RICH_MAX * rn))) {
            // weakly coupled wrap: e = r, no sweep (as in 2D)
            PLOOP(du[i] = r[i]);
            rn = rho_g * rn;
        } else if (rn > thr && scale > 0.0) {
            // BiCGSTAB on (I - G) e = r with the best iterate kept (as in 2D)
            PLOOP({ e[i] = T(0); eb[i] = T(0); rh[i] = r[i]; p[i] = T(0); v[i] = T(0); });
            double best = rn;
            int restarts = 0;
            double rho_old = 1.0, alpha = 1.0, omega = 1.0;
            for (int iter = 0; iter < pp.max_inner; ++iter) {
                double acc = 0.0;
                PLOOP(acc += (double)rh[i] * (double)r[i]);
                double rho = wave_sum(acc);
                if (fabs(rho) <= 1e-30 * rn * rn || !(omega != 0.0)) {
                    acc = 0.0;
                    PLOOP({ rh[i] = r[i]; p[i] = T(0); v[i] = T(0); acc += (double)r[i] * (double)r[i]; });
                    rho = wave_sum(acc);
                    rho_old = 1.0; alpha = 1.0; omega = 1.0;
                }
                const double beta = (rho / rho_old) * (alpha / omega);
                PLOOP(p[i] = r[i] + (T)beta * (p[i] - (T)omega * v[i]));
                {
                    GlobIO<T, CPL> io = make_gio<T, CPL>(p, xl, nx, nz, 1);
                    sweep<T, CPL, true, false, false, false, SIG1 != 0, -1, FULL>(g, s, active, lane, adj, srcbase, bnd, io, nullptr, zrows);
                }
                ++n_sw;
                acc = 0.0;
                PLOOP({
                    const T vv = p[i] - mk[i] * xl[i];
                    v[i] = vv;
                    acc += (double)rh[i] * (double)vv;
                });
                const double rv = wave_sum(acc);
                if (!isfinite(rv)) break;
                if (!(fabs(rv) > 1e-30 * fabs(rho))) {
                    if (restarts++ >= 4) break;
                    omega = 0.0;
                    continue;
                }
                alpha = rho / rv;
                acc = 0.0;
                PLOOP({
                    const T x = r[i] - (T)alpha * v[i];
                    sv[i] = x;
                    acc += (double)x * (double)x;
                });
                const double sn = sqrt(wave_sum(acc));
                ++n_it;
                if (sn <= thr) {
                    PLOOP(e[i] += (T)alpha * p[i]);
                    if (sn < best) {
                        best = sn;
                        PLOOP(eb[i] = e[i]);
                    }
                    break;
                }
                {
                    GlobIO<T, CPL> io = make_gio<T, CPL>(sv, xl, nx, nz, 1);
                    sweep<T, CPL, true, false, false, false, SIG1 != 0, -1, FULL>(g, s, active, lane, adj, srcbase, bnd, io, nullptr, zrows);
                }
                ++n_sw;
                double tt = 0.0, ts = 0.0;
                PLOOP({
                    const T x = sv[i] - mk[i] * xl[i];
                    t[i] = x;
                    tt += (double)x * (double)x;
                    ts += (double)x * (double)sv[i];
                });
                tt = wave_sum(tt);
                ts = wave_sum(ts);
                omega = tt > 0.0 ? ts / tt : 0.0;
                acc = 0.0;
                PLOOP({
                    e[i] += (T)alpha * p[i] + (T)omega * sv[i];
                    const T x = sv[i] - (T)omega * t[i];
                    r[i] = x;
                    acc += (double)x * (double)x;
                });
                rn = sqrt(wave_sum(acc));
                rho_old = rho;
                if (!isfinite(rn)) break;
                if (rn < best) {
                    best = rn;
                    PLOOP(eb[i] = e[i]);
                }
                if (rn <= thr) break;
            }
            rn = best;
            PLOOP(du[i] += eb[i]);
        }
        if (lane == 0) g.wres[s.sys] = scale > 0.0 ? rn / scale : 0.0;
        if (need) PLOOP(U[i] += du[i]);
    }
    // ---- phase C (see the 2D kernel)
    if (!pp.lag_wrap && need) {
        GlobIO<T, CPL> io = make_gio<T, CPL>(du, nullptr, nx, nz, 0);
        if (g.grad_axis == 0)
            sweep<T, CPL, true, false, true, true, SIG1 != 0, 0, FULL>(g, s, active, lane, adj, srcbase, bnd, io, &rd, zrows);
        else
            sweep<T, CPL, true, false, true, true, SIG1 != 0, 1, FULL>(g, s, active, lane, adj, srcbase, bnd, io, &rd, zrows);
        ++n_sw;
    }
    finish_system(g, s, active, lane, adj, pp, rd, n_it, n_sw);
}
#undef PLOOP

// ---------------------------------------------------------------------------
// Per-cell / per-wall sums over the systems' stored solutions (fixed order)
// and the next pass's inputs sigma T_L and T_w.  Forward: T_L = sum D x and
// T_w = sum ReLu(S.n)/sum ReLu(S.n) x at the wall cell.  Adjoint: Psi = sigma
// sum lambda and Phi_f = sum of c_a lambda over the directions entering
// through f (the transpose of the wall coupling).  A block owns a strip of RC
// solid cells (consecutive solid indices: one 128-byte segment of a system's
// FP32 values); each of its RQ waves holds the strip twice (lanes 0-31 and
// 32-63), and the 2 RQ half-waves split the systems in fixed chunks, so twice
// as many loads are in flight per strip as with one chunk per wave.  A
// half-wave stages the weights of RC systems at a time in LDS (D, or 1 in
// the adjoint, and the wall weights), zero beyond its chunk, so every
// half-wave runs the same trip count, in groups of RG in-range loads.  A wall face reads
// only its own cell's values, so the walls of the strip's cells are summed
// from the same loads.  Every sum is combined over the chunks in order.
// Pore entries of the outputs are never written: they are set to 0 once per
// solve (k_prep_sigma) and stay 0.
// ---------------------------------------------------------------------------
constexpr int RQ = 16;      // waves per reduction block
constexpr int RC = 32;      // solid cells per strip
constexpr int RH = 2 * RQ;  // system chunks per strip: one per half-wave
constexpr int RG = 16;      // loads in flight per lane: systems per group
static_assert(RC == 32 && RC % RG == 0 && RG % 4 == 0, "a strip is one half of a wave, read in groups of RG systems");

template <typename T>
__global__ void __launch_bounds__(64 * RQ) k_reduce_pass(const GeomDev* __restrict__ geoms, PassParams pp) {
    __shared__ double wt[RH][7][RC];       // per half-wave: row 0 D (or 1), rows 1..6 the wall weights
    __shared__ double part[RH][RC];
    const GeomDev& g = geoms[blockIdx.y];
    if (g.ctrl[CTRL_DONE] && pp.mode == 0) return;
    const int pass = g.ctrl[CTRL_PASS];
    const int out = (pass + 1) & 1;
    const int adj = pp.adjoint;
    const int nc = g.ncells, nf = g.nf, ns = g.n_sys, nd = g.n_dir, nsol = g.nsolid, xs = g.xs;
    if ((int)blockIdx.x * RC >= nsol) return;          // block-uniform
    const gptr_t<T> X = gview(reinterpret_cast<const T*>(g.X));
    const gptr_t<double> D = gview(g.Dw);
    const int q = threadIdx.x >> 6, cl = threadIdx.x & 63;
    const int h = cl >> 5, c = cl & (RC - 1);
    const int hq = 2 * q + h;                           // this half-wave's chunk
    const int j = blockIdx.x * RC + c;                  // solid index of this lane
    const bool in = j < nsol;
    const int js = in ? j : nsol - 1;                   // in-range loads, dropped below
    const int cell = in ? g.scell[j] : -1;
    const int per = (ns + RH - 1) / RH;                 // the same trip count in every chunk
    const int i0 = hq * per, i1 = min(ns, i0 + per);
    // wall faces of this lane's cell (bit f), and of the strip: the same in
    // every wave of the block
    int wm = 0;
    if (in) {
        const uint16_t w = g.fc[cell];
        for (int f = 0; f < nf; ++f) wm |= (fc_class(w, f) == FC_WALL ? 1 : 0) << f;
    }
    int wany = wm;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) wany |= shfl_xor(wany, m);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    double aw[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < per; r += RC) {
        // lane c of the half-wave: the weights of system i0 + r + c (forward
        // walls: ReLu(S.n) / sum; adjoint walls: c_a of the directions
        // entering through the face)
        const int is = i0 + r + c;
        const bool lv = is < i1;
        const int il = lv ? is : ns - 1;
        wt[hq][0][c] = lv ? (adj ? 1.0 : D[il]) : 0.0;
        if (wany) {
            double cf[6];
            if (!adj) {
#pragma unroll
                for (int f = 0; f < 6; ++f) cf[f] = g.wout[(size_t)min(f, nf - 1) * ns + il];
            } else {
                const int m = il / nd, l = il - m * nd;
                const double mf = g.mfp[m];
                const double sd3[3] = {g.dirs[l * 3], g.dirs[l * 3 + 1], g.dirs[l * 3 + 2]};
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const int ax = f >> 1;
                    const double sd = sd3[ax];
                    const double nsgn = (f & 1) ? 1.0 : -1.0;
                    cf[f] = sd * nsgn < 0.0 ? mf * fabs(sd) / g.h[ax] : 0.0;
                }
            }
#pragma unroll
            for (int f = 0; f < 6; ++f)
                if (f < nf && ((wany >> f) & 1)) wt[hq][1 + f][c] = lv ? cf[f] : 0.0;
        }
        // the wave reads back its own rows (LDS ops of a wave complete in order)
        __builtin_amdgcn_wave_barrier();
        // groups of RG systems: past the chunk's end the weights are 0 and the
        // loads stay in range
        const int nb = min(RC, (per - r + RG - 1) & ~(RG - 1));
        const int ib = i0 + r;
        for (int u0 = 0; u0 < nb; u0 += RG) {
            double xv[RG];
#pragma unroll
            for (int u = 0; u < RG; ++u) xv[u] = (double)X[(size_t)min(ib + u0 + u, ns - 1) * xs + js];
#pragma unroll
            for (int u = 0; u < RG; u += 4) {
                a0 += wt[hq][0][u0 + u] * xv[u];
                a1 += wt[hq][0][u0 + u + 1] * xv[u + 1];
                a2 += wt[hq][0][u0 + u + 2] * xv[u + 2];
                a3 += wt[hq][0][u0 + u + 3] * xv[u + 3];
            }
            if (wany) {
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    if (f >= nf || !((wany >> f) & 1)) continue;
                    const double* cp = &wt[hq][1 + f][u0];
#pragma unroll
                    for (int u = 0; u < RG; ++u) aw[f] += cp[u] * xv[u];   // zero weight: + 0
                }
            }
        }
        // this round's weights are read before the next round writes them
        __builtin_amdgcn_wave_barrier();
    }
    part[hq][c] = in ? (a0 + a1) + (a2 + a3) : 0.0;
    __syncthreads();
    const bool head = q == 0 && h == 0;                 // lanes 0..RC-1 of wave 0 write
    if (head && in) {
        double tot = part[0][c];
#pragma unroll
        for (int u = 1; u < RH; ++u) tot += part[u][c];
        if (!adj) g.T_L[cell] = tot;
        if (g.aa_m > 0) {
            g.ag[cell] = tot;              // the mixing step writes the next inputs
        } else {
            g.ax[cell] = tot;
            if (adj) g.lam_psi[(size_t)out * nc + cell] = g.sigma[cell] * tot;
            else g.sT[(size_t)out * nc + cell] = g.sigma[cell] * tot;
        }
    }
    if (!wany) return;                     // block-uniform
    double* bnd_out = g.bnd + ((size_t)(adj ? 2 : 0) + out) * nf * nc;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (f >= nf || !((wany >> f) & 1)) continue;
        __syncthreads();                   // the previous sum's reads are done
        part[hq][c] = aw[f];
        __syncthreads();
        if (head && ((wm >> f) & 1)) {
            double a = part[0][c];
#pragma unroll
            for (int u = 1; u < RH; ++u) a += part[u][c];
            const int wi = g.wall_idx[cell * nf + f];
            if (g.aa_m > 0) {
                g.ag[nc + wi] = a;
            } else {
                g.ax[nc + wi] = a;
                if (adj) g.lam_phi[(size_t)out * g.nwalls + wi] = a;
                else g.Tw[(size_t)out * g.nwalls + wi] = a;
                bnd_out[(size_t)f * nc + cell] = a;
            }
        }
    }
}

// kappa, history and the convergence test of Algorithm 1 (one block per geometry).
__global__ void k_finalize(const GeomDev* __restrict__ geoms, PassParams pp) {
    __shared__ double red[56];
    const GeomDev& g = geoms[blockIdx.x];
    if (g.ctrl[CTRL_DONE]) return;
    double k = 0.0, kf = 0.0, wr = 0.0;
    const int ns = g.n_sys, bd = blockDim.x;
    // thread t takes t, t + bd, ... in that order, 8 loads of each in flight
    for (int i0 = threadIdx.x; i0 < ns; i0 += 8 * bd) {
        double a[8], b[8], c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = min(i0 + u * bd, ns - 1);
            a[u] = g.ksys[i];
            b[u] = g.kfsys[i];
            c[u] = g.wres[i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + u * bd < ns) {
                k += a[u];
                kf += b[u];
                wr = fmax(wr, c[u]);
            }
    }
    // fixed-order: every thread sums a fixed strided subset, then block_sum
    block_sum2(k, kf, red);
    // max of the wrap residuals (every value is >= 0: max via the sum of a
    // one-hot is not needed, a plain block max suffices)
    __syncthreads();
    {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        for (int m2 = 32; m2 >= 1; m2 >>= 1) wr = fmax(wr, shfl_xor(wr, m2));
        if (lane == 0) red[36 + wid] = wr;
        __syncthreads();
        wr = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) wr = fmax(wr, red[36 + i]);
    }
    if (threadIdx.x == 0) {
        const int pass = g.ctrl[CTRL_PASS];
        if (pass >= pp.max_outer) {      // history is sized for max_outer passes
            g.ctrl[CTRL_DONE] = 1;
            return;
        }
        g.hist[pass] = k;
        g.hist_face[pass] = kf;
        g.wres_hist[pass] = wr;
        const int n = pass + 1;
        g.ctrl[CTRL_PASS] = n;
        // Algorithm 1's test on the relative change of kappa; with a bounded
        // number of inner iterations per pass the wrap rows must be solved too
        const bool wrap_ok = wr <= pp.wrap_tol;
        bool small = n >= 2 && fabs(k - g.hist[pass - 1]) <= pp.outer_tol * fabs(k);
        if (pp.stop_rule == 1) {
            // error estimate of a linear fixed-point iteration: the
            // contraction is the largest of the last two ratios of
            // successive changes and of the mean ratio over ten passes (the
            // window sees through a transient or noisy pair)
            small = false;
            if (n >= 12) {
                const double d0 = fabs(k - g.hist[pass - 1]);
                const double d1 = fabs(g.hist[pass - 1] - g.hist[pass - 2]);
                const double d2 = fabs(g.hist[pass - 2] - g.hist[pass - 3]);
                const double d10 = fabs(g.hist[pass - 10] - g.hist[pass - 11]);
                double rho = fmax(d1 > 0.0 ? d0 / d1 : 0.0, d2 > 0.0 ? d1 / d2 : 0.0);
                if (d10 > 0.0) rho = fmax(rho, pow(d0 / d10, 0.1));
                rho = fmin(rho, 0.995);
                small = d0 * rho / (1.0 - rho) <= pp.outer_tol * fabs(k);
            }
        }
        // with mixing, successive kappa can agree before the iterate has
        // settled: the error estimated from the fixed-point residual must
        // meet the tolerance too
        if (g.aa_m > 0) small = small && g.fscal[3] <= pp.outer_tol;
        if (!isfinite(k)) {
            g.ctrl[CTRL_NONFINITE] = 1;
            g.ctrl[CTRL_DONE] = 1;
        } else if (wrap_ok && small) {
            g.ctrl[CTRL_CONVERGED] = 1;
            g.ctrl[CTRL_DONE] = 1;
        } else if (n >= pp.max_outer) {
            g.ctrl[CTRL_DONE] = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Anderson mixing of the outer fixed point x -> G(x).  The pass computed
// G(x_k); with f_k = G(x_k) - x_k and the last aa_m differences dX, dF of
// iterates and residuals,
//   gamma = argmin |f_k - dF gamma|,   x_{k+1} = x_k + f_k - (dX + dF) gamma
// (gamma from the normal equations of the column-scaled dF, Cholesky in
// double; a failed factorisation drops the history and takes the plain step
// x_{k+1} = G(x_k)).  Two kernels over up to AAB_MAX blocks per geometry:
// the first stores the new difference column and the per-block partial dot
// products, the second sums them in a fixed order, solves the small system
// in every block (the same numbers everywhere), and writes the next pass's
// inputs: sigma T_L (or sigma sum lambda), the wall values and their inflow
// table entries.  The history counters are double buffered by pass parity.
// ---------------------------------------------------------------------------
constexpr int AAB_MAX = 256, AA_THREADS = 256, AA_NP = 2 * AA_MAX + 3;

struct AView {
    int n, B, c0, c1;
};
__device__ __forceinline__ AView aa_view(const GeomDev& g, int b) {
    AView v;
    v.n = g.n_aa;
    v.B = min(AAB_MAX, (v.n + AA_THREADS - 1) / AA_THREADS);
    const int chunk = (v.n + v.B - 1) / v.B;
    v.c0 = min(v.n, b * chunk);
    v.c1 = min(v.n, v.c0 + chunk);
    return v;
}

__global__ void __launch_bounds__(AA_THREADS) k_aa_partial(const GeomDev* __restrict__ geoms) {
    __shared__ double red[AA_NP][AA_THREADS / 64];
    const GeomDev& g = geoms[blockIdx.y];
    if (g.aa_m <= 0 || g.ctrl[CTRL_DONE]) return;
    const AView v = aa_view(g, blockIdx.x);
    if ((int)blockIdx.x >= v.B) return;
    const int n = v.n, M = g.aa_m;
    const int* ac = g.actl + 4 * (g.ctrl[CTRL_PASS] & 1);
    const int cnt = ac[0], head = ac[1], have = ac[2];
    const int slot = head;                            // the new column (when have)
    const int cnt1 = have ? min(cnt + 1, M) : cnt;    // valid columns: 0 .. cnt1-1
    double dA[AA_MAX], db[AA_MAX];
#pragma unroll
    for (int j = 0; j < AA_MAX; ++j) { dA[j] = 0.0; db[j] = 0.0; }
    double ff = 0.0, xx = 0.0, dxx = 0.0;
    for (int i = v.c0 + threadIdx.x; i < v.c1; i += blockDim.x) {
        // every load first (the stored columns from in-range slots, unused
        // ones dropped below), so they are in flight together
        const double x = g.ax[i], gi = g.ag[i], fp = g.afp[i], xp = g.axp[i];
        double hF[AA_MAX];
#pragma unroll
        for (int j = 0; j < AA_MAX; ++j) hF[j] = g.adF[(size_t)min(j, M - 1) * n + i];
        const double f = gi - x;
        xx += x * x;
        ff += f * f;
        double df = 0.0;
        if (have) {
            df = f - fp;
            const double dx = x - xp;
            dxx += dx * dx;
            g.adX[(size_t)slot * n + i] = dx;
            g.adF[(size_t)slot * n + i] = df;
        }
        g.axp[i] = x;
        g.afp[i] = f;
#pragma unroll
        for (int j = 0; j < AA_MAX; ++j) {
            if (j < cnt1) {
                const double Fj = (have && j == slot) ? df : hF[j];
                db[j] += Fj * f;
                if (have) dA[j] += df * Fj;
            }
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double sums[AA_NP];
#pragma unroll
    for (int j = 0; j < AA_MAX; ++j) {
        sums[j] = dA[j];
        sums[AA_MAX + j] = db[j];
    }
    sums[2 * AA_MAX] = ff;
    sums[2 * AA_MAX + 1] = xx;
    sums[2 * AA_MAX + 2] = dxx;
    wave_sum_n(sums);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < AA_NP; ++q) red[q][wid] = sums[q];
    __syncthreads();
    if (threadIdx.x < AA_NP) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[threadIdx.x][w];
        g.apart[(size_t)blockIdx.x * AA_NP + threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(AA_THREADS) k_aa_apply(const GeomDev* __restrict__ geoms, PassParams pp) {
    __shared__ double tot[AA_NP];
    __shared__ double wred[AA_NP][AA_THREADS / 64];
    __shared__ double gam[AA_MAX];
    const GeomDev& g = geoms[blockIdx.y];
    if (g.aa_m <= 0 || g.ctrl[CTRL_DONE]) return;
    const AView v = aa_view(g, blockIdx.x);
    if ((int)blockIdx.x >= v.B) return;
    const int n = v.n, M = g.aa_m, nc = g.ncells;
    const int adj = pp.adjoint;
    const int par = g.ctrl[CTRL_PASS] & 1;
    const int out = par ^ 1;                           // pass input buffers of the next pass
    const int* ac = g.actl + 4 * par;
    const int cnt = ac[0], head = ac[1], have = ac[2];
    const int slot = head;
    const int cnt1 = have ? min(cnt + 1, M) : cnt;
    // fixed-order sums of the per-block partials: thread b holds block b's
    // row (B <= blockDim), a butterfly per wave, then the waves in order
    {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
        const bool mine = (int)threadIdx.x < v.B;
        const double* row = g.apart + (size_t)(mine ? threadIdx.x : 0) * AA_NP;
        double sums[AA_NP];
#pragma unroll
        for (int q = 0; q < AA_NP; ++q) sums[q] = row[q];
#pragma unroll
        for (int q = 0; q < AA_NP; ++q) sums[q] = mine ? sums[q] : 0.0;
        wave_sum_n(sums);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < AA_NP; ++q) wred[q][wid] = sums[q];
        __syncthreads();
        if ((int)threadIdx.x < AA_NP) {
            double t = 0.0;
            for (int w = 0; w < nw; ++w) t += wred[threadIdx.x][w];
            tot[threadIdx.x] = t;
        }
        __syncthreads();
    }
    // The small least-squares solve on the first wave, one lane per entry of
    // the AA_MAX x AA_MAX Gram matrix: lane t holds entry (r, k) = (t / 8,
    // t % 8) and the vectors' entry j = t % 8.  Every loop runs over the
    // fixed AA_MAX; rows and columns beyond cnt1 are identity rows.
    static_assert(AA_MAX * AA_MAX == WAVE, "one lane per Gram matrix entry");
    if (threadIdx.x < WAVE) {
        const int t = threadIdx.x, r = t / AA_MAX, k = t % AA_MAX, j = k;
        const double* dxg = g.agram + M * M;            // |dX_j|^2 of the stored columns
        // this pass's Gram matrix: the new column's row from the partials,
        // the rest from the stored matrix (block 0 stores the new row)
        double a = r == k ? 1.0 : 0.0;
        if (r < cnt1 && k < cnt1) {
            const bool fresh = have && (r == slot || k == slot);
            a = fresh ? tot[r == slot ? k : r] : g.agram[r * M + k];
        }
        const bool vj = j < cnt1;
        const double dxn = vj ? ((have && j == slot) ? tot[2 * AA_MAX + 2] : dxg[j]) : 0.0;
        const double bj = vj ? tot[AA_MAX + j] : 0.0;
        const double gjj = shfl_at(a, (AA_MAX + 1) * j);
        if (blockIdx.x == 0 && have && t < cnt1) {
            const double val = tot[t];                  // new column against column t
            g.agram[slot * M + t] = val;
            g.agram[t * M + slot] = val;
            if (t == 0) g.agram[M * M + slot] = tot[2 * AA_MAX + 2];
        }
        // error estimate for the stop test: with f = (G - I) e for a linear G,
        // |e| <= |f| / s_min(I - G); s_min is estimated by the smallest
        // |dF_j| / |dX_j| over the stored columns (no columns: |f| itself)
        double sm = (vj && dxn > 0.0) ? sqrt(gjj / dxn) : 1.0;
#pragma unroll
        for (int m = 1; m < AA_MAX; m <<= 1) sm = fmin(sm, shfl_xor(sm, m));
        const double smin = fmax(fmin(sm, 1.0), 1e-3);
        const double sf = tot[2 * AA_MAX], sx = tot[2 * AA_MAX + 1];
        const double res = sx > 0.0 ? sqrt(sf / sx) : (sf > 0.0 ? INFINITY : 0.0);
        if (blockIdx.x == 0 && t == 0) g.fscal[3] = res / smin;
        // scaled normal equations with a small ridge, Cholesky in place
        // (right-looking: step p finishes column p and updates the trailing
        // block), then the two triangular solves; ok is wave-uniform
        const double dj = vj ? sqrt(gjj) : 1.0;
        bool ok = cnt1 > 0 && __all(dj > 0.0 && isfinite(dj));
        double y = 0.0;
        if (ok) {
            const double dr = shfl_at(dj, r);
            a = a / (dr * dj) + ((r == k && r < cnt1) ? 1e-10 : 0.0);
#pragma unroll
            for (int p = 0; p < AA_MAX; ++p) {
                const double s2 = shfl_at(a, (AA_MAX + 1) * p);
                ok = ok && s2 > 1e-14;
                const double lpp = sqrt(fmax(s2, 1e-300));
                if (k == p) a = r == p ? lpp : (r > p ? a / lpp : a);
                const double lr = shfl_at(a, AA_MAX * r + p), lk = shfl_at(a, AA_MAX * k + p);
                if (r > p && k > p && k <= r) a -= lr * lk;
            }
            y = bj / dj;
#pragma unroll
            for (int p = 0; p < AA_MAX; ++p) {
                const double yp = shfl_at(y, p) / shfl_at(a, (AA_MAX + 1) * p);
                const double ljp = shfl_at(a, AA_MAX * j + p);
                y = j == p ? yp : (j > p ? y - ljp * yp : y);
            }
#pragma unroll
            for (int p = AA_MAX - 1; p >= 0; --p) {
                const double zp = shfl_at(y, p) / shfl_at(a, (AA_MAX + 1) * p);
                const double lpj = shfl_at(a, AA_MAX * p + j);
                y = j == p ? zp : (j < p ? y - lpj * zp : y);
            }
            y = vj ? y / dj : 0.0;
            ok = ok && __all(isfinite(y));
        }
        if (t < AA_MAX) gam[t] = ok ? y : 0.0;
        if (blockIdx.x == 0 && t == 0) {
            int* ao = g.actl + 4 * out;
            if (ok || cnt1 == 0) {
                ao[0] = cnt1;
                ao[1] = have ? (slot + 1) % M : head;
            } else {          // drop the history; the next pass starts a new one
                ao[0] = 0;
                ao[1] = 0;
            }
            ao[2] = 1;
        }
    }
    __syncthreads();
    double* bnd_out = g.bnd + ((size_t)(adj ? 2 : 0) + out) * g.nf * nc;
    for (int i = v.c0 + threadIdx.x; i < v.c1; i += blockDim.x) {
        double hX[AA_MAX], hF[AA_MAX];       // loaded together, unused slots dropped
#pragma unroll
        for (int j = 0; j < AA_MAX; ++j) {
            const size_t o = (size_t)min(j, M - 1) * n + i;
            hX[j] = g.adX[o];
            hF[j] = g.adF[o];
        }
        double xn = g.axp[i] + g.afp[i];
#pragma unroll
        for (int j = 0; j < AA_MAX; ++j)
            if (j < cnt1) xn -= gam[j] * (hX[j] + hF[j]);
        if (i < nc) {
            const bool sol = fc_solid(g.fc[i]);
            xn = sol ? xn : 0.0;
            const double sx = sol ? g.sigma[i] * xn : 0.0;
            if (adj) g.lam_psi[(size_t)out * nc + i] = sx;
            else g.sT[(size_t)out * nc + i] = sx;
        } else {
            const int wi = i - nc;
            if (adj) g.lam_phi[(size_t)out * g.nwalls + wi] = xn;
            else g.Tw[(size_t)out * g.nwalls + wi] = xn;
            bnd_out[(size_t)g.wall_face[wi] * nc + g.wall_cell[wi]] = xn;
        }
        g.ax[i] = xn;
    }
}

// ---------------------------------------------------------------------------
// Fourier first guess: CG on the negated 5/7-point finite-volume Laplacian
// with adiabatic pores and the periodic jump (Appendix B on the structured
// grid), spread over up to FB_MAX blocks per geometry.  One kernel per
// iteration (the Chronopoulos-Gear arrangement of CG, below); it sums the
// per-block partials of the previous one in a fixed order (no atomics), so
// every block of a geometry takes the same decisions, and a converged
// geometry's blocks exit at once.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fourier_rhs(const GeomDev& g, uint16_t w, const double (&kf)[3]) {
    double b = 0.0;
    if (fc_solid(w))
        for (int f = 0; f < g.nf; ++f) {
            const int cl = fc_class(w, f);
            if (cl == FC_JUMP_P) b += kf[f >> 1] * g.dT;
            else if (cl == FC_JUMP_M) b -= kf[f >> 1] * g.dT;
        }
    return b;
}

constexpr int FB_MAX = 256, FB_THREADS = 256;

// This geometry's CG storage (in the fx region) and block b's cell range.
// r, s = A r and q = A p are double buffered by iteration parity; gp / dp hold
// the per-block partials of (r, r) and (r, s) by parity.  sc: [0] |b|, [1]
// done, [4] iterations, [6 + q] iterations done before an iteration of
// parity q, [8 + q] its (r, r) and [10 + q] its alpha.
// (the buffers are selected by ternaries, never by a run-time array index,
// which would put the view in private memory)
struct FView {
    double *x, *p, *r0, *r1, *s0, *s1, *q0, *q1, *gp0, *gp1, *dp0, *dp1, *sc;
    int n, B, c0, c1;
    __device__ double* r(int k) const { return k ? r1 : r0; }
    __device__ double* s(int k) const { return k ? s1 : s0; }
    __device__ double* q(int k) const { return k ? q1 : q0; }
    __device__ double* gp(int k) const { return k ? gp1 : gp0; }
    __device__ double* dp(int k) const { return k ? dp1 : dp0; }
};
__device__ __forceinline__ FView fourier_view(const GeomDev& g, int b) {
    FView v;
    const int n = g.ncells;
    v.n = n;
    v.B = min(FB_MAX, (n + FB_THREADS - 1) / FB_THREADS);
    double* f = g.fx;
    v.x = f;
    v.p = f + n;
    v.r0 = f + 2 * (size_t)n;
    v.r1 = f + 3 * (size_t)n;
    v.s0 = f + 4 * (size_t)n;
    v.s1 = f + 5 * (size_t)n;
    v.q0 = f + 6 * (size_t)n;
    v.q1 = f + 7 * (size_t)n;
    double* pt = f + 8 * (size_t)n;
    v.gp0 = pt;
    v.gp1 = pt + FB_MAX;
    v.dp0 = pt + 2 * FB_MAX;
    v.dp1 = pt + 3 * FB_MAX;
    v.sc = pt + 4 * FB_MAX;
    const int chunk = (n + v.B - 1) / v.B;
    v.c0 = min(n, b * chunk);
    v.c1 = min(n, v.c0 + chunk);
    return v;
}

__device__ __forceinline__ double axis_pick(double k0, double k1, double k2, int a) {
    return a == 0 ? k0 : (a == 1 ? k1 : k2);
}

// fixed-order sum of the B per-block partials, returned to every thread
__device__ __forceinline__ double sum_partials(const double* part, int B, double* red) {
    double t = 0.0;
    for (int i = threadIdx.x; i < B; i += blockDim.x) t += part[i];
    return block_sum(t, red);
}

// two of them in one pass (red: at least 34 doubles)
__device__ __forceinline__ void sum_partials2(const double* p, const double* q, int B, double* red, double& sp,
                                              double& sq) {
    sp = 0.0;
    sq = 0.0;
    for (int i = threadIdx.x; i < B; i += blockDim.x) {
        sp += p[i];
        sq += q[i];
    }
    block_sum2(sp, sq, red);
}

__global__ void __launch_bounds__(FB_THREADS) k_fourier_init(const GeomDev* __restrict__ geoms) {
    __shared__ double red[40];
    const GeomDev& g = geoms[blockIdx.y];
    const FView v = fourier_view(g, blockIdx.x);
    if ((int)blockIdx.x >= v.B) return;
    double kf[3];
    for (int a = 0; a < 3; ++a) kf[a] = (a < g.ndim) ? g.kappa_axis[a] / (g.h[a] * g.h[a]) : 0.0;
    // start from the linear profile T = -dT (i + 1/2) / n along the gradient
    // axis: the exact solution without pores, so the first residual lives
    // only next to pore faces
    const int ga = g.grad_axis;
    const double ng = (double)(ga == 0 ? g.nx : g.ny);
    auto lin = [&](int c) {
        const int i = ga == 0 ? c % g.nx : (c / g.nx) % g.ny;
        return -g.dT * ((double)i + 0.5) / ng;
    };
    double s = 0.0, bb = 0.0;
    for (int c = v.c0 + threadIdx.x; c < v.c1; c += blockDim.x) {
        const uint16_t w = g.fc[c];
        const CellPos cp = cell_pos(g, c);
        const double b = fourier_rhs(g, w, kf);
        double x0 = 0.0, r0 = 0.0;
        if (fc_solid(w)) {
            x0 = lin(c);
            double y = 0.0;
            for (int f = 0; f < g.nf; ++f)
                if (fc_class(w, f) != FC_WALL) y += kf[f >> 1] * (x0 - lin(nbr_cell(g, c, cp, f)));
            r0 = b - y;
        }
        v.x[c] = x0;
        v.r(0)[c] = r0;
        v.p[c] = 0.0;
        v.q(0)[c] = 0.0;
        s += r0 * r0;
        bb += b * b;
    }
    block_sum2(s, bb, red);
    if (threadIdx.x == 0) {
        v.gp(0)[blockIdx.x] = s;
        v.dp(1)[blockIdx.x] = bb;            // |b|^2 partials, read by k_fourier_norm
        if (blockIdx.x == 0) {
            v.sc[1] = 0.0;
            v.sc[4] = 0.0;
            v.sc[6] = 0.0;
        }
    }
}

// |b| of every geometry (one block each); a zero first residual is converged
__global__ void __launch_bounds__(FB_THREADS) k_fourier_norm(const GeomDev* __restrict__ geoms) {
    __shared__ double red[40];
    const GeomDev& g = geoms[blockIdx.x];
    const FView v = fourier_view(g, 0);
    double bb, rr;
    sum_partials2(v.dp(1), v.gp(0), v.B, red, bb, rr);
    if (threadIdx.x == 0) {
        v.sc[0] = sqrt(bb);
        if (!(bb > 0.0) || !(rr > 0.0)) v.sc[1] = 1.0;
    }
}

__device__ __forceinline__ void fourier_k(const GeomDev& g, double& k0, double& k1, double& k2) {
    k0 = g.kappa_axis[0] / (g.h[0] * g.h[0]);
    k1 = g.ndim > 1 ? g.kappa_axis[1] / (g.h[1] * g.h[1]) : 0.0;
    k2 = g.ndim > 2 ? g.kappa_axis[2] / (g.h[2] * g.h[2]) : 0.0;
}

// s_0 = A r_0 and the partials of (r_0, s_0).
__global__ void __launch_bounds__(FB_THREADS) k_fourier_s0(const GeomDev* __restrict__ geoms) {
    __shared__ double red[40];
    const GeomDev& g = geoms[blockIdx.y];
    const FView v = fourier_view(g, blockIdx.x);
    if ((int)blockIdx.x >= v.B) return;
    double k0, k1, k2;
    fourier_k(g, k0, k1, k2);
    const double* r = v.r(0);
    double d = 0.0;
    for (int c = v.c0 + threadIdx.x; c < v.c1; c += blockDim.x) {
        const uint16_t w = g.fc[c];
        const CellPos cp = cell_pos(g, c);
        double y = 0.0;
        if (fc_solid(w))
            for (int f = 0; f < g.nf; ++f) {
                if (fc_class(w, f) == FC_WALL) continue;
                y += axis_pick(k0, k1, k2, f >> 1) * (r[c] - r[nbr_cell(g, c, cp, f)]);
            }
        v.s(0)[c] = y;
        d += r[c] * y;
    }
    d = block_sum(d, red);
    if (threadIdx.x == 0) v.dp(0)[blockIdx.x] = d;
}

// One CG iteration in the Chronopoulos-Gear arrangement: s = A r and q = A p
// are carried by recurrence, so both inner products of an iteration, gamma =
// (r, r) and delta = (r, A r), come from one pass over the cells:
//   beta_k = gamma_k / gamma_{k-1},  alpha_k = gamma_k / (delta_k - beta_k
//   gamma_k / alpha_{k-1})  (k = 0: beta = 0, alpha = gamma / delta),
//   p = r + beta p,  q = s + beta q,  x += alpha p,  r' = r - alpha q,
//   s' = A r'  and the partials of (r', r'), (r', s').
// Iteration k (parity qq) reads r_k, s_k, q_{k-1} from buffers qq and writes
// r_{k+1}, s_{k+1}, q_k into buffers qq ^ 1; A r' at a cell needs r' at its
// neighbours, which every block forms itself from the unchanged buffers qq.
// The stop test (every block computes the same sums) is the one of the plain
// CG: |r_k| <= tol |b|, or max_iter iterations.
__global__ void __launch_bounds__(FB_THREADS) k_fourier_cg(const GeomDev* __restrict__ geoms, int qq,
                                                         double tol, int max_iter) {
    __shared__ double red[40];
    const GeomDev& g = geoms[blockIdx.y];
    const FView v = fourier_view(g, blockIdx.x);
    if ((int)blockIdx.x >= v.B || v.sc[1] != 0.0) return;
    double gam, del;
    sum_partials2(v.gp(qq), v.dp(qq), v.B, red, gam, del);
    const int it = (int)v.sc[6 + qq];
    if (!(sqrt(gam) > tol * v.sc[0]) || it >= max_iter) {
        if (blockIdx.x == 0 && threadIdx.x == 0) v.sc[1] = 1.0;
        return;
    }
    double alpha = gam / del, beta = 0.0;
    if (it > 0) {
        beta = gam / v.sc[8 + (qq ^ 1)];
        alpha = gam / (del - beta * gam / v.sc[10 + (qq ^ 1)]);
    }
    double k0, k1, k2;
    fourier_k(g, k0, k1, k2);
    const int nf = g.nf;
    const double *r = v.r(qq), *s = v.s(qq), *qo = v.q(qq);
    double *rn = v.r(qq ^ 1), *sn = v.s(qq ^ 1), *qn = v.q(qq ^ 1);
    double gs = 0.0, ds = 0.0;
    for (int c = v.c0 + threadIdx.x; c < v.c1; c += blockDim.x) {
        const uint16_t w = g.fc[c];
        const CellPos cp = cell_pos(g, c);
        double rc = 0.0, sa = 0.0, qc = 0.0;
        if (fc_solid(w)) {
            const double pc = r[c] + beta * v.p[c];
            v.p[c] = pc;
            qc = s[c] + beta * qo[c];
            v.x[c] += alpha * pc;
            rc = r[c] - alpha * qc;
            for (int f = 0; f < nf; ++f) {
                if (fc_class(w, f) == FC_WALL) continue;
                const int j = nbr_cell(g, c, cp, f);
                const double rj = r[j] - alpha * (s[j] + beta * qo[j]);
                sa += axis_pick(k0, k1, k2, f >> 1) * (rc - rj);
            }
        }
        rn[c] = rc;
        sn[c] = sa;
        qn[c] = qc;
        gs += rc * rc;
        ds += rc * sa;
    }
    block_sum2(gs, ds, red);
    if (threadIdx.x == 0) {
        v.gp(qq ^ 1)[blockIdx.x] = gs;
        v.dp(qq ^ 1)[blockIdx.x] = ds;
        if (blockIdx.x == 0) {
            v.sc[8 + qq] = gam;
            v.sc[10 + qq] = alpha;
            v.sc[6 + (qq ^ 1)] = (double)(it + 1);
            v.sc[4] = (double)(it + 1);
        }
    }
}

// geometries still iterating -> *pending (one block)
__global__ void __launch_bounds__(256) k_fourier_pending(const GeomDev* __restrict__ geoms, int n_geoms,
                                                        int* pending) {
    __shared__ double red[32];
    double c = 0.0;
    for (int i = threadIdx.x; i < n_geoms; i += blockDim.x) c += fourier_view(geoms[i], 0).sc[1] == 0.0 ? 1.0 : 0.0;
    c = block_sum(c, red);
    if (threadIdx.x == 0) *pending = (int)c;
}

// End of the Fourier solve, in two kernels over the geometry's cell blocks.
// The first stores per-block partials of the solid-cell sum of x and count
// (the mean, which the gauge removes) and of the plane flux through the
// periodic plane of the gradient axis (kappa_F; differences of x, so the mean
// drops out) in the CG's direction buffers, free once it has ended.  The
// second sums them in a fixed order in every block and writes the mean-free
// T_F as T_L, sigma T_F, the wall temperatures, the first iterate of the
// outer fixed point and the inflow tables: periodic jumps +-dT (fixed), walls
// T_w (updated every pass), interior 0; forward buffers 0 and 1, adjoint
// buffers 2 and 3 (no jump source; walls updated per pass).  A wall's first
// temperature is its cell's, so buffer 0's wall entries take the cell value.
// Block 0 also stores kappa_F and the CG statistics and resets the pass
// control words.
__global__ void __launch_bounds__(FB_THREADS) k_fourier_part(const GeomDev* __restrict__ geoms) {
    __shared__ double red[32];
    const GeomDev& g = geoms[blockIdx.y];
    const FView v = fourier_view(g, blockIdx.x);
    if ((int)blockIdx.x >= v.B) return;
    const int ga = g.grad_axis;
    const double* x = g.fx;
    double sx = 0.0, ns = 0.0, fl = 0.0;
    for (int c = v.c0 + threadIdx.x; c < v.c1; c += blockDim.x) {
        const uint16_t w = g.fc[c];
        if (!fc_solid(w)) continue;
        sx += x[c];
        ns += 1.0;
        const int f = 2 * ga;   // '-' face of the cell at index 0
        if (fc_class(w, f) == FC_JUMP_P) {
            const int j = nbr_cell(g, c, cell_pos(g, c), f);
            fl += g.kappa_axis[ga] * (x[j] + g.dT - x[c]) / g.h[ga];
        }
    }
    sx = block_sum(sx, red);
    ns = block_sum(ns, red);
    fl = block_sum(fl, red);
    if (threadIdx.x == 0) {
        v.s(0)[blockIdx.x] = sx;
        v.s(1)[blockIdx.x] = ns;
        v.q(0)[blockIdx.x] = fl;
    }
}

__global__ void __launch_bounds__(FB_THREADS) k_fourier_fill(const GeomDev* __restrict__ geoms) {
    __shared__ double red[40];
    const GeomDev& g = geoms[blockIdx.y];
    const FView v = fourier_view(g, blockIdx.x);
    if ((int)blockIdx.x >= v.B) return;
    const int n = g.ncells, nf = g.nf;
    double sx, sn;
    sum_partials2(v.s(0), v.s(1), v.B, red, sx, sn);
    const double mean = sx / sn;
    if (blockIdx.x == 0) {
        const int it = (int)v.sc[4];
        const double rn = sqrt(sum_partials(v.gp(it & 1), v.B, red));
        const double fl = sum_partials(v.q(0), v.B, red);
        const double bn = v.sc[0];
        const int ga = g.grad_axis;
        if (g.aa_m > 0 && threadIdx.x < 8) g.actl[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            g.fscal[0] = g.L[ga] / (g.dT * (double)g.n_perp) * fl;
            g.fscal[1] = (double)it;
            g.fscal[2] = bn > 0.0 ? rn / bn : 0.0;
            for (int i = 0; i < CTRL_N; ++i) g.ctrl[i] = 0;
        }
    }
    const double* x = g.fx;
    const size_t nb = (size_t)nf * n;
    for (int c = v.c0 + threadIdx.x; c < v.c1; c += blockDim.x) {
        const uint16_t w = g.fc[c];
        const bool sol = fc_solid(w);
        const double t = sol ? x[c] - mean : 0.0;
        g.T_L[c] = t;
        g.sT[c] = sol ? g.sigma[c] * t : 0.0;   // buffer 0
        g.ax[c] = t;
        for (int f = 0; f < nf; ++f) {
            const int cl = sol ? fc_class(w, f) : FC_INTERIOR;
            const double jv = cl == FC_JUMP_P ? g.dT : (cl == FC_JUMP_M ? -g.dT : 0.0);
            const size_t e = (size_t)f * n + c;
            g.bnd[e] = cl == FC_WALL ? t : jv;
            g.bnd[nb + e] = jv;
            g.bnd[2 * nb + e] = 0.0;
            g.bnd[3 * nb + e] = 0.0;
        }
    }
    for (int wi = blockIdx.x * blockDim.x + threadIdx.x; wi < g.nwalls; wi += v.B * blockDim.x) {
        const double t = x[g.wall_cell[wi]] - mean;
        g.Tw[wi] = t;
        g.ax[n + wi] = t;
    }
}

// sigma per cell (1 where not given or in pores) and its float copy; the
// pore entries of the per-cell pass arrays, which the reduction and the
// mixing never write, are set to 0 (the solid entries are left as they are,
// so a resumed solve keeps its state).
__global__ void __launch_bounds__(256) k_prep_sigma(const GeomDev* __restrict__ gp, const double* __restrict__ sig_in) {
    __shared__ double red[4];
    const GeomDev& g = *gp;
    const int nc = g.ncells;
    double vmin = INFINITY;         // smallest sigma over this block's solid cells
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
        const bool sol = fc_solid(g.fc[c]);
        double v = 1.0;
        if (sig_in && sol) v = sig_in[c];
        if (sol) vmin = fmin(vmin, v);
        g.sigma[c] = v;
        g.sigma_f[c] = (float)v;
        if (!sol) {
            g.T_L[c] = 0.0;
            g.sT[c] = 0.0;
            g.sT[nc + c] = 0.0;
            g.lam_psi[c] = 0.0;
            g.lam_psi[nc + c] = 0.0;
            g.ax[c] = 0.0;
            if (g.aa_m > 0) {
                g.ag[c] = 0.0;
                g.axp[c] = 0.0;
                g.afp[c] = 0.0;
            }
        }
    }
    for (int m = 32; m >= 1; m >>= 1) vmin = fmin(vmin, shfl_xor(vmin, m));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = vmin;
    __syncthreads();
    if (threadIdx.x == 0) g.fx[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// Smallest sigma over the solid cells into fscal[5]: the minimum of the
// per-block minima k_prep_sigma left in fx (one block).  The pass kernels
// bound the gain of a system's wrap map with it (see wrap_gain_bound).
__global__ void __launch_bounds__(256) k_sigma_min(const GeomDev* __restrict__ gp, int nblocks) {
    __shared__ double red[4];
    const GeomDev& g = *gp;
    double v = INFINITY;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v = fmin(v, g.fx[b]);
    for (int m = 32; m >= 1; m >>= 1) v = fmin(v, shfl_xor(v, m));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) g.fscal[5] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// Flux map of one geometry from the stored solutions of the replayed last
// sweep: J_i = sum_ml S_ml x_iml (one thread per cell, systems in order).
template <typename T>
__global__ void __launch_bounds__(256) k_flux(const GeomDev* __restrict__ gp, double* J_out) {
    const GeomDev& g = *gp;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncells) return;
    const int i = g.sidx[c];
    const gptr_t<T> X = gview(reinterpret_cast<const T*>(g.X));
    double j[3] = {0.0, 0.0, 0.0};
    if (i >= 0)
        for (int sys = 0; sys < g.n_sys; ++sys) {
            const double x = (double)X[(size_t)sys * g.xs + i];
#pragma unroll
            for (int a = 0; a < 3; ++a) j[a] += g.S[sys * 3 + a] * x;
        }
    for (int a = 0; a < g.ndim; ++a) J_out[(size_t)c * g.ndim + a] = j[a];
}

// Adjoint gradient of one geometry: -sum_ml lambda_iml (T_iml - T_L,i) from
// the stored adjoint solutions and the stored forward state.
template <typename T>
__global__ void __launch_bounds__(256) k_grad(const GeomDev* __restrict__ gp, double* grad_out) {
    const GeomDev& g = *gp;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncells) return;
    const int i = g.sidx[c];
    const gptr_t<T> X = gview(reinterpret_cast<const T*>(g.X));
    const double tl = g.T_L[c];
    double acc = 0.0;
    if (i >= 0)
        for (int sys = 0; sys < g.n_sys; ++sys) {
            const size_t e = (size_t)sys * g.xs + i;
            acc += (double)X[e] * (g.Tstore[e] - tl);
        }
    grad_out[c] = i >= 0 ? -acc : 0.0;
}

// Energy balance of the last pass (paper, section Model: T_L is fixed by
// energy conservation, sum_ml alpha_ml sigma_i (T_iml - T_L,i) = 0 at the
// fixed point).  With alpha = D sum alpha the residual of cell i is
// sum alpha |sigma_i sum_ml D_ml T_iml - sigma_i T_L,i^in|, measured against
// the mean weighted magnitude sum alpha sum_i sum_ml D_ml |T_iml| / N_solid;
// sum alpha cancels.  One block per 64 solid cells writes its maximum and its
// sum; k_energy_finish combines them in a fixed order into fscal[4].
constexpr int EQ = 16;      // waves per energy block: system chunks of one 64-cell strip

template <typename T>
__global__ void __launch_bounds__(64 * EQ) k_energy(const GeomDev* __restrict__ gp) {
    __shared__ double pm[EQ][64], ps[EQ][64];
    const GeomDev& g = *gp;
    const int nsol = g.nsolid, ns = g.n_sys, xs = g.xs;
    const int q = threadIdx.x >> 6, cl = threadIdx.x & 63;
    const int j = blockIdx.x * 64 + cl;
    const bool in = j < nsol;
    const int js = in ? j : nsol - 1;           // in-range loads, dropped below
    const gptr_t<T> X = gview(reinterpret_cast<const T*>(g.X));
    const gptr_t<double> D = gview(g.Dw);
    const int per = (ns + EQ - 1) / EQ;
    const int i0 = q * per, i1 = min(ns, i0 + per);
    double t[4] = {0.0, 0.0, 0.0, 0.0}, a[4] = {0.0, 0.0, 0.0, 0.0};
    int i = i0;
    for (; i + 3 < i1; i += 4) {
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = (double)X[(size_t)(i + u) * xs + js];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            t[u] += D[i + u] * x[u];
            a[u] += D[i + u] * fabs(x[u]);
        }
    }
    for (; i < i1; ++i) {
        const double x = (double)X[(size_t)i * xs + js];
        t[0] += D[i] * x;
        a[0] += D[i] * fabs(x);
    }
    pm[q][cl] = (t[0] + t[1]) + (t[2] + t[3]);
    ps[q][cl] = (a[0] + a[1]) + (a[2] + a[3]);
    __syncthreads();
    if (q == 0) {
        double tl = 0.0, ab = 0.0, r = 0.0;
#pragma unroll
        for (int u = 0; u < EQ; ++u) {
            tl += pm[u][cl];
            ab += ps[u][cl];
        }
        if (in) {
            const int cell = g.scell[j];
            const int buf = (g.ctrl[CTRL_PASS] + 1) & 1;     // the last pass's input
            r = fabs(g.sigma[cell] * tl - g.sT[(size_t)buf * g.ncells + cell]);
        } else {
            ab = 0.0;
        }
        for (int m = 32; m >= 1; m >>= 1) {
            r = fmax(r, shfl_xor(r, m));
            ab += shfl_xor(ab, m);
        }
        if (cl == 0) {
            g.fx[2 * blockIdx.x] = r;
            g.fx[2 * blockIdx.x + 1] = ab;
        }
    }
}

__global__ void __launch_bounds__(256) k_energy_finish(const GeomDev* __restrict__ gp, int nblocks) {
    __shared__ double red[40];
    const GeomDev& g = *gp;
    double r = 0.0, ab = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        r = fmax(r, g.fx[2 * b]);
        ab += g.fx[2 * b + 1];
    }
    for (int m = 32; m >= 1; m >>= 1) r = fmax(r, shfl_xor(r, m));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = r;
    __syncthreads();
    double rm = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) rm = fmax(rm, red[w]);
    __syncthreads();
    ab = block_sum(ab, red);
    if (threadIdx.x == 0) {
        const double mean = g.nsolid > 0 ? ab / (double)g.nsolid : 0.0;
        g.fscal[4] = mean > 0.0 ? rm / mean : 0.0;
    }
}

// Lattice temperature of one geometry with the solid-cell mean removed.
__global__ void __launch_bounds__(1024) k_output(const GeomDev* __restrict__ gp, double* T_L_out) {
    __shared__ double red[32];
    const GeomDev& g = *gp;
    const int n = g.ncells;
    if (T_L_out) {
        double sx = 0.0, ns = 0.0;
        for (int c = threadIdx.x; c < n; c += blockDim.x)
            if (fc_solid(g.fc[c])) { sx += g.T_L[c]; ns += 1.0; }
        sx = block_sum(sx, red);
        ns = block_sum(ns, red);
        const double mean = ns > 0.0 ? sx / ns : 0.0;
        for (int c = threadIdx.x; c < n; c += blockDim.x)
            T_L_out[c] = fc_solid(g.fc[c]) ? g.T_L[c] - mean : 0.0;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static_assert(fourier_scratch_doubles(0) == 4 * FB_MAX + 16 && fourier_scratch_doubles(1) == 4 * FB_MAX + 24,
              "Fourier scratch carve and kernels disagree");
static_assert(aa_partial_doubles() == (size_t)AAB_MAX * AA_NP, "mixing partials carve and kernels disagree");

int fourier_blocks(int max_cells) {
    const int b = (max_cells + FB_THREADS - 1) / FB_THREADS;
    return b < FB_MAX ? b : FB_MAX;
}

hipError_t launch_fourier_init(const GeomDev* geoms_dev, int n_geoms, int max_cells, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_fourier_init, dim3(fourier_blocks(max_cells), n_geoms), dim3(FB_THREADS), 0, st, geoms_dev);
    hipLaunchKernelGGL(k_fourier_norm, dim3(n_geoms), dim3(FB_THREADS), 0, st, geoms_dev);
    hipLaunchKernelGGL(k_fourier_s0, dim3(fourier_blocks(max_cells), n_geoms), dim3(FB_THREADS), 0, st, geoms_dev);
    return hipGetLastError();
}

hipError_t launch_fourier_iter(const GeomDev* geoms_dev, int n_geoms, int max_cells, int parity, double tol,
                               int max_iter, hipStream_t st) {
    (void)hipGetLastError();
    const dim3 grid(fourier_blocks(max_cells), n_geoms);
    hipLaunchKernelGGL(k_fourier_cg, grid, dim3(FB_THREADS), 0, st, geoms_dev, parity, tol, max_iter);
    return hipGetLastError();
}

hipError_t launch_fourier_pending(const GeomDev* geoms_dev, int n_geoms, int* pending_dev, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_fourier_pending, dim3(1), dim3(256), 0, st, geoms_dev, n_geoms, pending_dev);
    return hipGetLastError();
}

hipError_t launch_fourier_finish(const GeomDev* geoms_dev, int n_geoms, int max_cells, hipStream_t st) {
    (void)hipGetLastError();
    const dim3 grid(fourier_blocks(max_cells), n_geoms);
    hipLaunchKernelGGL(k_fourier_part, grid, dim3(FB_THREADS), 0, st, geoms_dev);
    hipLaunchKernelGGL(k_fourier_fill, grid, dim3(FB_THREADS), 0, st, geoms_dev);
    return hipGetLastError();
}

template <typename T, int CPL, bool FULL>
static hipError_t launch_sweep_f(const GeomDev* g, const Item* it, int n, int waves, PassParams pp,
                                 size_t lds, hipStream_t st) {
    (void)hipGetLastError();
    const dim3 grid(n), block(64 * waves);
    if (pp.adjoint) {
        if (pp.sigma1) hipLaunchKernelGGL((k_sweep_pass<T, CPL, 1, 1, FULL>), grid, block, lds, st, g, it, n, pp);
        else hipLaunchKernelGGL((k_sweep_pass<T, CPL, 1, 0, FULL>), grid, block, lds, st, g, it, n, pp);
    } else {
        if (pp.sigma1) hipLaunchKernelGGL((k_sweep_pass<T, CPL, 0, 1, FULL>), grid, block, lds, st, g, it, n, pp);
        else hipLaunchKernelGGL((k_sweep_pass<T, CPL, 0, 0, FULL>), grid, block, lds, st, g, it, n, pp);
    }
    return hipGetLastError();
}

template <typename T, int CPL>
static hipError_t launch_sweep_t(const GeomDev* g, const Item* it, int n, int waves, PassParams pp,
                                 size_t lds, hipStream_t st, int full) {
    return full ? launch_sweep_f<T, CPL, true>(g, it, n, waves, pp, lds, st)
                : launch_sweep_f<T, CPL, false>(g, it, n, waves, pp, lds, st);
}

template <typename T, int CPL, bool FULL>
static hipError_t launch_sweep3_f(const GeomDev* g, const Item* it, int n, int waves, PassParams pp,
                                  size_t lds, hipStream_t st) {
    (void)hipGetLastError();
    const dim3 grid(n), block(64 * waves);
    if (pp.adjoint) {
        if (pp.sigma1) hipLaunchKernelGGL((k_sweep_pass3<T, CPL, 1, 1, FULL>), grid, block, lds, st, g, it, n, pp);
        else hipLaunchKernelGGL((k_sweep_pass3<T, CPL, 1, 0, FULL>), grid, block, lds, st, g, it, n, pp);
    } else {
        if (pp.sigma1) hipLaunchKernelGGL((k_sweep_pass3<T, CPL, 0, 1, FULL>), grid, block, lds, st, g, it, n, pp);
        else hipLaunchKernelGGL((k_sweep_pass3<T, CPL, 0, 0, FULL>), grid, block, lds, st, g, it, n, pp);
    }
    return hipGetLastError();
}

template <typename T, int CPL>
static hipError_t launch_sweep3_t(const GeomDev* g, const Item* it, int n, int waves, PassParams pp,
                                  size_t lds, hipStream_t st, int full) {
    return full ? launch_sweep3_f<T, CPL, true>(g, it, n, waves, pp, lds, st)
                : launch_sweep3_f<T, CPL, false>(g, it, n, waves, pp, lds, st);
}

hipError_t launch_sweep_pass(int precision, int cpl, int nz, const GeomDev* g, const Item* it,
                             int n, int waves, PassParams pp, size_t lds, hipStream_t st, int full) {
    if (nz > 1) {
        if (precision == 0) {
            switch (cpl) {
                case 1: return launch_sweep3_t<double, 1>(g, it, n, waves, pp, lds, st, full);
                case 2: return launch_sweep3_t<double, 2>(g, it, n, waves, pp, lds, st, full);
                case 3: return launch_sweep3_t<double, 3>(g, it, n, waves, pp, lds, st, full);
                default: return launch_sweep3_t<double, 4>(g, it, n, waves, pp, lds, st, full);
            }
        }
        switch (cpl) {
            case 1: return launch_sweep3_t<float, 1>(g, it, n, waves, pp, lds, st, full);
            case 2: return launch_sweep3_t<float, 2>(g, it, n, waves, pp, lds, st, full);
            case 3: return launch_sweep3_t<float, 3>(g, it, n, waves, pp, lds, st, full);
            default: return launch_sweep3_t<float, 4>(g, it, n, waves, pp, lds, st, full);
        }
    }
    if (precision == 0) {
        switch (cpl) {
            case 1: return launch_sweep_t<double, 1>(g, it, n, waves, pp, lds, st, full);
            case 2: return launch_sweep_t<double, 2>(g, it, n, waves, pp, lds, st, full);
            case 3: return launch_sweep_t<double, 3>(g, it, n, waves, pp, lds, st, full);
            default: return launch_sweep_t<double, 4>(g, it, n, waves, pp, lds, st, full);
        }
    }
    switch (cpl) {
        case 1: return launch_sweep_t<float, 1>(g, it, n, waves, pp, lds, st, full);
        case 2: return launch_sweep_t<float, 2>(g, it, n, waves, pp, lds, st, full);
        case 3: return launch_sweep_t<float, 3>(g, it, n, waves, pp, lds, st, full);
        default: return launch_sweep_t<float, 4>(g, it, n, waves, pp, lds, st, full);
    }
}

// 3D: the pass's sources (sigma T_L, or sigma sum lambda in the adjoint) and
// inflow tables, read from the buffers the pass's sweeps consume (the rule of
// the pass kernel), in the compute type: qrec = [src | bnd face 0 | ... ].
template <typename T>
__global__ void __launch_bounds__(256) k_pack3(const GeomDev* __restrict__ geoms, PassParams pp) {
    const GeomDev& g = geoms[blockIdx.y];
    if (pp.mode == 0 && g.ctrl[CTRL_DONE]) return;
    const int pass = g.ctrl[CTRL_PASS];
    const int buf = (pp.mode == 1) ? ((pass + 1) & 1) : (pass & 1);
    const size_t nc = (size_t)g.ncells, nb = (size_t)g.nf * nc;
    const double* src = (pp.adjoint ? g.lam_psi : g.sT) + (size_t)buf * nc;
    const double* bnd = g.bnd + ((size_t)(pp.adjoint ? 2 : 0) + buf) * nb;
    T* out = static_cast<T*>(g.qrec);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc + nb; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (T)(i < nc ? src[i] : bnd[i - nc]);
}

hipError_t launch_pack3(int precision, const GeomDev* geoms_dev, int n_geoms, int max_cells, PassParams pp,
                        hipStream_t st) {
    int blocks = (7 * max_cells + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    (void)hipGetLastError();
    if (precision == 1) hipLaunchKernelGGL(k_pack3<float>, dim3(blocks, n_geoms), dim3(256), 0, st, geoms_dev, pp);
    else hipLaunchKernelGGL(k_pack3<double>, dim3(blocks, n_geoms), dim3(256), 0, st, geoms_dev, pp);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_queue_t(const GeomDev* g, const Item* it, int n, int waves, PassParams pp, hipStream_t st,
                                 int* queue, int groups) {
    (void)hipGetLastError();
    const dim3 grid(groups), block(64 * waves);
    if (pp.adjoint) {
        if (pp.sigma1) hipLaunchKernelGGL((k_sweep_queue<T, 1, 1>), grid, block, 0, st, g, it, n, pp, queue);
        else hipLaunchKernelGGL((k_sweep_queue<T, 1, 0>), grid, block, 0, st, g, it, n, pp, queue);
    } else {
        if (pp.sigma1) hipLaunchKernelGGL((k_sweep_queue<T, 0, 1>), grid, block, 0, st, g, it, n, pp, queue);
        else hipLaunchKernelGGL((k_sweep_queue<T, 0, 0>), grid, block, 0, st, g, it, n, pp, queue);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_queue(int precision, const GeomDev* g, const Item* it, int n, int waves, PassParams pp,
                              hipStream_t st, int* queue) {
    // enough groups to fill every SIMD; a group that starts once the queue is
    // empty leaves at once
    const int cap = 8192 / (waves > 1 ? waves : 1);
    const int groups = n < cap ? (n > 1 ? n : 1) : cap;
    return precision == 1 ? launch_queue_t<float>(g, it, n, waves, pp, st, queue, groups)
                          : launch_queue_t<double>(g, it, n, waves, pp, st, queue, groups);
}

hipError_t launch_pack_rows(int precision, const GeomDev* geoms_dev, int n_geoms, int max_cells, PassParams pp,
                            hipStream_t st, int* queue) {
    // four records per cell; at most 512 blocks per geometry (grid-stride)
    int blocks = (4 * max_cells + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 512 ? 512 : blocks);
    (void)hipGetLastError();
    if (precision == 1) hipLaunchKernelGGL(k_pack_rows<float>, dim3(blocks, n_geoms), dim3(256), 0, st, geoms_dev, pp, queue);
    else hipLaunchKernelGGL(k_pack_rows<double>, dim3(blocks, n_geoms), dim3(256), 0, st, geoms_dev, pp, queue);
    return hipGetLastError();
}

hipError_t launch_reduce_pass(int precision, const GeomDev* geoms_dev, int n_geoms, int max_solid,
                              PassParams pp, hipStream_t st) {
    int blocks = (max_solid + RC - 1) / RC;
    if (blocks < 1) blocks = 1;
    (void)hipGetLastError();
    if (precision == 1) hipLaunchKernelGGL(k_reduce_pass<float>, dim3(blocks, n_geoms), dim3(64 * RQ), 0, st, geoms_dev, pp);
    else hipLaunchKernelGGL(k_reduce_pass<double>, dim3(blocks, n_geoms), dim3(64 * RQ), 0, st, geoms_dev, pp);
    return hipGetLastError();
}

// Gauge of the outer iteration with a mode table.  The interpolated weights
// do not conserve energy exactly (S_ml is not alpha_ml Lambda_m s_l), so the
// pass map has no fixed point: its iterates drift by a common constant each
// pass, which no conductivity sees.  Removing that drift (the mean lattice
// temperature over the solid cells is set back to 0 after every pass) leaves
// a map with a fixed point, which Anderson mixing and the lagged wrap need.
// The stored wrap inflows stay as they are: re-centred, the next inputs are
// close to this pass's, whose inflows they hold.  ax[n_aa] carries the shift
// from the first kernel to the second.
__global__ void __launch_bounds__(256) k_gauge_mean(const GeomDev* __restrict__ geoms) {
    __shared__ double red[32];
    const GeomDev& g = geoms[blockIdx.x];
    if (!g.gauge || g.ctrl[CTRL_DONE]) return;
    double s = 0.0, ns = 0.0;
    for (int c = threadIdx.x; c < g.ncells; c += blockDim.x)
        if (fc_solid(g.fc[c])) { s += g.T_L[c]; ns += 1.0; }
    s = block_sum(s, red);
    ns = block_sum(ns, red);
    if (threadIdx.x == 0) g.ax[g.n_aa] = ns > 0.0 ? s / ns : 0.0;
}

__global__ void __launch_bounds__(256) k_gauge_apply(const GeomDev* __restrict__ geoms) {
    const GeomDev& g = geoms[blockIdx.y];
    if (!g.gauge || g.ctrl[CTRL_DONE]) return;
    const double d = g.ax[g.n_aa];
    const int out = (g.ctrl[CTRL_PASS] + 1) & 1;
    const int nc = g.ncells;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) {
        if (!fc_solid(g.fc[i])) return;
        if (g.aa_m > 0) {
            g.ag[i] -= d;
        } else {
            g.sT[(size_t)out * nc + i] -= g.sigma[i] * d;
            g.ax[i] -= d;
        }
    } else if (i < nc + g.nwalls) {
        const int wi = i - nc;
        if (g.aa_m > 0) {
            g.ag[i] -= d;
        } else {
            g.Tw[(size_t)out * g.nwalls + wi] -= d;
            g.ax[i] -= d;
            g.bnd[((size_t)out * g.nf + g.wall_face[wi]) * nc + g.wall_cell[wi]] -= d;
        }
    }
}

hipError_t launch_gauge(const GeomDev* geoms_dev, int n_geoms, int max_aa, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_gauge_mean, dim3(n_geoms), dim3(256), 0, st, geoms_dev);
    hipLaunchKernelGGL(k_gauge_apply, dim3((max_aa + 255) / 256, n_geoms), dim3(256), 0, st, geoms_dev);
    return hipGetLastError();
}

hipError_t launch_finalize(const GeomDev* geoms_dev, int n_geoms, PassParams pp, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_finalize, dim3(n_geoms), dim3(256), 0, st, geoms_dev, pp);
    return hipGetLastError();
}

// Mode-resolved kappa (paper Eq. mode-resolved, cell-centred form): a gather
// of the per-system sums with each mode's interpolation weights, measured
// from the mean lattice temperature (sum_i T_L,i = sum_ml D_ml sum_i T_iml;
// the weights of a mode add up to 1).  One block: the D-weighted total in a
// fixed-order tree, then the modes strided over the threads.
__global__ void __launch_bounds__(256) k_kappa_modes(const int* __restrict__ sys, const double* __restrict__ w,
                                                     const double* __restrict__ Sg, int n_modes, int terms,
                                                     const double* __restrict__ D, int n_sys,
                                                     const double* __restrict__ kraw, double pref,
                                                     double* __restrict__ out) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double a = 0.0;
    for (int i = t; i < n_sys; i += 256) a += D[i] * kraw[i];
    red[t] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double tot_L = red[0];
    for (int mu = t; mu < n_modes; mu += 256) {
        double s = 0.0;
        for (int k = 0; k < terms; ++k) {
            const double c = w[(size_t)mu * terms + k];
            if (c != 0.0) s += c * kraw[sys[(size_t)mu * terms + k]];
        }
        out[mu] = pref * Sg[mu] * (s - tot_L);
    }
}

hipError_t launch_kappa_modes(const int* sys, const double* w, const double* Sg, int n_modes, int terms,
                              const double* D, int n_sys, const double* kraw, double pref, double* out,
                              hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_kappa_modes, dim3(1), dim3(256), 0, st, sys, w, Sg, n_modes, terms, D, n_sys, kraw,
                       pref, out);
    return hipGetLastError();
}

hipError_t launch_anderson(const GeomDev* geoms_dev, int n_geoms, int max_naa, PassParams pp, hipStream_t st) {
    (void)hipGetLastError();
    int b = (max_naa + AA_THREADS - 1) / AA_THREADS;
    if (b > AAB_MAX) b = AAB_MAX;
    const dim3 grid(b, n_geoms);
    hipLaunchKernelGGL(k_aa_partial, grid, dim3(AA_THREADS), 0, st, geoms_dev);
    hipLaunchKernelGGL(k_aa_apply, grid, dim3(AA_THREADS), 0, st, geoms_dev, pp);
    return hipGetLastError();
}

hipError_t launch_energy(const GeomDev* geom_dev, int precision, int nsolid, hipStream_t st) {
    const int blocks = nsolid > 0 ? (nsolid + 63) / 64 : 1;
    (void)hipGetLastError();
    if (precision == 1) hipLaunchKernelGGL(k_energy<float>, dim3(blocks), dim3(64 * EQ), 0, st, geom_dev);
    else hipLaunchKernelGGL(k_energy<double>, dim3(blocks), dim3(64 * EQ), 0, st, geom_dev);
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(256), 0, st, geom_dev, blocks);
    return hipGetLastError();
}

hipError_t launch_prep_sigma(const GeomDev* g_dev, int ncells, const double* sig, hipStream_t st) {
    int blocks = (ncells + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_prep_sigma, dim3(blocks), dim3(256), 0, st, g_dev, sig);
    hipLaunchKernelGGL(k_sigma_min, dim3(1), dim3(256), 0, st, g_dev, blocks);
    return hipGetLastError();
}

hipError_t launch_output(const GeomDev* geom_dev, int precision, int ncells, double* T_L_out, double* J_out,
                         double* grad_out, hipStream_t st) {
    (void)hipGetLastError();
    const dim3 grid((ncells + 255) / 256);
    if (T_L_out) hipLaunchKernelGGL(k_output, dim3(1), dim3(1024), 0, st, geom_dev, T_L_out);
    if (J_out) {
        if (precision == 1) hipLaunchKernelGGL(k_flux<float>, grid, dim3(256), 0, st, geom_dev, J_out);
        else hipLaunchKernelGGL(k_flux<double>, grid, dim3(256), 0, st, geom_dev, J_out);
    }
    if (grad_out) {
        if (precision == 1) hipLaunchKernelGGL(k_grad<float>, grid, dim3(256), 0, st, geom_dev, grad_out);
        else hipLaunchKernelGGL(k_grad<double>, grid, dim3(256), 0, st, geom_dev, grad_out);
    }
    return hipGetLastError();
}
