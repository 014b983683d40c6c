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

__device__ __forceinline__ int nbr_cell(const GeomDev& g, int cell, int f) {
    int ix = cell % g.nx, iy = (cell / g.nx) % g.ny, iz = cell / (g.nx * g.ny);
    const int a = f >> 1, step = (f & 1) ? 1 : -1;
    if (a == 0) ix = (ix + step + g.nx) % g.nx;
    else if (a == 1) iy = (iy + step + g.ny) % g.ny;
    else iz = (iz + step + g.nz) % g.nz;
    return ix + g.nx * (iy + g.ny * iz);
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
    return s;
}

// a[i] for a small array and a runtime index without forcing it to memory
template <typename T>
__device__ __forceinline__ T pick3(const T (&a)[3], int i) { return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]); }

template <typename T>
__device__ __forceinline__ T sigma_of(const GeomDev& g, int cell);
template <>
__device__ __forceinline__ double sigma_of<double>(const GeomDev& g, int cell) { return g.sigma[cell]; }
template <>
__device__ __forceinline__ float sigma_of<float>(const GeomDev& g, int cell) { return g.sigma_f[cell]; }

// Reduction state of the lockstep final sweep.
struct Red {
    double* lds;      // W * NV * ROW doubles
    int w, W, NV, ROW;
    int item;         // global item index
    int local;        // item index within the geometry
    int want_J, store_T, adjoint;
    double kacc, kface;
};

// ---------------------------------------------------------------------------
// The upwind sweep.  WITH_B: include the pass sources b; otherwise the only
// source is the wrap inflow u.  RED: lockstep reductions (all waves of the
// block must call it together).  Returns the last row (jj = ny-1) in xl.
// ---------------------------------------------------------------------------
template <typename T, int CPL, int NZ, bool WITH_B, bool RED>
__device__ __forceinline__ void sweep(const GeomDev& g, const SysC<T>& s, int active, int lane,
                      const double* __restrict__ srcbase, const double* __restrict__ wallv,
                      const T (&u)[NZ][CPL], T (&xl)[NZ][CPL], Red* rd) {
    T xr[NZ][CPL];
#pragma unroll
    for (int k = 0; k < NZ; ++k)
#pragma unroll
        for (int c = 0; c < CPL; ++c) xr[k][c] = T(0);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    constexpr int ND = NZ > 1 ? 3 : 2;
    const int adj = RED ? rd->adjoint : 0;
    for (int jj = 0; jj < ny; ++jj) {
        const int iy = s.pos[1] ? jj : ny - 1 - jj;
        for (int kk = 0; kk < NZ; ++kk) {
            if (kk >= nz) break;
            const int iz = (NZ > 1) ? (s.pos[2] ? kk : nz - 1 - kk) : 0;
            const int rowbase = nx * (iy + ny * iz);
            T a[CPL], q[CPL];
            T Al = T(0), Ql = T(1), Pl = T(0);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int p = lane * CPL + c;
                T av = T(0), qv = T(1), pv = T(0);      // identity beyond the row
                if (p < nx) {
                    av = T(0); qv = T(0); pv = T(1);      // pore: breaks the chain
                    const int ix = s.pos[0] ? p : nx - 1 - p;
                    const int cell = rowbase + ix;
                    const uint16_t w = g.fc[cell];
                    if (active && fc_solid(w)) {
                        const int clx = fc_class(w, s.fin[0]);
                        const int cly = fc_class(w, s.fin[1]);
                        const int clz = (NZ > 1) ? fc_class(w, s.fin[2]) : FC_WALL;
                        const T sg = sigma_of<T>(g, cell);
                        const T cz = (NZ > 1) ? s.c[2] : T(0);
                        const T d = sg + s.c[0] + s.c[1] + cz;
                        const T rdv = T(1) / d;
                        T src = T(0);
                        if (WITH_B) {
                            double sd = srcbase[cell];
                            if (adj) sd = s.kw + s.Dml * sd;
#pragma unroll
                            for (int ax = 0; ax < ND; ++ax) {
                                const int cl = ax == 0 ? clx : (ax == 1 ? cly : clz);
                                if (cl == FC_WALL) {
                                    const int wi = g.wall_idx[cell * g.nf + s.fin[ax]];
                                    const double wv = wallv[wi];
                                    sd += adj ? g.wout[s.fin[ax] * g.n_sys + s.sys] * wv : s.cd[ax] * wv;
                                } else if (!adj && cl == FC_JUMP_P) {
                                    sd += s.cd[ax] * g.dT;
                                } else if (!adj && cl == FC_JUMP_M) {
                                    sd -= s.cd[ax] * g.dT;
                                }
                            }
                            src = (T)sd;
                        }
                        T yin = T(0);
                        if (cly != FC_WALL) yin = (jj == 0) ? u[kk][c] : s.c[1] * xr[kk][c];
                        T zin = T(0);
                        if (NZ > 1 && clz != FC_WALL && kk > 0) zin = cz * xr[kk > 0 ? kk - 1 : 0][c];
                        av = (src + yin + zin) * rdv;
                        const bool xs = (clx != FC_WALL);
                        qv = xs ? s.c[0] * rdv : T(0);
                        pv = (sg + s.c[1] + cz + (xs ? T(0) : s.c[0])) * rdv;
                    }
                }
                a[c] = av;
                q[c] = qv;
                Al = av + qv * Al;
                Pl = pv + qv * Pl;
                Ql = qv * Ql;
            }
            // inclusive scan of affine maps across the wavefront
            T A = Al, Q = Ql, P = Pl;
#pragma unroll
            for (int off = 1; off < WAVE; off <<= 1) {
                const T A2 = shfl_up(A, off), Q2 = shfl_up(Q, off), P2 = shfl_up(P, off);
                if (lane >= off) {
                    A = A + Q * A2;
                    P = P + Q * P2;
                    Q = Q * Q2;
                }
            }
            const T At = shfl_at(A, WAVE - 1), Pt = shfl_at(P, WAVE - 1);
            const T xin = (Pt > T(0)) ? At / Pt : T(0);   // cyclic closure x_{-1} = x_{nx-1}
            T Ae = shfl_up(A, 1), Qe = shfl_up(Q, 1);
            if (lane == 0) { Ae = T(0); Qe = T(1); }
            T xp = Ae + Qe * xin;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const T xv = a[c] + q[c] * xp;
                const int p = lane * CPL + c;
                xr[kk][c] = (p < nx) ? xv : T(0);
                xp = xv;
            }
            if (jj == ny - 1) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) xl[kk][c] = xr[kk][c];
            }
            if (RED) {
                // ---- per-row reductions, lockstep across the block's waves
                double* buf = rd->lds;
                const int ROW = rd->ROW, NV = rd->NV, W = rd->W;
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int p = lane * CPL + c;
                    double xv = (double)xr[kk][c];
                    double* slot = buf + (size_t)(rd->w * NV) * ROW + p;
                    double tw[3] = {0.0, 0.0, 0.0};
                    if (p < nx && active) {
                        const int ix = s.pos[0] ? p : nx - 1 - p;
                        const int cell = rowbase + ix;
                        const uint16_t wv = g.fc[cell];
                        if (fc_solid(wv)) {
                            rd->kacc += xv;
                            if (adj) {
                                // p^T lambda: forward jump inflow = reversed outflow faces
#pragma unroll
                                for (int ax = 0; ax < ND; ++ax) {
                                    const int cl = fc_class(wv, s.fout[ax]);
                                    if (cl == FC_JUMP_P) rd->kface += s.cd[ax] * g.dT * xv;
                                    else if (cl == FC_JUMP_M) rd->kface -= s.cd[ax] * g.dT * xv;
                                }
                            }
                            // kappa through the periodic plane of the gradient axis
                            if (!adj && g.grad_axis == 0 && p == nx - 1 && fc_class(wv, s.fout[0]) != FC_WALL)
                                rd->kface += xv + (s.pos[0] ? g.dT : 0.0);
                            if (!adj && g.grad_axis == 1 && jj == ny - 1 && fc_class(wv, s.fout[1]) != FC_WALL)
                                rd->kface += xv + (s.pos[1] ? g.dT : 0.0);
#pragma unroll
                            for (int ax = 0; ax < ND; ++ax)
                                if (fc_class(wv, s.fout[ax]) == FC_WALL)
                                    tw[ax] = adj ? s.cd[ax] * xv : g.wout[s.fout[ax] * g.n_sys + s.sys] * xv;
                            if (rd->store_T) g.Tstore[(size_t)s.sys * g.ncells + cell] = xv;
                            if (adj) {
                                // gradient partial: lambda (T - T_L)
                                const double Tf = g.Tstore[(size_t)s.sys * g.ncells + cell];
                                slot[(size_t)(1 + ND) * ROW] = xv * (Tf - g.T_L[cell]);
                            }
                        } else {
                            xv = 0.0;
                            if (adj) slot[(size_t)(1 + ND) * ROW] = 0.0;
                        }
                    } else {
                        xv = 0.0;
                        if (adj) slot[(size_t)(1 + ND) * ROW] = 0.0;
                    }
                    slot[0] = adj ? xv : s.Dml * xv;
#pragma unroll
                    for (int ax = 0; ax < ND; ++ax) slot[(size_t)(1 + ax) * ROW] = tw[ax];
                    if (rd->want_J)
#pragma unroll
                        for (int ax = 0; ax < ND; ++ax)
                            slot[(size_t)(1 + ND + ax) * ROW] = s.S[ax] * xv;
                }
                __syncthreads();
                const int nvu = 1 + ND + ((rd->want_J || adj) ? (adj ? 1 : ND) : 0);
                for (int idx = threadIdx.x; idx < nx * nvu; idx += blockDim.x) {
                    const int p = idx % nx, v = idx / nx;
                    double sum = 0.0;
                    for (int ww = 0; ww < W; ++ww) sum += buf[(size_t)(ww * NV + v) * ROW + p];
                    const int ix = s.pos[0] ? p : nx - 1 - p;
                    const int cell = rowbase + ix;
                    const uint16_t wv = g.fc[cell];
                    if (v == 0) {
                        g.part_TL[(size_t)rd->local * g.ncells + cell] = fc_solid(wv) ? sum : 0.0;
                    } else if (v <= ND) {
                        const int fo = pick3(s.fout, v - 1);
                        if (fc_solid(wv) && fc_class(wv, fo) == FC_WALL)
                            g.part_Tw[(size_t)rd->local * g.nwalls + g.wall_idx[cell * g.nf + fo]] = sum;
                    } else if (adj) {
                        g.part_G[(size_t)rd->local * g.ncells + cell] = sum;
                    } else {
                        const int ax = v - 1 - ND;
                        g.part_J[((size_t)rd->local * g.ncells + cell) * ND + ax] = sum;
                    }
                }
                __syncthreads();
            }
        }
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
                const uint16_t w = g.fc[ix + g.nx * (iy + g.ny * iz)];
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

#define VLOOP(body)                       \
    _Pragma("unroll") for (int k = 0; k < NZ; ++k) \
    _Pragma("unroll") for (int c = 0; c < CPL; ++c) { body; }

// ---------------------------------------------------------------------------
// One outer pass for every work item (block = one item = W systems sharing a
// direction).
// ---------------------------------------------------------------------------
template <typename T, int CPL, int NZ>
__global__ void __launch_bounds__(512) k_sweep_pass(const GeomDev* __restrict__ geoms,
                                                     const Item* __restrict__ items, int n_items,
                                                     PassParams pp) {
    extern __shared__ double lds[];
    const int it = blockIdx.x;
    if (it >= n_items) return;
    const Item item = items[it];
    const GeomDev& g = geoms[item.geom];
    if (pp.mode == 0 && g.ctrl[CTRL_DONE]) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, W = blockDim.x >> 6;
    const int m = item.m0 + w;
    const int active = (w < item.nm) && (m < g.n_mfp);
    const int adj = pp.adjoint;
    const SysC<T> s = make_sys<T>(g, active ? m : item.m0, item.l, adj);
    const int pass = g.ctrl[CTRL_PASS];
    const int buf_in = (pp.mode == 1) ? ((pass + 1) & 1) : (pass & 1);
    const double* srcbase = adj ? (g.lam_psi + (size_t)buf_in * g.ncells) : (g.sT + (size_t)buf_in * g.ncells);
    const double* wallv = adj ? (g.lam_phi + (size_t)buf_in * g.nwalls) : (g.Tw + (size_t)buf_in * g.nwalls);
    T* Uall = reinterpret_cast<T*>(g.U) + (adj ? (size_t)g.n_sys * g.nwrap : 0);

    T u[NZ][CPL], xl[NZ][CPL], mk[NZ][CPL];
    wrap_mask<T, CPL, NZ>(g, s, active, lane, mk);
    // warm start from the previous pass
    VLOOP({
        const int p = lane * CPL + c;
        u[k][c] = (active && k < g.nz && p < g.nx) ? Uall[(size_t)s.sys * g.nwrap + k * g.nx + p] : T(0);
    });
    long long n_it = 0, n_sw = 0;
    const bool has_wrap = g.periodic[1] != 0;
    if (pp.mode == 0 && active && has_wrap) {
        T z[NZ][CPL];
        sweep<T, CPL, NZ, true, false>(g, s, active, lane, srcbase, wallv, u, z, nullptr);
        ++n_sw;
        T r[NZ][CPL];
        VLOOP(r[k][c] = mk[k][c] * z[k][c] - u[k][c]);
        T ez[NZ][CPL];
        VLOOP(ez[k][c] = mk[k][c] * z[k][c]);
        const double scale = sqrt(vdot<T, CPL, NZ>(ez, ez));
        double rn = sqrt(vdot<T, CPL, NZ>(r, r));
        const double thr = pp.inner_tol * scale;
        if (rn > thr && scale > 0.0) {
            T rh[NZ][CPL], p[NZ][CPL], v[NZ][CPL], sv[NZ][CPL], t[NZ][CPL];
            VLOOP({ rh[k][c] = r[k][c]; p[k][c] = T(0); v[k][c] = T(0); });
            double rho_old = 1.0, alpha = 1.0, omega = 1.0;
            for (int iter = 0; iter < pp.max_inner; ++iter) {
                double rho = vdot<T, CPL, NZ>(rh, r);
                if (fabs(rho) <= 1e-30 * rn * rn || !(omega != 0.0)) {
                    // breakdown: restart with the current residual as shadow
                    VLOOP({ rh[k][c] = r[k][c]; p[k][c] = T(0); v[k][c] = T(0); });
                    rho = vdot<T, CPL, NZ>(r, r);
                    rho_old = 1.0; alpha = 1.0; omega = 1.0;
                }
                const double beta = (rho / rho_old) * (alpha / omega);
                VLOOP(p[k][c] = r[k][c] + (T)beta * (p[k][c] - (T)omega * v[k][c]));
                sweep<T, CPL, NZ, false, false>(g, s, active, lane, srcbase, wallv, p, xl, nullptr);
                ++n_sw;
                VLOOP(v[k][c] = p[k][c] - mk[k][c] * xl[k][c]);
                const double rv = vdot<T, CPL, NZ>(rh, v);
                if (rv == 0.0) break;
                alpha = rho / rv;
                VLOOP(sv[k][c] = r[k][c] - (T)alpha * v[k][c]);
                const double sn = sqrt(vdot<T, CPL, NZ>(sv, sv));
                ++n_it;
                if (sn <= thr) {
                    VLOOP(u[k][c] += (T)alpha * p[k][c]);
                    break;
                }
                sweep<T, CPL, NZ, false, false>(g, s, active, lane, srcbase, wallv, sv, xl, nullptr);
                ++n_sw;
                VLOOP(t[k][c] = sv[k][c] - mk[k][c] * xl[k][c]);
                const double tt = vdot<T, CPL, NZ>(t, t);
                omega = tt > 0.0 ? vdot<T, CPL, NZ>(t, sv) / tt : 0.0;
                VLOOP(u[k][c] += (T)alpha * p[k][c] + (T)omega * sv[k][c]);
                VLOOP(r[k][c] = sv[k][c] - (T)omega * t[k][c]);
                rn = sqrt(vdot<T, CPL, NZ>(r, r));
                rho_old = rho;
                if (rn <= thr) break;
            }
        }
        VLOOP({
            const int pp_ = lane * CPL + c;
            if (k < g.nz && pp_ < g.nx) Uall[(size_t)s.sys * g.nwrap + k * g.nx + pp_] = u[k][c];
        });
    }
    // final sweep with the lockstep reductions
    Red rd;
    rd.lds = lds;
    rd.w = w;
    rd.W = W;
    rd.NV = 1 + 2 * (NZ > 1 ? 3 : 2);
    rd.ROW = WAVE * CPL;
    rd.item = it;
    rd.local = item.local;
    rd.want_J = pp.want_J;
    rd.store_T = pp.store_T;
    rd.adjoint = adj;
    rd.kacc = 0.0;
    rd.kface = 0.0;
    sweep<T, CPL, NZ, true, true>(g, s, active, lane, srcbase, wallv, u, xl, &rd);
    ++n_sw;
    const double ks = wave_sum(rd.kacc), kf = wave_sum(rd.kface);
    if (active && lane == 0) {
        if (adj) {
            g.ksys[s.sys] = kf;                 // this system's share of p^T lambda
            g.kfsys[s.sys] = 0.0;
        } else {
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
// Per-cell / per-wall sums of the item partials (fixed order) and the next
// pass's inputs sigma T_L and T_w.
// ---------------------------------------------------------------------------
__global__ void k_reduce_pass(const GeomDev* __restrict__ geoms, PassParams pp) {
    const GeomDev& g = geoms[blockIdx.y];
    if (g.ctrl[CTRL_DONE] && pp.mode == 0) return;
    const int pass = g.ctrl[CTRL_PASS];
    const int out = (pass + 1) & 1;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    const int adj = pp.adjoint;
    for (int cell = tid; cell < g.ncells; cell += stride) {
        double acc = 0.0;
        for (int i = 0; i < g.n_items; ++i) acc += g.part_TL[(size_t)i * g.ncells + cell];
        const bool sol = fc_solid(g.fc[cell]);
        if (adj) {
            g.lam_psi[(size_t)out * g.ncells + cell] = sol ? g.sigma[cell] * acc : 0.0;
        } else {
            g.T_L[cell] = sol ? acc : 0.0;
            g.sT[(size_t)out * g.ncells + cell] = sol ? g.sigma[cell] * acc : 0.0;
        }
    }
    for (int wi = tid; wi < g.nwalls; wi += stride) {
        const int f = g.wall_face[wi];
        const int ax = f >> 1;
        const double nsgn = (f & 1) ? 1.0 : -1.0;
        double acc = 0.0;
        // items whose direction leaves the cell through this face (forward) or
        // enters it (adjoint: outflow of the reversed direction)
        for (int i = 0; i < g.n_items; ++i) {
            const int l = i / g.n_grp;          // items are ordered (l, MFP group)
            const double sn = g.dirs[l * 3 + ax] * nsgn;
            if ((!adj && sn > 0.0) || (adj && sn < 0.0)) acc += g.part_Tw[(size_t)i * g.nwalls + wi];
        }
        if (adj) g.lam_phi[(size_t)out * g.nwalls + wi] = acc;
        else g.Tw[(size_t)out * g.nwalls + wi] = acc;
    }
}

// kappa, history and the convergence test of Algorithm 1 (one block per geometry).
__global__ void k_finalize(const GeomDev* __restrict__ geoms, PassParams pp) {
    __shared__ double red[32];
    const GeomDev& g = geoms[blockIdx.x];
    if (g.ctrl[CTRL_DONE]) return;
    double k = 0.0, kf = 0.0;
    for (int i = threadIdx.x; i < g.n_sys; i += blockDim.x) {
        k += g.ksys[i];
        kf += g.kfsys[i];
    }
    // fixed-order: every thread sums a fixed strided subset, then block_sum
    k = block_sum(k, red);
    kf = block_sum(kf, red);
    if (threadIdx.x == 0) {
        const int pass = g.ctrl[CTRL_PASS];
        if (pass >= pp.max_outer) {      // history is sized for max_outer passes
            g.ctrl[CTRL_DONE] = 1;
            return;
        }
        g.hist[pass] = k;
        g.hist_face[pass] = kf;
        const int n = pass + 1;
        g.ctrl[CTRL_PASS] = n;
        if (!isfinite(k)) {
            g.ctrl[CTRL_NONFINITE] = 1;
            g.ctrl[CTRL_DONE] = 1;
        } else if (n >= 2 && fabs(k - g.hist[pass - 1]) <= pp.outer_tol * fabs(k)) {
            g.ctrl[CTRL_CONVERGED] = 1;
            g.ctrl[CTRL_DONE] = 1;
        } else if (n >= pp.max_outer) {
            g.ctrl[CTRL_DONE] = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Fourier first guess: CG on the negated 5/7-point finite-volume Laplacian
// with adiabatic pores and the periodic jump (one block per geometry).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_fourier(const GeomDev* __restrict__ geoms, double tol,
                                                 int max_iter) {
    __shared__ double red[32];
    const GeomDev& g = geoms[blockIdx.x];
    const int n = g.ncells;
    double* x = g.fx;
    double* r = g.fx + n;
    double* p = g.fx + 2 * (size_t)n;
    double* Ap = g.fx + 3 * (size_t)n;
    double kf[3];
    for (int a = 0; a < 3; ++a) kf[a] = (a < g.ndim) ? g.kappa_axis[a] / (g.h[a] * g.h[a]) : 0.0;
    const int nf = g.nf;
    // b = sum over jump faces of k/h^2 delta dT  (system: -Lap T = b)
    double rr = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const uint16_t w = g.fc[c];
        double b = 0.0;
        if (fc_solid(w))
            for (int f = 0; f < nf; ++f) {
                const int cl = fc_class(w, f);
                if (cl == FC_JUMP_P) b += kf[f >> 1] * g.dT;
                else if (cl == FC_JUMP_M) b -= kf[f >> 1] * g.dT;
            }
        x[c] = 0.0;
        r[c] = b;
        p[c] = b;
        rr += b * b;
    }
    rr = block_sum(rr, red);
    const double bn = sqrt(rr);
    int iter = 0;
    double rn = bn;
    if (bn > 0.0) {
        for (iter = 0; iter < max_iter; ++iter) {
            double pap = 0.0;
            for (int c = threadIdx.x; c < n; c += blockDim.x) {
                const uint16_t w = g.fc[c];
                double y = 0.0;
                if (fc_solid(w)) {
                    const double pc = p[c];
                    for (int f = 0; f < nf; ++f)
                        if (fc_class(w, f) != FC_WALL) y += kf[f >> 1] * (pc - p[nbr_cell(g, c, f)]);
                }
                Ap[c] = y;
                pap += p[c] * y;
            }
            pap = block_sum(pap, red);
            const double alpha = rr / pap;
            double rr2 = 0.0;
            for (int c = threadIdx.x; c < n; c += blockDim.x) {
                x[c] += alpha * p[c];
                const double rv = r[c] - alpha * Ap[c];
                r[c] = rv;
                rr2 += rv * rv;
            }
            rr2 = block_sum(rr2, red);
            rn = sqrt(rr2);
            if (rn <= tol * bn) { ++iter; break; }
            const double beta = rr2 / rr;
            rr = rr2;
            for (int c = threadIdx.x; c < n; c += blockDim.x) p[c] = r[c] + beta * p[c];
            __syncthreads();
        }
    }
    __syncthreads();
    // mean over solid cells -> 0
    double sx = 0.0, ns = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x)
        if (fc_solid(g.fc[c])) { sx += x[c]; ns += 1.0; }
    sx = block_sum(sx, red);
    ns = block_sum(ns, red);
    const double mean = sx / ns;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const bool sol = fc_solid(g.fc[c]);
        const double t = sol ? x[c] - mean : 0.0;
        x[c] = t;
        g.T_L[c] = t;
        g.sT[c] = sol ? g.sigma[c] * t : 0.0;   // buffer 0
    }
    __syncthreads();
    for (int wi = threadIdx.x; wi < g.nwalls; wi += blockDim.x) g.Tw[wi] = x[g.wall_cell[wi]];
    // kappa_F: plane flux through the periodic plane of the gradient axis
    const int ga = g.grad_axis;
    double fl = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const uint16_t w = g.fc[c];
        if (!fc_solid(w)) continue;
        const int f = 2 * ga;   // '-' face of the cell at index 0
        if (fc_class(w, f) == FC_JUMP_P) {
            const int j = nbr_cell(g, c, f);
            fl += g.kappa_axis[ga] * (x[j] + g.dT - x[c]) / g.h[ga];
        }
    }
    fl = block_sum(fl, red);
    if (threadIdx.x == 0) {
        g.fscal[0] = g.L[ga] / (g.dT * (double)g.n_perp) * fl;
        g.fscal[1] = (double)iter;
        g.fscal[2] = bn > 0.0 ? rn / bn : 0.0;
        for (int i = 0; i < CTRL_N; ++i) g.ctrl[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// Matrix-free upwind apply y = (sigma + Lambda_m A_l) x (or A_l^T) for a set
// of systems; one thread per (cell, system), cell-major within a system so
// the x-neighbour loads are coalesced and the y-neighbour row comes from L2.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_apply(const GeomDev* __restrict__ gp, const double* __restrict__ sigma,
                        const int* __restrict__ sys_ids, int n_sys, const T* __restrict__ x,
                        T* __restrict__ y, int transpose) {
    const GeomDev& g = *gp;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    const int si = blockIdx.y;
    if (cell >= g.ncells || si >= n_sys) return;
    const int sys = sys_ids[si];
    const uint16_t w = g.fc[cell];
    const size_t off = (size_t)si * g.ncells;
    if (!fc_solid(w) || sys < 0 || sys >= g.n_sys) { y[off + cell] = T(0); return; }
    const int m = sys / g.n_dir, l = sys % g.n_dir;
    const double lam = g.mfp[m];
    const double sg = sigma ? sigma[cell] : 1.0;
    const T xc = x[off + cell];
    double acc = sg * (double)xc;
    for (int a = 0; a < g.ndim; ++a) {
        double sa = g.dirs[l * 3 + a];
        if (transpose) sa = -sa;
        if (sa == 0.0) continue;
        const double ca = lam * fabs(sa) / g.h[a];
        acc += ca * (double)xc;
        const int fin = 2 * a + (sa > 0.0 ? 0 : 1);
        if (fc_class(w, fin) != FC_WALL) acc -= ca * (double)x[off + nbr_cell(g, cell, fin)];
    }
    y[off + cell] = (T)acc;
}


// sigma per cell (1 where not given or in pores) and its float copy.
__global__ void k_prep_sigma(const GeomDev* __restrict__ gp, const double* __restrict__ sig_in) {
    const GeomDev& g = *gp;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.ncells; c += gridDim.x * blockDim.x) {
        double v = 1.0;
        if (sig_in && fc_solid(g.fc[c])) v = sig_in[c];
        g.sigma[c] = v;
        g.sigma_f[c] = (float)v;
    }
}

// Outputs of one geometry: T_L with the solid-cell mean removed, the flux map
// J (sum of the item partials of the replayed last pass) and the adjoint
// gradient -sum_ml lambda (T - T_L).
__global__ void __launch_bounds__(1024) k_output(const GeomDev* __restrict__ gp, double* T_L_out,
                                                double* J_out, double* grad_out) {
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
    if (J_out) {
        for (int e = threadIdx.x; e < n * g.ndim; e += blockDim.x) {
            double acc = 0.0;
            for (int i = 0; i < g.n_items; ++i) acc += g.part_J[(size_t)i * n * g.ndim + e];
            J_out[e] = fc_solid(g.fc[e / g.ndim]) ? acc : 0.0;
        }
    }
    if (grad_out) {
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            double acc = 0.0;
            for (int i = 0; i < g.n_items; ++i) acc += g.part_G[(size_t)i * n + c];
            grad_out[c] = fc_solid(g.fc[c]) ? -acc : 0.0;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_fourier(const GeomDev* geoms_dev, int n_geoms, double tol, int max_iter,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_fourier, dim3(n_geoms), dim3(1024), 0, st, geoms_dev, tol, max_iter);
    return hipGetLastError();
}

template <typename T, int CPL, int NZ>
static hipError_t launch_sweep_t(const GeomDev* g, const Item* it, int n, int waves, PassParams pp,
                                 size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((k_sweep_pass<T, CPL, NZ>), dim3(n), dim3(64 * waves), lds, st, g, it, n, pp);
    return hipGetLastError();
}

hipError_t launch_sweep_pass(int precision, int cpl, int nz, const GeomDev* g, const Item* it,
                             int n, int waves, PassParams pp, size_t lds, hipStream_t st) {
    if (nz > 1) {
        if (precision == 0) return launch_sweep_t<double, 1, 16>(g, it, n, waves, pp, lds, st);
        return launch_sweep_t<float, 1, 16>(g, it, n, waves, pp, lds, st);
    }
    if (precision == 0) {
        switch (cpl) {
            case 1: return launch_sweep_t<double, 1, 1>(g, it, n, waves, pp, lds, st);
            case 2: return launch_sweep_t<double, 2, 1>(g, it, n, waves, pp, lds, st);
            case 3: return launch_sweep_t<double, 3, 1>(g, it, n, waves, pp, lds, st);
            default: return launch_sweep_t<double, 4, 1>(g, it, n, waves, pp, lds, st);
        }
    }
    switch (cpl) {
        case 1: return launch_sweep_t<float, 1, 1>(g, it, n, waves, pp, lds, st);
        case 2: return launch_sweep_t<float, 2, 1>(g, it, n, waves, pp, lds, st);
        case 3: return launch_sweep_t<float, 3, 1>(g, it, n, waves, pp, lds, st);
        default: return launch_sweep_t<float, 4, 1>(g, it, n, waves, pp, lds, st);
    }
}

hipError_t launch_reduce_pass(const GeomDev* geoms_dev, int n_geoms, int max_cells, int max_walls,
                              PassParams pp, hipStream_t st) {
    const int work = max_cells > max_walls ? max_cells : max_walls;
    int blocks = (work + 255) / 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_reduce_pass, dim3(blocks, n_geoms), dim3(256), 0, st, geoms_dev, pp);
    return hipGetLastError();
}

hipError_t launch_finalize(const GeomDev* geoms_dev, int n_geoms, PassParams pp, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(n_geoms), dim3(256), 0, st, geoms_dev, pp);
    return hipGetLastError();
}

hipError_t launch_apply(int precision, int transpose, const GeomDev* g_dev, const GeomDev& g_host,
                        const double* sigma, const int* sys_ids, int n_sys, const void* x, void* y,
                        hipStream_t st) {
    dim3 grid((g_host.ncells + 255) / 256, n_sys);
    if (precision == 0)
        hipLaunchKernelGGL(k_apply<double>, grid, dim3(256), 0, st, g_dev, sigma, sys_ids, n_sys,
                           (const double*)x, (double*)y, transpose);
    else
        hipLaunchKernelGGL(k_apply<float>, grid, dim3(256), 0, st, g_dev, sigma, sys_ids, n_sys,
                           (const float*)x, (float*)y, transpose);
    return hipGetLastError();
}

hipError_t launch_prep_sigma(const GeomDev* g_dev, int ncells, const double* sig, hipStream_t st) {
    int blocks = (ncells + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_prep_sigma, dim3(blocks), dim3(256), 0, st, g_dev, sig);
    return hipGetLastError();
}

hipError_t launch_output(const GeomDev* geoms_dev, int n_geoms, double* T_L_out, double* J_out,
                         double* grad_out, hipStream_t st) {
    (void)n_geoms;
    hipLaunchKernelGGL(k_output, dim3(1), dim3(1024), 0, st, geoms_dev, T_L_out, J_out, grad_out);
    return hipGetLastError();
}
