// gfx950 matrix-free upwind apply of the aMFP-BTE systems (paper: Appendix A,
// Eq. (iter2), left-hand side): y = (sigma + Lambda_m A_l) x, or with A_l^T,
// for a set of (m, l) systems at once.  Not on the pass path (the pass
// kernels solve the systems by sweeps); used by obte_upwind_apply.
#include "obte_internal.h"

namespace {

// ---------------------------------------------------------------------------
// Matrix-free upwind apply y = (sigma + Lambda_m A_l) x (or A_l^T) for a set
// of systems.  A block owns 256 consecutive cells and APPLY_SYS systems: the
// cell's face classes, sigma and neighbour indices are decoded once and
// reused for every system, the systems' coefficients are formed once per
// block (LDS), and a (cell, system) pair then costs its centre and upwind
// neighbour loads, a few FMAs and one store.  Cells are the fast index of
// both arrays, so centre loads and stores are coalesced, and neighbour loads
// fall on lines this block (x) or a recent block of the same system (y, z)
// fetched.  The loads of all systems are issued before the first store.
// ---------------------------------------------------------------------------
constexpr int APPLY_SYS = 8;

// The dispatcher hands consecutive workgroups to the eight XCDs in turn.
// Give each XCD a contiguous range of the logical (system group, cell tile)
// order instead, so the tiles one block's neighbour loads reach (the row and
// plane before, same system) were fetched into the same XCD's L2.
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_order(int w, int n) {
    const int per = n / N_XCD;
    return w < per * N_XCD ? (w % N_XCD) * per + w / N_XCD : w;
}

template <typename T>
__global__ void __launch_bounds__(256) k_apply(const GeomDev* __restrict__ gp, const double* __restrict__ sigma,
                                               const int* __restrict__ sys_ids, int n_sys,
                                               const T* __restrict__ x, T* __restrict__ y, int transpose) {
    __shared__ double coef[APPLY_SYS][3];   // Lambda_m |s_a| / h_a (0: no flux along a)
    __shared__ int from_plus[APPLY_SYS][3]; // 1: the upwind neighbour along a is on the + side
    __shared__ int valid[APPLY_SYS];
    const GeomDev& g = *gp;
    const int tiles = (g.ncells + 255) / 256;
    const int lb = xcd_order(blockIdx.x, gridDim.x);
    const int tile = lb % tiles;
    const int s0 = (lb / tiles) * APPLY_SYS;
    const int ns = min(APPLY_SYS, n_sys - s0);
    if (threadIdx.x < APPLY_SYS * 3) {
        const int k = threadIdx.x / 3, a = threadIdx.x % 3;
        const int sys = k < ns ? sys_ids[s0 + k] : -1;
        const bool ok = sys >= 0 && sys < g.n_sys;
        double c = 0.0;
        int plus = 0;
        if (ok && a < g.ndim) {
            const int m = sys / g.n_dir, l = sys % g.n_dir;
            double sa = g.dirs[l * 3 + a];
            if (transpose) sa = -sa;
            c = g.mfp[m] * fabs(sa) / g.h[a];
            plus = sa > 0.0 ? 0 : 1;
        }
        coef[k][a] = c;
        from_plus[k][a] = plus;
        if (a == 0) valid[k] = ok;
    }
    __syncthreads();
    const int cell = tile * blockDim.x + threadIdx.x;
    if (cell >= g.ncells) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const uint16_t w = g.fc[cell];
    const bool sol = fc_solid(w);
    const double sg = sigma ? sigma[cell] : 1.0;
    // both neighbours along every axis (periodic wrap; a wall side is masked
    // by its face class), decoded once for all systems
    const int ix = cell % nx, iy = (cell / nx) % ny, iz = cell / (nx * ny);
    int nb[3][2];
    bool open[3][2];
    nb[0][0] = cell + (ix > 0 ? -1 : nx - 1);
    nb[0][1] = cell + (ix < nx - 1 ? 1 : 1 - nx);
    nb[1][0] = cell + (iy > 0 ? -nx : nx * (ny - 1));
    nb[1][1] = cell + (iy < ny - 1 ? nx : -nx * (ny - 1));
    nb[2][0] = cell + (iz > 0 ? -nx * ny : nx * ny * (nz - 1));
    nb[2][1] = cell + (iz < nz - 1 ? nx * ny : -nx * ny * (nz - 1));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        open[a][0] = fc_class(w, 2 * a) != FC_WALL;
        open[a][1] = fc_class(w, 2 * a + 1) != FC_WALL;
    }
    const size_t nc = (size_t)g.ncells;
    T xc[APPLY_SYS], xn[APPLY_SYS][3];
    // loads of every system first (a missing system re-reads system 0)
#pragma unroll
    for (int k = 0; k < APPLY_SYS; ++k) {
        const T* xk = x + (size_t)(s0 + (k < ns ? k : 0)) * nc;
        xc[k] = xk[cell];
#pragma unroll
        for (int a = 0; a < 3; ++a) xn[k][a] = xk[from_plus[k][a] ? nb[a][1] : nb[a][0]];
    }
#pragma unroll
    for (int k = 0; k < APPLY_SYS; ++k) {
        if (k >= ns) break;
        double acc = sg * (double)xc[k];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double ca = coef[k][a];
            const bool op = from_plus[k][a] ? open[a][1] : open[a][0];
            acc += ca * (double)xc[k];
            acc -= op ? ca * (double)xn[k][a] : 0.0;
        }
        y[(size_t)(s0 + k) * nc + cell] = (sol && valid[k]) ? (T)acc : T(0);
    }
}

// N consecutive cells of one row per thread (32 bytes: four doubles or
// eight floats; rows of a multiple of N cells): the centre values, the
// upwind y and z neighbours and the store are 32-byte accesses, and the x
// neighbours come from the same registers except one value at the group's
// edge.  Per thread NS systems, whose loads are all issued before the first
// store; the results are written past the caches (streaming stores), so the
// L2 keeps the inputs the neighbouring tiles read again.
template <typename T, int N>
struct alignas(N * sizeof(T)) Vec {
    T v[N];
};

template <typename T, int NS, int N>
__global__ void __launch_bounds__(256) k_applyv(const GeomDev* __restrict__ gp, const double* __restrict__ sigma,
                                                const int* __restrict__ sys_ids, int n_sys,
                                                const T* __restrict__ x, T* __restrict__ y, int transpose) {
    __shared__ double coef[NS][3];
    __shared__ int from_plus[NS][3];
    __shared__ int valid[NS];
    const GeomDev& g = *gp;
    const int tiles = (g.ncells / N + 255) / 256;
    const int lb = xcd_order(blockIdx.x, gridDim.x);
    const int tile = lb % tiles;
    const int s0 = (lb / tiles) * NS;
    const int ns = min(NS, n_sys - s0);
    if (threadIdx.x < NS * 3) {
        const int k = threadIdx.x / 3, a = threadIdx.x % 3;
        const int sys = k < ns ? sys_ids[s0 + k] : -1;
        const bool ok = sys >= 0 && sys < g.n_sys;
        double c = 0.0;
        int plus = 0;
        if (ok && a < g.ndim) {
            const int m = sys / g.n_dir, l = sys % g.n_dir;
            double sa = g.dirs[l * 3 + a];
            if (transpose) sa = -sa;
            c = g.mfp[m] * fabs(sa) / g.h[a];
            plus = sa > 0.0 ? 0 : 1;
        }
        coef[k][a] = c;
        from_plus[k][a] = plus;
        if (a == 0) valid[k] = ok;
    }
    __syncthreads();
    const int c0 = N * (tile * blockDim.x + threadIdx.x);
    if (c0 >= g.ncells) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const bool d3 = g.ndim == 3;
    uint16_t w[N];
    double sg[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        w[j] = g.fc[c0 + j];
        sg[j] = sigma ? sigma[c0 + j] : 1.0;
    }
    const int ix = c0 % nx, iy = (c0 / nx) % ny, iz = c0 / (nx * ny);
    const int left = c0 + (ix > 0 ? -1 : nx - 1);                          // x neighbour of the first cell, - side
    const int right = c0 + N - 1 + (ix + N - 1 < nx - 1 ? 1 : 1 - nx);     // of the last cell, + side
    const int ym = c0 + (iy > 0 ? -nx : nx * (ny - 1)), yp = c0 + (iy < ny - 1 ? nx : -nx * (ny - 1));
    const int zm = c0 + (iz > 0 ? -nx * ny : nx * ny * (nz - 1));
    const int zp = c0 + (iz < nz - 1 ? nx * ny : -nx * ny * (nz - 1));
    const size_t nc = (size_t)g.ncells;
    Vec<T, N> xc[NS], xy[NS], xz[NS];
    T xb[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const T* xk = x + (size_t)(s0 + (k < ns ? k : 0)) * nc;
        xc[k] = *reinterpret_cast<const Vec<T, N>*>(xk + c0);
        xb[k] = xk[from_plus[k][0] ? right : left];
        xy[k] = *reinterpret_cast<const Vec<T, N>*>(xk + (from_plus[k][1] ? yp : ym));
        if (d3) xz[k] = *reinterpret_cast<const Vec<T, N>*>(xk + (from_plus[k][2] ? zp : zm));
        else xz[k] = xc[k];
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        if (k >= ns) break;
        const int px = from_plus[k][0], py = from_plus[k][1], pz = from_plus[k][2];
        const double cx = coef[k][0], cy = coef[k][1], cz = coef[k][2];
        T* yk = y + (size_t)(s0 + k) * nc + c0;
        Vec<T, N> out;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const double xv = (double)xc[k].v[j];
            const T xl = j > 0 ? xc[k].v[j > 0 ? j - 1 : 0] : xb[k];
            const T xr = j < N - 1 ? xc[k].v[j < N - 1 ? j + 1 : N - 1] : xb[k];
            double acc = sg[j] * xv;
            acc += cx * xv;
            acc -= fc_class(w[j], px) != FC_WALL ? cx * (double)(px ? xr : xl) : 0.0;
            acc += cy * xv;
            acc -= fc_class(w[j], 2 + py) != FC_WALL ? cy * (double)xy[k].v[j] : 0.0;
            acc += cz * xv;
            acc -= (d3 && fc_class(w[j], 4 + pz) != FC_WALL) ? cz * (double)xz[k].v[j] : 0.0;
            out.v[j] = (fc_solid(w[j]) && valid[k]) ? (T)acc : T(0);
        }
        // 16-byte streaming stores of the group
        using V16 = T __attribute__((ext_vector_type(16 / sizeof(T))));
        constexpr int E = 16 / sizeof(T);
#pragma unroll
        for (int h = 0; h < N / E; ++h) {
            V16 v;
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = out.v[h * E + e];
            __builtin_nontemporal_store(v, reinterpret_cast<V16*>(yk) + h);
        }
    }
}

}  // namespace

hipError_t launch_apply(int precision, int transpose, const GeomDev* g_dev, const GeomDev& g_host,
                        const double* sigma, const int* sys_ids, int n_sys, const void* x, void* y,
                        hipStream_t st) {
    (void)hipGetLastError();
    // the vector form: rows of a multiple of N cells (32 bytes of values per
    // thread) and 32-byte aligned x, y, so that no access straddles a row or
    // is misaligned
    const int N = precision == 0 ? 4 : 8;
    const bool vec = g_host.nx % N == 0 && (uintptr_t)x % 32 == 0 && (uintptr_t)y % 32 == 0;
    if (vec) {
        constexpr int NS = 4;
        const int groups = (g_host.ncells / N + 255) / 256 * ((n_sys + NS - 1) / NS);
        if (precision == 0)
            hipLaunchKernelGGL((k_applyv<double, NS, 4>), dim3(groups), dim3(256), 0, st, g_dev, sigma, sys_ids,
                               n_sys, (const double*)x, (double*)y, transpose);
        else
            hipLaunchKernelGGL((k_applyv<float, NS, 8>), dim3(groups), dim3(256), 0, st, g_dev, sigma, sys_ids,
                               n_sys, (const float*)x, (float*)y, transpose);
        return hipGetLastError();
    }
    dim3 grid((g_host.ncells + 255) / 256 * ((n_sys + APPLY_SYS - 1) / APPLY_SYS));
    if (precision == 0)
        hipLaunchKernelGGL(k_apply<double>, grid, dim3(256), 0, st, g_dev, sigma, sys_ids, n_sys,
                           (const double*)x, (double*)y, transpose);
    else
        hipLaunchKernelGGL(k_apply<float>, grid, dim3(256), 0, st, g_dev, sigma, sys_ids, n_sys,
                           (const float*)x, (float*)y, transpose);
    return hipGetLastError();
}
