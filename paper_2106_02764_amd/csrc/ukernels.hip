// gfx950 kernels of the unstructured-mesh path (paper: section Geometry
// module; Appendix A with general face vectors R_ij = A_ij n_ij / V_i;
// Appendix B, heat conduction with the non-orthogonal correction).
//
// Heat conduction (Eq. (final2)): the primary flux is implicit, the
// secondary flux explicit.  One workgroup runs the whole outer iteration of
// a mesh: least-squares cell gradients of the current T, the secondary flux
// of every face, then a conjugate-gradient solve of the volume-scaled
// primary-flux Laplacian (warm-started from the current T), until T stops
// changing.
//
// Transport: one wavefront owns one (m, l) system.  Within a direction the
// cells are ordered upwind (the host sorts them into levels whose cells
// depend only on earlier levels, the periodic faces cut), so a sweep is one
// pass over the levels with the solution in LDS.  The values entering
// through periodic faces form the system's wrap vector u; BiCGSTAB solves
// (I - G) e = r for its correction, G being one sweep with u as the only
// source, as on the structured grids.  All sums are in a fixed order: FP64
// results are bitwise reproducible.
#include "umesh_internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int UF_THREADS = 1024;

__device__ __forceinline__ double shfl_xor(double v, int m) { return __shfl_xor(v, m, WAVE); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, shfl_xor(v, m));
    return v;
}

// Block-wide sum (every thread gets the same value; waves combined in order).
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[k];
    return s;
}

// N block-wide sums in one exchange (each value summed as block_sum does;
// red: at least 16 N doubles)
template <int N>
__device__ void block_sum_n(double (&v)[N], double* red) {
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = wave_sum(v[n]);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int n = 0; n < N; ++n) red[n * 16 + w] = v[n];
    __syncthreads();
#pragma unroll
    for (int n = 0; n < N; ++n) {
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += red[n * 16 + k];
        v[n] = s;
    }
}

__device__ double block_max(double v, double* red) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s = fmax(s, red[k]);
    return s;
}

// ---------------------------------------------------------------------------
// heat conduction with the explicit secondary flux
// ---------------------------------------------------------------------------
__device__ __forceinline__ void uface_gradient(const UFourierDev& f, int fc, double& gx, double& gy) {
    const int i = f.fi[fc], j = f.fj[fc];
    const double w = f.fw[fc];
    gx = (1.0 - w) * f.g[2 * i] + w * f.g[2 * j];
    gy = (1.0 - w) * f.g[2 * i + 1] + w * f.g[2 * j + 1];
}

// (A x)_i for A = minus the volume-scaled primary-flux Laplacian
__device__ __forceinline__ double uapply(const UFourierDev& f, const double* x, int i) {
    double y = 0.0;
    const double xi = x[i];
    for (int k = f.nb_ptr[i]; k < f.nb_ptr[i + 1]; ++k) y += f.nb_a[k] * (xi - x[f.nb_j[k]]);
    return y;
}

__device__ __forceinline__ double udiag(const UFourierDev& f, int i) {
    double d = 0.0;
    for (int k = f.nb_ptr[i]; k < f.nb_ptr[i + 1]; ++k) d += f.nb_a[k];
    return d > 0.0 ? d : 1.0;
}

// ---- the outer iteration over several blocks of UFB cells.  Every sum is
// taken as per-block partials that each consumer adds in block order, so
// every block takes the same decisions and FP64 results are reproducible.
constexpr int UFB = 256;
enum { UP_RR0, UP_RR1, UP_G0, UP_G1, UP_D0, UP_D1, UP_BB, UP_ST, UP_DM, UP_TM };
static_assert(UP_TM + 1 == UF_SLOTS, "partial slots of the heat-conduction kernels");

__host__ __device__ __forceinline__ int uf_blocks(int ns) { return (ns + UFB - 1) / UFB; }

// fixed-order sum (or max) of the B partials of a slot, in every thread
__device__ __forceinline__ double uf_sum(const UFourierDev& f, int slot, int B, double* red) {
    const double v = (int)threadIdx.x < B ? f.fpart[slot * UF_MAXB + threadIdx.x] : 0.0;
    return block_sum(v, red);
}
__device__ __forceinline__ double uf_max(const UFourierDev& f, int slot, int B, double* red) {
    const double v = (int)threadIdx.x < B ? f.fpart[slot * UF_MAXB + threadIdx.x] : 0.0;
    return block_max(v, red);
}

__device__ __forceinline__ void ucell_gradient(const UFourierDev& f, int i) {
    double gx = 0.0, gy = 0.0;
    const double Ti = f.T[i];
    for (int k = f.nb_ptr[i]; k < f.nb_ptr[i + 1]; ++k) {
        const double q = f.T[f.nb_j[k]] + f.nb_del[k] * f.dT - Ti;
        gx += f.nb_w[2 * k] * q;
        gy += f.nb_w[2 * k + 1] * q;
    }
    f.g[2 * i] = gx;
    f.g[2 * i + 1] = gy;
}

// cell gradients of the current T
__global__ void __launch_bounds__(UFB) k_uf_grad(const UFourierDev* __restrict__ fp) {
    const UFourierDev& f = *fp;
    const int i = blockIdx.x * UFB + threadIdx.x;
    if (i < f.ns) ucell_gradient(f, i);
}

// the secondary flux of every face from the interpolated face gradient
__global__ void __launch_bounds__(UFB) k_uf_face(const UFourierDev* __restrict__ fp) {
    const UFourierDev& f = *fp;
    const int fc = blockIdx.x * UFB + threadIdx.x;
    if (fc >= f.nfaces) return;
    double gx, gy;
    uface_gradient(f, fc, gx, gy);
    f.bf[fc] = gx * f.fc[2 * fc] + gy * f.fc[2 * fc + 1];
}

// b = -(P + B) (the right-hand side of A T = b, A = -Laplacian), the previous
// iterate, the diagonal and the first residual r = b - A T (warm start from
// T); partials of |b|^2 and r.r.  The CG's direction p and its image s of
// the iteration before the first are 0.
__global__ void __launch_bounds__(UFB) k_uf_init(const UFourierDev* __restrict__ fp) {
    __shared__ double red[UFB / 64];
    const UFourierDev& f = *fp;
    const int i = blockIdx.x * UFB + threadIdx.x;
    double bb = 0.0, rr = 0.0;
    if (i < f.ns) {
        double s = f.P[i];
        for (int k = f.nb_ptr[i]; k < f.nb_ptr[i + 1]; ++k) {
            const int code = f.nb_f[k];
            const double v = f.bf[code >> 1];
            s += (code & 1) ? -v : v;
        }
        const double ri = -s - uapply(f, f.T, i);
        f.tp[i] = f.T[i];
        f.dg[i] = udiag(f, i);
        f.r[i] = ri;
        f.p[i] = 0.0;
        f.s0[i] = 0.0;             // read as the previous s by the first iteration (parity 0)
        bb = s * s;
        rr = ri * ri;
    }
    bb = block_sum(bb, red);
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        f.fpart[UP_BB * UF_MAXB + blockIdx.x] = bb;
        f.fpart[UP_RR0 * UF_MAXB + blockIdx.x] = rr;
        if (blockIdx.x == 0) {
            f.fsc[0] = 0.0;            // this solve's CG runs
            f.fsc[10] = 0.0;           // iterations done before the next one of parity 0
        }
    }
}

// w = A u with u = M^-1 r (M the diagonal) for the first residual, and the
// partials of gamma = r.u and delta = w.u (parity 0)
__global__ void __launch_bounds__(UFB) k_uf_w0(const UFourierDev* __restrict__ fp) {
    __shared__ double red[UFB / 64];
    const UFourierDev& f = *fp;
    const int i = blockIdx.x * UFB + threadIdx.x;
    double gm = 0.0, dl = 0.0;
    if (i < f.ns) {
        const double ui = f.r[i] / f.dg[i];
        double w = 0.0;
        for (int k = f.nb_ptr[i]; k < f.nb_ptr[i + 1]; ++k) {
            const int j = f.nb_j[k];
            w += f.nb_a[k] * (ui - f.r[j] / f.dg[j]);
        }
        f.w0[i] = w;
        gm = f.r[i] * ui;
        dl = w * ui;
    }
    gm = block_sum(gm, red);
    dl = block_sum(dl, red);
    if (threadIdx.x == 0) {
        f.fpart[UP_G0 * UF_MAXB + blockIdx.x] = gm;
        f.fpart[UP_D0 * UF_MAXB + blockIdx.x] = dl;
    }
}

// One preconditioned CG iteration in the Chronopoulos-Gear arrangement (one
// kernel: both inner products of an iteration come from one pass).  With u =
// M^-1 r, w = A u and s = A p carried by recurrence, iteration k (parity q):
//   gamma = r.u, delta = w.u (partials of parity q), the stop test on r.r;
//   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma /
//   alpha_prev)  (k = 0: beta = 0, alpha = gamma / delta);
//   p = u + beta p, s = w + beta s, T += alpha p, r' = r - alpha s,
//   u' = M^-1 r', w' = A u', and the partials of r'.u', w'.u', r'.r'.
// r, w and s are double buffered by parity (r0 = r, r1), and A u' at a cell
// needs u' at its neighbours, which every block forms from the unchanged
// parity-q buffers.  Scalars: fsc[6 + q] gamma, fsc[8 + q] alpha and
// fsc[10 + q] the iterations done before an iteration of parity q.
__global__ void __launch_bounds__(UFB) k_uf_cg(const UFourierDev* __restrict__ fp, int q, double cg_tol,
                                               int max_cg) {
    __shared__ double red[4 * 16];
    const UFourierDev& f = *fp;
    if (f.fsc[0] != 0.0) return;
    const int B = uf_blocks(f.ns);
    // the four sums of the partials in one exchange (block order, as uf_sum)
    double sm[4] = {0.0, 0.0, 0.0, 0.0};
    if ((int)threadIdx.x < B) {
        sm[0] = f.fpart[(UP_RR0 + q) * UF_MAXB + threadIdx.x];
        sm[1] = f.fpart[UP_BB * UF_MAXB + threadIdx.x];
        sm[2] = f.fpart[(UP_G0 + q) * UF_MAXB + threadIdx.x];
        sm[3] = f.fpart[(UP_D0 + q) * UF_MAXB + threadIdx.x];
    }
    block_sum_n(sm, red);
    const double rr = sm[0], bb = sm[1], gam = sm[2], del = sm[3];
    const int it = (int)f.fsc[10 + q];
    double alpha = gam / del, beta = 0.0;
    if (it > 0) {
        beta = gam / f.fsc[6 + (q ^ 1)];
        alpha = gam / (del - beta * gam / f.fsc[8 + (q ^ 1)]);
    }
    if (!(rr > cg_tol * cg_tol * bb) || it >= max_cg || !(alpha > 0.0) || !isfinite(alpha)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) f.fsc[0] = 1.0;
        return;
    }
    const double* r = q ? f.r1 : f.r;
    const double* w = q ? f.w1 : f.w0;
    const double* so = q ? f.s1 : f.s0;       // s of the previous iteration (parity q ^ 1 wrote it here)
    double* rn = q ? f.r : f.r1;
    double* wn = q ? f.w0 : f.w1;
    double* sn = q ? f.s0 : f.s1;
    const int i = blockIdx.x * UFB + threadIdx.x;
    double gm = 0.0, dl = 0.0, r2 = 0.0;
    if (i < f.ns) {
        const double pc = r[i] / f.dg[i] + beta * f.p[i];
        const double sc = w[i] + beta * so[i];
        f.p[i] = pc;
        f.T[i] += alpha * pc;
        const double ri = r[i] - alpha * sc;
        const double ui = ri / f.dg[i];
        double wv = 0.0;
        for (int k = f.nb_ptr[i]; k < f.nb_ptr[i + 1]; ++k) {
            const int j = f.nb_j[k];
            const double rj = r[j] - alpha * (w[j] + beta * so[j]);
            wv += f.nb_a[k] * (ui - rj / f.dg[j]);
        }
        rn[i] = ri;
        wn[i] = wv;
        sn[i] = sc;
        gm = ri * ui;
        dl = wv * ui;
        r2 = ri * ri;
    }
    double en[3] = {gm, dl, r2};
    block_sum_n(en, red);
    if (threadIdx.x == 0) {
        f.fpart[(UP_G0 + (q ^ 1)) * UF_MAXB + blockIdx.x] = en[0];
        f.fpart[(UP_D0 + (q ^ 1)) * UF_MAXB + blockIdx.x] = en[1];
        f.fpart[(UP_RR0 + (q ^ 1)) * UF_MAXB + blockIdx.x] = en[2];
        if (blockIdx.x == 0) {
            f.fsc[6 + q] = gam;
            f.fsc[8 + q] = alpha;
            f.fsc[10 + (q ^ 1)] = (double)(it + 1);
            f.fsc[2] += 1.0;
        }
    }
}

// end of an outer iteration: partials of the sum of T ...
__global__ void __launch_bounds__(UFB) k_uf_sum(const UFourierDev* __restrict__ fp) {
    __shared__ double red[UFB / 64];
    const UFourierDev& f = *fp;
    const int i = blockIdx.x * UFB + threadIdx.x;
    const double v = block_sum(i < f.ns ? f.T[i] : 0.0, red);
    if (threadIdx.x == 0) f.fpart[UP_ST * UF_MAXB + blockIdx.x] = v;
}

// ... the mean removed, and partials of max |T - T_prev| and max |T|
__global__ void __launch_bounds__(UFB) k_uf_center(const UFourierDev* __restrict__ fp) {
    __shared__ double red[UFB / 64];
    const UFourierDev& f = *fp;
    const double mean = uf_sum(f, UP_ST, uf_blocks(f.ns), red) / (double)f.ns;
    const int i = blockIdx.x * UFB + threadIdx.x;
    double dmax = 0.0, tmax = 0.0;
    if (i < f.ns) {
        const double v = f.T[i] - mean;
        f.T[i] = v;
        dmax = fabs(v - f.tp[i]);
        tmax = fabs(v);
    }
    dmax = block_max(dmax, red);
    tmax = block_max(tmax, red);
    if (threadIdx.x == 0) {
        f.fpart[UP_DM * UF_MAXB + blockIdx.x] = dmax;
        f.fpart[UP_TM * UF_MAXB + blockIdx.x] = tmax;
    }
}

// ... the change and the outer stop test (one block)
__global__ void __launch_bounds__(UFB) k_uf_change(const UFourierDev* __restrict__ fp, double tol) {
    __shared__ double red[UFB / 64];
    const UFourierDev& f = *fp;
    const int B = uf_blocks(f.ns);
    const double dmax = uf_max(f, UP_DM, B, red), tmax = uf_max(f, UP_TM, B, red);
    if (threadIdx.x == 0) {
        f.fsc[3] += 1.0;
        f.fsc[4] = tmax > 0.0 ? dmax / tmax : 0.0;
        f.fsc[5] = dmax <= tol * fmax(tmax, 1e-300) ? 1.0 : 0.0;
    }
}

// kappa_F: the total face flux (primary + secondary) across the periodic
// plane of the gradient axis, from the final T's gradients (one block; the
// gradients are taken by k_uf_grad before it); the statistics into out
__global__ void __launch_bounds__(UF_THREADS) k_uf_kappa(const UFourierDev* __restrict__ fp) {
    __shared__ double red[UF_THREADS / 64];
    const UFourierDev& f = *fp;
    double tot = 0.0;
    for (int c = threadIdx.x; c < f.ncut; c += blockDim.x) {
        const int fc = f.cut_f[c];
        double gx, gy;
        uface_gradient(f, fc, gx, gy);
        const int ip = f.cut_s[c] > 0 ? f.fi[fc] : f.fj[fc];
        const int jn = f.cut_s[c] > 0 ? f.fj[fc] : f.fi[fc];
        const double a = f.cut_K[3 * c], kx = f.cut_K[3 * c + 1], ky = f.cut_K[3 * c + 2];
        const double gd = gx * f.cut_d[2 * c] + gy * f.cut_d[2 * c + 1];
        // a = n.K n / (n.d); the secondary part g.K n - (n.K n)(g.d)/(n.d)
        tot += f.cut_A[c] * (a * (f.T[jn] + f.dT - f.T[ip]) + (gx * kx + gy * ky) - a * gd);
    }
    tot = block_sum(tot, red);
    if (threadIdx.x == 0) {
        f.out[0] = f.Lg / (f.dT * f.Aperp) * tot;
        f.out[1] = f.fsc[3];
        f.out[2] = f.fsc[2];
        f.out[3] = f.fsc[4];
    }
}

// ---------------------------------------------------------------------------
// transport: one pass for every system
// ---------------------------------------------------------------------------
struct USys {
    int sys, l, lb, nlev, nw;
    double lam;
    const int* up;
    const double* del;
};

// One sweep of the system: x (LDS) from the sources (src: sigma T_L and the
// wall values; else none) and the wrap inflow staged in LDS.  The workgroup
// is one wavefront, whose LDS accesses are executed in program order, so
// level k + 1 reads what level k wrote without a barrier; the table entries
// of a lane's cell in the next level (independent of the solution, and all
// indexed by the sweep position: the pass's sources are packed in sweep
// order by k_upack) are loaded two levels ahead of their solve.
struct UEnt {
    int i;
    double d, sg, b;              // outflow sum, sigma, sigma T_L + the wall inflow
    int code[UFACES];             // cell / wrap-slot inflows (walls folded into b)
    double c[UFACES];
};

__device__ __forceinline__ void ufetch(const UGeomDev& g, const USys& s, bool src, int p, UEnt& e) {
    const size_t pl = (size_t)s.l * g.ns + p;
    e.i = g.ord[pl];
    e.d = g.dout[pl];
    e.sg = g.psg[pl];
    const double b0 = g.pb0[pl], bw = g.pbw[pl];
#pragma unroll
    for (int q = 0; q < UFACES; ++q) {
        const int code = g.inc[pl * UFACES + q];
        e.code[q] = code <= UWALL0 ? UNONE : code;
        e.c[q] = g.inv[pl * UFACES + q];
    }
    e.b = src ? b0 + s.lam * bw : 0.0;
}

// The pass's sources in every direction's sweep order: sigma, sigma T_L and
// the inflow wall sum of the cell at each position (one thread per position).
__global__ void __launch_bounds__(256) k_upack(const UGeomDev* __restrict__ gp) {
    const UGeomDev& g = *gp;
    const size_t n = (size_t)g.n_dir * g.ns;
    for (size_t pl = (size_t)blockIdx.x * blockDim.x + threadIdx.x; pl < n; pl += (size_t)gridDim.x * blockDim.x) {
        const int i = g.ord[pl];
        double wall = 0.0;
#pragma unroll
        for (int q = 0; q < UFACES; ++q) {
            const int code = g.inc[pl * UFACES + q];
            const bool w = code <= UWALL0;
            wall += w ? g.inv[pl * UFACES + q] * g.T_w[UWALL0 - code] : 0.0;
        }
        const double sg = g.sigma[i];
        g.psg[pl] = sg;
        g.pb0[pl] = sg * g.T_L[i];
        g.pbw[pl] = wall;
    }
}

// The wrap inflow follows the solution in LDS (uin = x + ns), so an inflow
// code indexes both: x[code] is the upwind cell's value for code < ns and the
// wrap slot's for code >= ns; unused faces read x[0] and drop it (no branch).
__device__ __forceinline__ void usolve(const UGeomDev& g, const USys& s, const UEnt& e, double* x, const double* uin) {
    (void)uin;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < UFACES; ++q) {
        const int code = e.code[q];
        const double v = x[code >= 0 ? code : 0];       // read always, selected
        acc += code >= 0 ? e.c[q] * v : 0.0;
    }
    x[e.i] = (e.b + s.lam * acc) / (e.sg + s.lam * e.d);
}

__device__ void usweep(const UGeomDev& g, const USys& s, bool src, double* x, const double* uin) {
    const int lane = threadIdx.x;
    // level k spans positions [lp[k], lp[k + 1]); past the last level the
    // bounds clamp to its end (empty ranges).  At level k the entries of level
    // k + 2 are fetched (two levels of loads in flight) and the bound that
    // ends level k + 3 is loaded a level before it is needed.
    const int* lp = g.lptr + s.lb;
    const int L = s.nlev;
    auto bound = [&](int k) { return lp[k < L ? k : L]; };
    int a0 = bound(0), a1 = bound(1), e1 = bound(2), e2 = bound(3);
    // every lane fetches (beyond its level: the level's last entry, or the
    // first position), so no load sits in a branch: the compiler then counts
    // the loads in flight exactly and waits only for the level it solves
    auto pos = [&](int lo, int hi) { return lo + lane < hi ? lo + lane : (hi > 0 ? hi - 1 : 0); };
    UEnt cur, nxt, nx2;
    ufetch(g, s, src, pos(a0, a1), cur);
    ufetch(g, s, src, pos(a1, e1), nxt);
    for (int k = 0; k < L; ++k) {
        const int e3 = bound(k + 4);
        ufetch(g, s, src, pos(e1, e2), nx2);
        if (a0 + lane < a1) usolve(g, s, cur, x, uin);
        for (int p = a0 + lane + WAVE; p < a1; p += WAVE) {
            UEnt e;
            ufetch(g, s, src, p, e);
            usolve(g, s, e, x, uin);
        }
        // keeps the compiler from moving this level's LDS accesses past the
        // next level's
        __builtin_amdgcn_wave_barrier();
        cur = nxt;
        nxt = nx2;
        a0 = a1;
        a1 = e1;
        e1 = e2;
        e2 = e3;
    }
}

template <int WPL>
__device__ __forceinline__ void ustage(const USys& s, const double (&v)[WPL], double* uin) {
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const int q = k * WAVE + threadIdx.x;
        if (q < s.nw) uin[q] = v[k];
    }
    __builtin_amdgcn_wave_barrier();
}

// G v: the values a homogeneous sweep with inflow v carries back across the
// periodic faces
template <int WPL>
__device__ __forceinline__ void ugather(const USys& s, const double* x, double (&out)[WPL]) {
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const int q = k * WAVE + threadIdx.x;
        out[k] = q < s.nw ? x[s.up[q]] : 0.0;
    }
}

template <int WPL>
__device__ __forceinline__ double udot(const double (&a)[WPL], const double (&b)[WPL]) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < WPL; ++k) v += a[k] * b[k];
    return wave_sum(v);
}

template <int WPL>
__global__ void __launch_bounds__(WAVE) k_upass(const UGeomDev* __restrict__ gp, double inner_tol, double inner_rtol,
                                                int max_inner) {
    extern __shared__ double lds[];
    const UGeomDev& g = *gp;
    const int lane = threadIdx.x;
    USys s;
    // longest MFPs first (they take the most wrap iterations); the direction
    // is the fast index, so with the workgroups dealt to the eight XCDs in
    // turn each XCD sweeps a fixed subset of the directions and their tables
    // stay in its L2
    s.l = (int)blockIdx.x % g.n_dir;
    const int m = g.n_mfp - 1 - (int)blockIdx.x / g.n_dir;
    s.sys = m * g.n_dir + s.l;
    s.lam = g.mfp[m];
    s.lb = g.lbase[s.l];
    s.nlev = g.nlev[s.l];
    s.nw = g.nwrap[s.l];
    s.up = g.wup + (size_t)s.l * g.wmax;
    s.del = g.wdel + (size_t)s.l * g.wmax;
    double* x = lds;
    double* uin = lds + g.ns;
    double* U = g.U + (size_t)s.sys * g.wmax;
    double u[WPL], ez[WPL], r[WPL];
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const int q = k * WAVE + lane;
        u[k] = q < s.nw ? U[q] : 0.0;
    }
    // ---- the sweep with the sources and the wrap inflow of the last pass
    ustage(s, u, uin);
    usweep(g, s, true, x, uin);
    ugather(s, x, ez);
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
        const int q = k * WAVE + lane;
        if (q < s.nw) ez[k] += s.del[q];
        r[k] = ez[k] - u[k];
    }
    const double scale = sqrt(udot(ez, ez));
    double rn = sqrt(udot(r, r));
    long long its = 0;
    // this pass's target: inner_tol relative to the inflow, or (forcing
    // term) a cut by inner_rtol of the residual the pass started from; the
    // rest carries into the next pass through U
    const double thr = fmax(inner_tol * scale, inner_rtol * rn);
    if (s.nw > 0 && scale > 0.0 && rn > thr) {
        // ---- BiCGSTAB on (I - G) e = r, the best iterate kept
        double e[WPL], eb[WPL], rh[WPL], p[WPL], v[WPL], sv[WPL], tt[WPL], gx[WPL];
#pragma unroll
        for (int k = 0; k < WPL; ++k) {
            e[k] = 0.0; eb[k] = 0.0; rh[k] = r[k]; p[k] = 0.0; v[k] = 0.0;
        }
        double best = rn, rho_old = 1.0, alpha = 1.0, omega = 1.0;
        int restarts = 0;
        for (int it = 0; it < max_inner; ++it) {
            double rho = udot(rh, r);
            if (fabs(rho) <= 1e-30 * rn * rn || !(omega != 0.0)) {
#pragma unroll
                for (int k = 0; k < WPL; ++k) { rh[k] = r[k]; p[k] = 0.0; v[k] = 0.0; }
                rho = udot(r, r);
                rho_old = 1.0; alpha = 1.0; omega = 1.0;
            }
            const double beta = (rho / rho_old) * (alpha / omega);
#pragma unroll
            for (int k = 0; k < WPL; ++k) p[k] = r[k] + beta * (p[k] - omega * v[k]);
            ustage(s, p, uin);
            usweep(g, s, false, x, uin);
            ugather(s, x, gx);
#pragma unroll
            for (int k = 0; k < WPL; ++k) v[k] = p[k] - gx[k];
            const double rv = udot(rh, v);
            if (!isfinite(rv)) break;
            if (!(fabs(rv) > 1e-30 * fabs(rho))) {
                if (restarts++ >= 4) break;
                omega = 0.0;
                continue;
            }
            alpha = rho / rv;
#pragma unroll
            for (int k = 0; k < WPL; ++k) sv[k] = r[k] - alpha * v[k];
            const double sn = sqrt(udot(sv, sv));
            ++its;
            if (sn <= thr) {
#pragma unroll
                for (int k = 0; k < WPL; ++k) e[k] += alpha * p[k];
                if (sn < best) {
                    best = sn;
#pragma unroll
                    for (int k = 0; k < WPL; ++k) eb[k] = e[k];
                }
                break;
            }
            ustage(s, sv, uin);
            usweep(g, s, false, x, uin);
            ugather(s, x, gx);
#pragma unroll
            for (int k = 0; k < WPL; ++k) tt[k] = sv[k] - gx[k];
            const double t2 = udot(tt, tt);
            omega = t2 > 0.0 ? udot(tt, sv) / t2 : 0.0;
#pragma unroll
            for (int k = 0; k < WPL; ++k) {
                e[k] += alpha * p[k] + omega * sv[k];
                r[k] = sv[k] - omega * tt[k];
            }
            rn = sqrt(udot(r, r));
            rho_old = rho;
            if (!isfinite(rn)) break;
            if (rn < best) {
                best = rn;
#pragma unroll
                for (int k = 0; k < WPL; ++k) eb[k] = e[k];
            }
            if (rn <= thr) break;
        }
        rn = best;
        // ---- the corrected inflow, and the final sweep with it
#pragma unroll
        for (int k = 0; k < WPL; ++k) {
            u[k] += eb[k];
            const int q = k * WAVE + lane;
            if (q < s.nw) U[q] = u[k];
        }
        ustage(s, u, uin);
        usweep(g, s, true, x, uin);
    }
    // ---- the stored solution and this system's kappa shares
    double kc = 0.0;
    double* X = g.X + (size_t)s.sys * g.ns;
    for (int i = lane; i < g.ns; i += WAVE) {
        const double xv = x[i];
        X[i] = xv;
        kc += g.V[i] * xv;
    }
    kc = wave_sum(kc);
    const double Sx = g.S[2 * s.sys], Sy = g.S[2 * s.sys + 1];
    double kf = 0.0;
    for (int c = lane; c < g.ncut; c += WAVE) {
        const double sn = Sx * g.cut_An[2 * c] + Sy * g.cut_An[2 * c + 1];     // A_f S . n
        const double up = sn > 0.0 ? x[g.cut_i[c]] : x[g.cut_j[c]] + g.dT;
        kf -= sn * up;                 // flow from the + side cell out across the cut
    }
    kf = wave_sum(kf);
    if (lane == 0) {
        const double Sg = g.S[2 * s.sys + g.grad_axis];
        g.ksys[s.sys] = g.Lg / (g.dT * g.Vbox) * Sg * kc;
        g.kfsys[s.sys] = g.Lg / (g.dT * g.Aperp) * kf;
        g.iters[s.sys] += its;
        g.wres[s.sys] = scale > 0.0 ? rn / scale : 0.0;
    }
}

// T_L = sum D x per cell, T_w = sum of the outgoing weights times x at the
// wall's cell.  A block owns 64 cells (or 64 wall faces); its UQ waves sum
// fixed chunks of the systems, combined in order.
constexpr int UQ = 16;

__global__ void __launch_bounds__(64 * UQ) k_ureduce(const UGeomDev* __restrict__ gp) {
    __shared__ double part[UQ][64];
    const UGeomDev& g = *gp;
    const int q = threadIdx.x >> 6, cl = threadIdx.x & 63;
    const int cblocks = (g.ns + 63) / 64;
    const bool walls = (int)blockIdx.x >= cblocks;
    const int t = (walls ? (int)blockIdx.x - cblocks : (int)blockIdx.x) * 64 + cl;
    const int n = walls ? g.nwalls : g.ns;
    const bool in = t < n;
    const int cell = in ? (walls ? g.wcell[t] : t) : 0;
    const int per = (g.n_sys + UQ - 1) / UQ;
    const int i0 = q * per, i1 = min(g.n_sys, i0 + per);
    // eight systems' values in flight per lane, four running sums
    auto wgt = [&](int k) { return walls ? (in ? g.wout[(size_t)t * g.n_sys + k] : 0.0) : g.Dw[k]; };
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = i0;
    for (; i + 7 < i1; i += 8) {
        double xv[8], wv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = g.X[(size_t)(i + u) * g.ns + cell];
#pragma unroll
        for (int u = 0; u < 8; ++u) wv[u] = wgt(i + u);
        a0 += wv[0] * xv[0];
        a1 += wv[1] * xv[1];
        a2 += wv[2] * xv[2];
        a3 += wv[3] * xv[3];
        a0 += wv[4] * xv[4];
        a1 += wv[5] * xv[5];
        a2 += wv[6] * xv[6];
        a3 += wv[7] * xv[7];
    }
    for (; i < i1; ++i) a0 += wgt(i) * g.X[(size_t)i * g.ns + cell];
    part[q][cl] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (q == 0 && in) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < UQ; ++u) acc += part[u][cl];
        if (walls) g.T_w[t] = acc;
        else g.T_L[t] = acc;
    }
}

__global__ void __launch_bounds__(256) k_ukappa(const UGeomDev* __restrict__ gp) {
    __shared__ double red[4];
    const UGeomDev& g = *gp;
    double a = 0.0, b = 0.0, w = 0.0;
    // fixed order: each thread a contiguous chunk, then the block in order
    const int per = (g.n_sys + blockDim.x - 1) / blockDim.x;
    const int i0 = threadIdx.x * per, i1 = min(g.n_sys, i0 + per);
    for (int i = i0; i < i1; ++i) {
        a += g.ksys[i];
        b += g.kfsys[i];
        w = fmax(w, g.wres[i]);
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    w = block_max(w, red);
    if (threadIdx.x == 0) {
        g.kap[0] = a;
        g.kap[1] = b;
        g.kap[2] = w;
    }
}

}  // namespace

hipError_t ulaunch_fourier_start(const UFourierDev* f_dev, int ns, int nfaces, hipStream_t st) {
    (void)hipGetLastError();
    const int B = uf_blocks(ns), BF = (nfaces + UFB - 1) / UFB;
    hipLaunchKernelGGL(k_uf_grad, dim3(B), dim3(UFB), 0, st, f_dev);
    if (BF > 0) hipLaunchKernelGGL(k_uf_face, dim3(BF), dim3(UFB), 0, st, f_dev);
    hipLaunchKernelGGL(k_uf_init, dim3(B), dim3(UFB), 0, st, f_dev);
    hipLaunchKernelGGL(k_uf_w0, dim3(B), dim3(UFB), 0, st, f_dev);
    return hipGetLastError();
}

hipError_t ulaunch_fourier_cg(const UFourierDev* f_dev, int ns, int iters, double cg_tol, int max_cg,
                              hipStream_t st) {
    (void)hipGetLastError();
    const int B = uf_blocks(ns);
    for (int k = 0; k < iters; ++k) {
        // the parity of an iteration is its count's, which is even at the
        // start of every chunk (chunks are even and a solve starts at 0)
        hipLaunchKernelGGL(k_uf_cg, dim3(B), dim3(UFB), 0, st, f_dev, k & 1, cg_tol, max_cg);
    }
    return hipGetLastError();
}

hipError_t ulaunch_fourier_end(const UFourierDev* f_dev, int ns, double tol, hipStream_t st) {
    (void)hipGetLastError();
    const int B = uf_blocks(ns);
    hipLaunchKernelGGL(k_uf_sum, dim3(B), dim3(UFB), 0, st, f_dev);
    hipLaunchKernelGGL(k_uf_center, dim3(B), dim3(UFB), 0, st, f_dev);
    hipLaunchKernelGGL(k_uf_change, dim3(1), dim3(UFB), 0, st, f_dev, tol);
    return hipGetLastError();
}

hipError_t ulaunch_fourier_kappa(const UFourierDev* f_dev, int ns, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_uf_grad, dim3(uf_blocks(ns)), dim3(UFB), 0, st, f_dev);
    hipLaunchKernelGGL(k_uf_kappa, dim3(1), dim3(UF_THREADS), 0, st, f_dev);
    return hipGetLastError();
}

hipError_t ulaunch_pass(const UGeomDev* g_dev, int n_sys, int n_pos, int wpl, size_t lds_bytes, double inner_tol,
                        double inner_rtol, int max_inner, hipStream_t st) {
    (void)hipGetLastError();
    int blocks = (n_pos + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    hipLaunchKernelGGL(k_upack, dim3(blocks), dim3(256), 0, st, g_dev);
    switch (wpl) {
    case 1: hipLaunchKernelGGL(k_upass<1>, dim3(n_sys), dim3(WAVE), lds_bytes, st, g_dev, inner_tol, inner_rtol, max_inner); break;
    case 2: hipLaunchKernelGGL(k_upass<2>, dim3(n_sys), dim3(WAVE), lds_bytes, st, g_dev, inner_tol, inner_rtol, max_inner); break;
    case 4: hipLaunchKernelGGL(k_upass<4>, dim3(n_sys), dim3(WAVE), lds_bytes, st, g_dev, inner_tol, inner_rtol, max_inner); break;
    case 8: hipLaunchKernelGGL(k_upass<8>, dim3(n_sys), dim3(WAVE), lds_bytes, st, g_dev, inner_tol, inner_rtol, max_inner); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t ulaunch_reduce(const UGeomDev* g_dev, int ns, int nwalls, hipStream_t st) {
    (void)hipGetLastError();
    const int blocks = (ns + 63) / 64 + (nwalls + 63) / 64;
    hipLaunchKernelGGL(k_ureduce, dim3(blocks), dim3(64 * UQ), 0, st, g_dev);
    hipLaunchKernelGGL(k_ukappa, dim3(1), dim3(256), 0, st, g_dev);
    return hipGetLastError();
}
