// Host driver of the aMFP-BTE library: argument checking, face classes,
// material weights, workspace carving, the outer source iteration
// (Algorithm 1) replayed as HIP graphs, outputs, adjoint, checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/obte.h"
#include "obte_internal.h"

namespace {

thread_local std::string g_err;

obte_status fail(obte_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(OBTE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Cleanup calls whose failure must not abort the caller: report them when
// OBTE_DEBUG is set and clear HIP's per-thread last error so the next
// launch check sees only its own status.
void soft(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        if (getenv("OBTE_DEBUG")) fprintf(stderr, "obte: %s: %s\n", what, hipGetErrorString(e));
        (void)hipGetLastError();
    }
}

// kappa history capacity (passes); fixed so the workspace layout does not
// depend on max_outer and a checkpoint can be resumed with a larger cap.
constexpr int HIST_CAP = 1 << 16;

// checkpoint file tag (format: header of 9 ints, then the state arrays)
constexpr int CKPT_MAGIC = 0x4f425447;

}  // namespace

// A captured graph kept across calls while the launches it was captured from
// (the key: pointers, counts and parameters, as bytes) are unchanged.
struct GraphSlot {
    std::vector<unsigned char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void reset();
};

struct obte_mesh {
    // geometry
    int ndim = 2, nx = 1, ny = 1, nz = 1, nf = 4, ncells = 0, nsolid = 0, nwalls = 0;
    double L[3] = {0, 0, 0}, h[3] = {0, 0, 0}, dT = 1.0;
    int periodic[3] = {0, 0, 0};
    int grad_axis = 0;
    std::vector<uint16_t> fc;
    std::vector<int> wall_idx, wall_cell, wall_face;
    // material
    bool has_material = false;
    int n_mfp = 0, n_dir = 0, n_sys = 0;
    std::vector<double> mfp, dirs3, dir_w, kappa_m, alpha, Dw, S, wout, kappa_axis;
    // device tables (library-owned)
    int device = -1;
    uint16_t* d_fc = nullptr;
    std::vector<int> sidx, scell;   // solid index of each cell (-1 in pores), cell of each solid index
    int *d_sidx = nullptr, *d_scell = nullptr;
    int *d_wall_cell = nullptr, *d_wall_face = nullptr, *d_wall_idx = nullptr;
    double *d_mfp = nullptr, *d_dirs = nullptr, *d_D = nullptr, *d_S = nullptr, *d_wout = nullptr,
           *d_kax = nullptr;
    GeomDev* d_geom = nullptr;      // single-geometry view (apply, outputs)
    // results of the last solve
    bool solved = false, adj_ready = false;
    const void* last_ws = nullptr;
    const double* last_sigma = nullptr;
    double kappa = 0, kappa_face = 0, kappa_fourier = 0;
    std::vector<double> kappa_per_mfp;
    std::vector<long long> sys_iters, sys_sweeps;   // per system, summed over the passes
    GeomDev host_view{};
    int last_precision = 0, last_waves = 0, last_max_outer = 0, last_keep = 0;
    int last_waves_cls[4] = {0, 0, 0, 0}, last_dispatch = 0;
    // mode table (optional): per mode up to MODE_TERMS (system, weight) pairs
    // and its flux weight along the gradient axis; kappa_mu of the last solve
    int n_modes = 0;
    std::vector<int> mode_sys;
    std::vector<double> mode_w, mode_Sg, kappa_mode;
    int* d_mode_sys = nullptr;
    double *d_mode_w = nullptr, *d_mode_Sg = nullptr, *d_kmode = nullptr;
    bool modes_solved = false;
    // pinned host staging for the per-solve read-backs (grown on demand)
    char* h_stage = nullptr;
    size_t h_stage_bytes = 0;
    // graphs of the last single-mesh solve / adjoint, reused by the next call
    // with the same workspace, options and tables
    GraphSlot g_fourier, g_pass, g_adj;
};

void GraphSlot::reset() {
    if (exec) soft(hipGraphExecDestroy(exec), "hipGraphExecDestroy");
    if (graph) soft(hipGraphDestroy(graph), "hipGraphDestroy");
    exec = nullptr;
    graph = nullptr;
    key.clear();
}

template <typename... Ts>
std::vector<unsigned char> graph_key(const Ts&... parts) {
    std::vector<unsigned char> k;
    auto add = [&](const auto& v) {
        const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
        k.insert(k.end(), p, p + sizeof v);
    };
    (add(parts), ...);
    return k;
}

// The instantiated graph of `enqueue` captured on st: the slot's when its key
// matches (then the slot keeps ownership), else a new capture, which the slot
// takes over (or, without a slot, the caller destroys via *owned_graph).
template <class F>
obte_status slot_graph(GraphSlot* slot, const std::vector<unsigned char>& key, hipStream_t st, F enqueue,
                       hipGraphExec_t* exec_out, hipGraph_t* owned_graph) {
    *owned_graph = nullptr;
    if (slot && slot->exec && slot->key == key) {
        *exec_out = slot->exec;
        return OBTE_OK;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const obte_status s = enqueue();
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (s != OBTE_OK) {
        if (graph) soft(hipGraphDestroy(graph), "hipGraphDestroy");
        return s;
    }
    if (e != hipSuccess) return fail(OBTE_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        soft(hipGraphDestroy(graph), "hipGraphDestroy");
        return fail(OBTE_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e2));
    }
    if (slot) {
        slot->reset();
        slot->graph = graph;
        slot->exec = exec;
        slot->key = key;
    } else {
        *owned_graph = graph;
    }
    *exec_out = exec;
    return OBTE_OK;
}

namespace {

// ---------------------------------------------------------------------------
// workspace layout of one geometry
// ---------------------------------------------------------------------------
struct Layout {
    size_t sigma, sigma_f, sT, Tw, T_L, U, X, ksys, kfsys, iters, sweeps, hist, hist_face, ctrl, fx, fscal,
        Tstore, lam_psi, lam_phi, grad, bnd, wres, wres_hist, kry, ax, actl, ag,
        axp, afp, adX, adF, agram, apart, kraw, qrec, qoff, qsg, qalt, total;
};

// Linear interpolation weights of x on the sorted values v (clamped to the
// end nodes): up to two (index into v, weight) pairs.
int bracket_linear(const std::vector<double>& v, double x, int* idx, double* w) {
    const int n = (int)v.size();
    if (x <= v[0]) { idx[0] = 0; w[0] = 1.0; return 1; }
    if (x >= v[n - 1]) { idx[0] = n - 1; w[0] = 1.0; return 1; }
    int a = (int)(std::upper_bound(v.begin(), v.end(), x) - v.begin()) - 1;
    const double t = (x - v[a]) / (v[a + 1] - v[a]);
    idx[0] = a; w[0] = 1.0 - t;
    idx[1] = a + 1; w[1] = t;
    return 2;
}

// The same on sorted angles in [0, 2 pi), wrapping around.
int bracket_cyclic(const std::vector<double>& v, double x, int* idx, double* w) {
    const double two_pi = 2.0 * M_PI;
    const int n = (int)v.size();
    x = std::fmod(std::fmod(x, two_pi) + two_pi, two_pi);
    int b = (int)(std::upper_bound(v.begin(), v.end(), x) - v.begin());
    const int a = (b - 1 + n) % n;
    b %= n;
    const double gap = std::fmod(v[b] - v[a] + two_pi, two_pi);
    const double t = gap > 0.0 ? std::fmod(x - v[a] + two_pi, two_pi) / gap : 0.0;
    idx[0] = a; w[0] = 1.0 - t;
    idx[1] = b; w[1] = t;
    return 2;
}

constexpr int MODE_TERMS = 8;

// Spread every mode over the (MFP, direction) grid (see obte_material_desc).
obte_status mode_weights(obte_mesh* m, const obte_material_desc* d) {
    const int nd = m->ndim, nm = d->n_modes;
    std::vector<int> morder(m->n_mfp);
    for (int i = 0; i < m->n_mfp; ++i) morder[i] = i;
    std::sort(morder.begin(), morder.end(), [&](int a, int b) { return m->mfp[a] < m->mfp[b]; });
    std::vector<double> mv(m->n_mfp);
    for (int i = 0; i < m->n_mfp; ++i) mv[i] = m->mfp[morder[i]];
    for (int i = 1; i < m->n_mfp; ++i)
        if (!(mv[i] > mv[i - 1])) return fail(OBTE_ERR_ARG, "MFP nodes must be distinct for a mode table");
    auto angle = [](double y, double x) {
        const double a = std::atan2(y, x);
        return a < 0.0 ? a + 2.0 * M_PI : a;
    };
    // angular grid: 2D sorted azimuths; 3D distinct polar angles x azimuths
    std::vector<double> thv, phv;
    std::vector<int> lmap;            // (polar index, azimuth index) -> direction
    auto uniq = [](std::vector<double> v) {
        std::sort(v.begin(), v.end());
        std::vector<double> u;
        for (double x : v)
            if (u.empty() || x - u.back() > 1e-9) u.push_back(x);
        return u;
    };
    std::vector<double> th(m->n_dir), ph(m->n_dir);
    for (int l = 0; l < m->n_dir; ++l) {
        const double* s = &m->dirs3[l * 3];
        ph[l] = angle(s[1], s[0]);
        th[l] = std::acos(std::max(-1.0, std::min(1.0, s[2])));
    }
    phv = uniq(ph);
    if (nd == 2) {
        if ((int)phv.size() != m->n_dir) return fail(OBTE_ERR_ARG, "mode table: directions must have distinct angles");
        lmap.assign(m->n_dir, -1);
        for (int l = 0; l < m->n_dir; ++l)
            lmap[std::lower_bound(phv.begin(), phv.end(), ph[l] - 1e-9) - phv.begin()] = l;
    } else {
        thv = uniq(th);
        if (thv.size() * phv.size() != (size_t)m->n_dir)
            return fail(OBTE_ERR_ARG, "3D mode table needs a tensor (polar x azimuth) direction grid");
        lmap.assign(m->n_dir, -1);
        for (int l = 0; l < m->n_dir; ++l) {
            const int k = (int)(std::lower_bound(thv.begin(), thv.end(), th[l] - 1e-9) - thv.begin());
            const int j = (int)(std::lower_bound(phv.begin(), phv.end(), ph[l] - 1e-9) - phv.begin());
            if (lmap[k * phv.size() + j] >= 0) return fail(OBTE_ERR_ARG, "3D mode table: repeated direction");
            lmap[k * phv.size() + j] = l;
        }
    }
    // components per mode: ndim, or 3 in a 2D domain (the in-plane part is used)
    const int md = d->mode_dim > 0 ? d->mode_dim : nd;
    if (!(md == nd || (md == 3 && nd == 2)))
        return fail(OBTE_ERR_ARG, "mode_dim %d does not fit a %dD mesh", d->mode_dim, nd);
    m->n_modes = nm;
    m->mode_sys.assign((size_t)nm * MODE_TERMS, 0);
    m->mode_w.assign((size_t)nm * MODE_TERMS, 0.0);
    m->mode_Sg.assign(nm, 0.0);
    double asum = 0.0, net[3] = {0.0, 0.0, 0.0}, scale = 0.0;
    for (int mu = 0; mu < nm; ++mu) {
        const double a = d->mode_alpha[mu];
        if (!(a >= 0.0) || !std::isfinite(a)) return fail(OBTE_ERR_ARG, "mode_alpha[%d] must be >= 0", mu);
        double lam2 = 0.0;
        for (int ax = 0; ax < md; ++ax) {
            const double f = d->mode_F[mu * md + ax];
            if (!std::isfinite(f)) return fail(OBTE_ERR_ARG, "mode_F[%d] is not finite", mu);
            if (ax >= nd) continue;
            lam2 += f * f;
            net[ax] += a * f;
            scale += a * std::fabs(f);
        }
        // a mode that does not move in this domain keeps T_L: it drops out
        if (lam2 > 0.0) asum += a;
    }
    if (!(asum > 0.0)) return fail(OBTE_ERR_ARG, "no mode with a nonzero MFP and weight");
    for (int ax = 0; ax < nd; ++ax)
        if (std::fabs(net[ax]) > 1e-9 * scale) return fail(OBTE_ERR_ARG, "mode table carries a net flux along axis %d", ax);
    m->Dw.assign(m->n_sys, 0.0);
    m->S.assign(3 * m->n_sys, 0.0);
    m->kappa_axis.assign(3, 0.0);
    for (int mu = 0; mu < nm; ++mu) {
        const double* F = &d->mode_F[mu * md];
        const double a = d->mode_alpha[mu];
        double lam = 0.0;
        for (int ax = 0; ax < nd; ++ax) lam += F[ax] * F[ax];
        lam = std::sqrt(lam);
        if (lam == 0.0) continue;          // no grid weight, kappa_mu = 0
        int im[2], ip[2], it[2];
        double wm[2], wp[2], wt[2];
        const int nmm = bracket_linear(mv, lam, im, wm);
        const int npp = bracket_cyclic(phv, angle(F[1], F[0]), ip, wp);
        int ntt = 1;
        it[0] = 0; wt[0] = 1.0;
        if (nd == 3) ntt = bracket_linear(thv, std::acos(std::max(-1.0, std::min(1.0, F[2] / lam))), it, wt);
        int k = 0;
        for (int i = 0; i < nmm; ++i)
            for (int t = 0; t < ntt; ++t)
                for (int j = 0; j < npp; ++j) {
                    const int l = nd == 2 ? lmap[ip[j]] : lmap[it[t] * phv.size() + ip[j]];
                    const int sys = morder[im[i]] * m->n_dir + l;
                    const double c = wm[i] * wt[t] * wp[j];
                    m->mode_sys[(size_t)mu * MODE_TERMS + k] = sys;
                    m->mode_w[(size_t)mu * MODE_TERMS + k] = c;
                    ++k;
                    m->Dw[sys] += c * a / asum;
                    for (int ax = 0; ax < nd; ++ax) m->S[sys * 3 + ax] += c * a * F[ax];
                }
        m->mode_Sg[mu] = a * F[m->grad_axis];
        for (int ax = 0; ax < nd; ++ax) m->kappa_axis[ax] += a * F[ax] * F[ax];
    }
    // the T_L weights unnormalised (kept for reference; the kernels use D)
    m->alpha.assign(m->n_sys, 0.0);
    for (int sys = 0; sys < m->n_sys; ++sys) m->alpha[sys] = m->Dw[sys] * asum;
    return OBTE_OK;
}

// Systems per workgroup when the caller leaves it to the library: 4 in 2D;
// 1 in 3D, where the longest-MFP-first queue balances best with the finest
// grain (measured on the 64x64x16 membrane: 9.9 against 9.6 solves/s at 4).
int auto_waves(const obte_mesh* m) {
    int w = m->nz > 1 ? 1 : 4;
    if (m->n_mfp < w) w = m->n_mfp;
    return std::max(1, w);
}

int n_groups(const obte_mesh* m, int waves) { return (m->n_mfp + waves - 1) / waves; }

Layout make_layout(const obte_mesh* m, const obte_solve_opts* o, int waves) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t nc = (size_t)m->ncells, nw = (size_t)std::max(m->nwalls, 1);
    const size_t tsz = (o->precision == OBTE_FP32) ? 4 : 8;
    const size_t nwrap = (size_t)m->nx * m->nz;
    L.sigma = take(nc * 8);
    L.sigma_f = take(nc * 4);
    L.sT = take(2 * nc * 8);
    L.Tw = take(2 * nw * 8);
    L.T_L = take(nc * 8);
    L.ksys = take((size_t)m->n_sys * 8);
    L.kfsys = take((size_t)m->n_sys * 8);
    L.iters = take((size_t)m->n_sys * 8);
    L.sweeps = take((size_t)m->n_sys * 8);
    L.ctrl = take(CTRL_N * 4);
    L.fx = take(fourier_scratch_doubles(nc) * 8);
    L.fscal = take(8 * 8);
    L.lam_psi = take(2 * nc * 8);
    L.lam_phi = take(2 * nw * 8);
    L.grad = take(nc * 8);
    L.bnd = take(4 * (size_t)m->nf * nc * 8);
    L.wres = take((size_t)m->n_sys * 8);
    L.hist = take((size_t)HIST_CAP * 8);
    L.hist_face = take((size_t)HIST_CAP * 8);
    L.wres_hist = take((size_t)HIST_CAP * 8);
    const size_t naa = nc + (size_t)m->nwalls;
    L.ax = take((naa + 1) * 8);            // + the gauge shift of the pass
    L.actl = take(8 * 4);
    L.kraw = take((size_t)m->n_sys * 8);
    // the parts below depend on precision / keep_state / accel, so
    // the state a resumed solve reads (above, and U) keeps its place
    L.U = take(2 * (size_t)m->n_sys * nwrap * tsz);
    L.kry = m->nz > 1 ? take((size_t)m->n_sys * KRY3_VECS * nwrap * tsz) : 0;
    const size_t nsol = x_stride(m->nsolid);
    L.Tstore = o->keep_state ? take((size_t)m->n_sys * nsol * 8) : 0;
    L.X = take((size_t)m->n_sys * nsol * tsz);
    // 2D: the pass inputs in the four sweep orientations' order
    L.qrec = m->nz == 1 ? take(4 * nc * 4 * tsz) : take((1 + (size_t)m->nf) * nc * tsz);
    L.qoff = m->nz == 1 ? take(4 * nc * 4) : 0;
    L.qsg = m->nz == 1 ? take(4 * nc * tsz) : 0;
    L.qalt = m->nz == 1 ? take(4 * nc * 2 * tsz) : 0;
    // last: the mixing history (an adjoint may use another depth than the
    // forward solve whose stored state it reads)
    const size_t M = (size_t)std::max(o->accel, 0);
    L.ag = M ? take(naa * 8) : 0;
    L.axp = M ? take(naa * 8) : 0;
    L.afp = M ? take(naa * 8) : 0;
    L.adX = M ? take(M * naa * 8) : 0;
    L.adF = M ? take(M * naa * 8) : 0;
    L.agram = M ? take((M * M + M) * 8) : 0;
    L.apart = M ? take(aa_partial_doubles() * 8) : 0;
    L.total = off;
    return L;
}

GeomDev make_view(const obte_mesh* m, char* ws, const Layout& L, int waves, int accel) {
    GeomDev g{};
    g.n_aa = m->ncells + m->nwalls;
    g.aa_m = accel;
    g.nx = m->nx; g.ny = m->ny; g.nz = m->nz; g.ndim = m->ndim; g.nf = m->nf;
    g.ncells = m->ncells; g.nwalls = m->nwalls; g.nwrap = m->nx * m->nz; g.nsolid = m->nsolid;
    g.xs = (int)x_stride(m->nsolid);
    for (int a = 0; a < 3; ++a) { g.periodic[a] = m->periodic[a]; g.h[a] = m->h[a]; g.L[a] = m->L[a]; }
    g.grad_axis = m->grad_axis;
    g.dT = m->dT;
    g.n_mfp = m->n_mfp; g.n_dir = m->n_dir; g.n_sys = m->n_sys;
    g.n_perp = m->ncells / (m->grad_axis == 0 ? m->nx : (m->grad_axis == 1 ? m->ny : m->nz));
    g.fc = m->d_fc; g.sidx = m->d_sidx; g.scell = m->d_scell; g.wall_cell = m->d_wall_cell; g.wall_face = m->d_wall_face; g.wall_idx = m->d_wall_idx;
    g.mfp = m->d_mfp; g.dirs = m->d_dirs; g.Dw = m->d_D; g.S = m->d_S; g.wout = m->d_wout;
    g.gauge = m->n_modes > 0 ? 1 : 0;
    g.kappa_axis = m->d_kax;
    // kappa_face plane cells per sweep quadrant (2D): solid cells that are
    // last along the gradient axis in that quadrant's sweep order and whose
    // outflow face there is open
    if (m->nz == 1 && !m->fc.empty())
        for (int q = 0; q < 4; ++q) {
            const int negx = q & 1, negy = q >> 1, ga = m->grad_axis;
            const int fo = ga == 0 ? 1 - negx : 3 - negy;
            int cnt = 0;
            if (ga == 0) {
                const int ix = negx ? 0 : m->nx - 1;
                for (int iy = 0; iy < m->ny; ++iy) {
                    const uint16_t w = m->fc[(size_t)iy * m->nx + ix];
                    cnt += fc_solid(w) && fc_class(w, fo) != FC_WALL;
                }
            } else {
                const int iy = negy ? 0 : m->ny - 1;
                for (int ix = 0; ix < m->nx; ++ix) {
                    const uint16_t w = m->fc[(size_t)iy * m->nx + ix];
                    cnt += fc_solid(w) && fc_class(w, fo) != FC_WALL;
                }
            }
            g.qnk[q] = cnt;
        }
    if (ws) {
        g.sigma = (double*)(ws + L.sigma);
        g.sigma_f = (float*)(ws + L.sigma_f);
        g.sT = (double*)(ws + L.sT);
        g.Tw = (double*)(ws + L.Tw);
        g.T_L = (double*)(ws + L.T_L);
        g.U = ws + L.U;
        g.kry = L.kry ? ws + L.kry : nullptr;
        g.X = ws + L.X;
        g.ksys = (double*)(ws + L.ksys);
        g.kfsys = (double*)(ws + L.kfsys);
        g.iters = (long long*)(ws + L.iters);
        g.sweeps = (long long*)(ws + L.sweeps);
        g.hist = (double*)(ws + L.hist);
        g.hist_face = (double*)(ws + L.hist_face);
        g.ctrl = (int*)(ws + L.ctrl);
        g.fx = (double*)(ws + L.fx);
        g.fscal = (double*)(ws + L.fscal);
        g.Tstore = L.Tstore ? (double*)(ws + L.Tstore) : nullptr;
        g.lam_psi = (double*)(ws + L.lam_psi);
        g.lam_phi = (double*)(ws + L.lam_phi);
        g.gradient = (double*)(ws + L.grad);
        g.bnd = (double*)(ws + L.bnd);
        g.wres = (double*)(ws + L.wres);
        g.wres_hist = (double*)(ws + L.wres_hist);
        g.ax = (double*)(ws + L.ax);
        g.actl = (int*)(ws + L.actl);
        g.kraw = (double*)(ws + L.kraw);
        g.qrec = ws + L.qrec;
        if (m->nz == 1) {
            g.qoff = (uint32_t*)(ws + L.qoff);
            g.qsg = ws + L.qsg;
            g.qalt = ws + L.qalt;
        }
        if (accel > 0) {
            g.ag = (double*)(ws + L.ag);
            g.axp = (double*)(ws + L.axp);
            g.afp = (double*)(ws + L.afp);
            g.adX = (double*)(ws + L.adX);
            g.adF = (double*)(ws + L.adF);
            g.agram = (double*)(ws + L.agram);
            g.apart = (double*)(ws + L.apart);
        }
    }
    return g;
}

template <typename T>
obte_status upload(T** dst, const std::vector<T>& src) {
    if (*dst) { soft(hipFree(*dst), "hipFree(table)"); *dst = nullptr; }
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    HIPCHK(hipMalloc((void**)dst, bytes));
    if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return OBTE_OK;
}

void free_dev(obte_mesh* m) {
    m->g_fourier.reset();
    m->g_pass.reset();
    m->g_adj.reset();
    void* ptrs[] = {m->d_fc, m->d_sidx, m->d_scell, m->d_wall_cell, m->d_wall_face, m->d_wall_idx, m->d_mfp, m->d_dirs,
                    m->d_D, m->d_S, m->d_wout, m->d_kax, m->d_geom, m->d_mode_sys, m->d_mode_w,
                    m->d_mode_Sg, m->d_kmode};
    for (void* p : ptrs)
        if (p) soft(hipFree(p), "hipFree(table)");
    m->d_fc = nullptr; m->d_sidx = m->d_scell = nullptr; m->d_wall_cell = m->d_wall_face = m->d_wall_idx = nullptr;
    m->d_mfp = m->d_dirs = m->d_D = m->d_S = m->d_wout = m->d_kax = nullptr;
    m->d_geom = nullptr;
    m->d_mode_sys = nullptr;
    m->d_mode_w = m->d_mode_Sg = m->d_kmode = nullptr;
}

obte_status check_opts(const obte_solve_opts* o) {
    if (!o) return fail(OBTE_ERR_ARG, "opts is NULL");
    if (o->precision != OBTE_FP64 && o->precision != OBTE_FP32)
        return fail(OBTE_ERR_ARG, "precision must be OBTE_FP64 or OBTE_FP32");
    if (!(o->outer_tol >= 0.0) || o->max_outer < 1 || o->max_outer >= HIST_CAP)
        return fail(OBTE_ERR_ARG, "outer_tol must be >= 0 and 1 <= max_outer < %d", HIST_CAP);
    if (!(o->inner_tol > 0.0) || o->max_inner < 0)
        return fail(OBTE_ERR_ARG, "inner_tol must be > 0 and max_inner >= 0");
    if (o->waves_per_group < 0 || o->waves_per_group > 8)
        return fail(OBTE_ERR_ARG, "waves_per_group must be in 0..8");
    if (o->passes_per_graph < 0) return fail(OBTE_ERR_ARG, "passes_per_graph must be >= 0");
    if (!(o->fourier_tol > 0.0) || o->max_fourier < 0)
        return fail(OBTE_ERR_ARG, "fourier_tol must be > 0 and max_fourier >= 0");
    if (o->init != 0 && o->init != 1) return fail(OBTE_ERR_ARG, "init must be 0 or 1");
    if (o->lag_wrap != 0 && o->lag_wrap != 1) return fail(OBTE_ERR_ARG, "lag_wrap must be 0 or 1");
    if (!(o->wrap_tol >= 0.0)) return fail(OBTE_ERR_ARG, "wrap_tol must be >= 0");
    if (!(o->inner_rtol >= 0.0 && o->inner_rtol < 1.0)) return fail(OBTE_ERR_ARG, "inner_rtol must be in [0, 1)");
    if (o->stop_rule != 0 && o->stop_rule != 1) return fail(OBTE_ERR_ARG, "stop_rule must be 0 or 1");
    if (o->accel < 0 || o->accel > AA_MAX) return fail(OBTE_ERR_ARG, "accel must be in 0..%d", AA_MAX);
    for (int c = 0; c < 4; ++c)
        if (o->waves_by_class[c] < 0 || o->waves_by_class[c] > 8)
            return fail(OBTE_ERR_ARG, "waves_by_class[%d] must be in 0..8", c);
    if (o->dispatch < 0 || o->dispatch > 2) return fail(OBTE_ERR_ARG, "dispatch must be 0, 1 or 2");
    return OBTE_OK;
}

// ---------------------------------------------------------------------------
// live kernel timing with HIP events recorded on the caller's stream
// ---------------------------------------------------------------------------
struct Timer {
    bool on = false;
    std::vector<hipEvent_t> ev;     // pairs: (start, stop) for sweep, then reduce, per pass
    int K = 0;
    double sweep_ms = 0, reduce_ms = 0, fourier_ms = 0;
    int launches = 0;
    hipEvent_t f0 = nullptr, f1 = nullptr;
    obte_status init(int passes) {
        K = passes;
        ev.resize(4 * (size_t)K, nullptr);
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        HIPCHK(hipEventCreate(&f0));
        HIPCHK(hipEventCreate(&f1));
        on = true;
        return OBTE_OK;
    }
    // after the stream synchronised: accumulate the K passes just replayed
    obte_status collect(int passes_done) {
        for (int k = 0; k < passes_done && k < K; ++k) {
            float a = 0, b = 0;
            hipError_t e1 = hipEventElapsedTime(&a, ev[4 * k], ev[4 * k + 1]);
            hipError_t e2 = hipEventElapsedTime(&b, ev[4 * k + 2], ev[4 * k + 3]);
            if (e1 != hipSuccess || e2 != hipSuccess) {
                soft(e1 != hipSuccess ? e1 : e2, "hipEventElapsedTime");
                continue;
            }
            sweep_ms += a;
            reduce_ms += b;
            ++launches;
        }
        return OBTE_OK;
    }
    ~Timer() {
        for (auto e : ev)
            if (e) soft(hipEventDestroy(e), "hipEventDestroy");
        if (f0) soft(hipEventDestroy(f0), "hipEventDestroy");
        if (f1) soft(hipEventDestroy(f1), "hipEventDestroy");
    }
};

// ---------------------------------------------------------------------------
// the outer loop shared by obte_solve, obte_solve_batch and obte_adjoint
// ---------------------------------------------------------------------------
struct Run {
    std::vector<obte_mesh*> meshes;
    std::vector<GeomDev> views;
    std::vector<Item> items;
    // device copies of the views and the item list, and the pending count,
    // in the caller's workspace after the geometries (no allocation per call)
    GeomDev* d_views = nullptr;
    Item* d_items = nullptr;
    int* d_pending = nullptr;     // geometries whose Fourier CG still iterates
    size_t state_off = 0, state_bytes = 0;
    // items grouped by cells per lane (ceil(nx / 64)): one launch per class,
    // so a narrow geometry of a batch does not run the widest row's kernel
    int cls_first[5] = {}, cls_count[5] = {};
    size_t cls_lds[5] = {};
    int cls_waves[5] = {4, 4, 4, 4, 4};   // systems per workgroup of each launch class
    int cls_full[5] = {1, 1, 1, 1, 1};    // class whose every row is exactly 64 * class cells
    int nzmax = 1, precision = 0, accel = 0;
    // 2D with dispatch = 2: every item in one persistent launch of queue_waves
    // waves per group, the groups taking items from the device counter d_queue
    int queue = 0, queue_waves = 1;
    int* d_queue = nullptr;
    int gauge = 0;                // some geometry has a mode table (re-centred passes)
    int max_cells = 0, max_walls = 0, max_solid = 0;
    // pinned host slots for the loop read-backs (two per loop, see
    // speculative loops below); null: plain synchronous read-backs
    int* h_pin = nullptr;
    // the views in pinned memory (staged upload), or null
    const GeomDev* h_views = nullptr;
};

// Pinned staging of a mesh: bytes [0, STAGE_LOOP) hold the loop read-back
// slots, the rest the per-solve result read-backs.  Grown only while no copy
// into it is in flight (at a solve's start, or after a stream synchronize).
constexpr size_t STAGE_LOOP = 256;
static_assert((4 + 2 * CTRL_N) * sizeof(int) <= STAGE_LOOP, "loop read-back slots exceed the staging head");
obte_status ensure_stage(obte_mesh* m, size_t need) {
    if (m->h_stage_bytes >= need) return OBTE_OK;
    if (m->h_stage) soft(hipHostFree(m->h_stage), "hipHostFree(stage)");
    m->h_stage = nullptr;
    m->h_stage_bytes = 0;
    HIPCHK(hipHostMalloc((void**)&m->h_stage, need, hipHostMallocDefault));
    m->h_stage_bytes = need;
    return OBTE_OK;
}

// Two events for a speculative loop, destroyed with it.
struct EventPair {
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t create() {
        hipError_t e = hipEventCreateWithFlags(&ev[0], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[1], hipEventDisableTiming);
        return e;
    }
    ~EventPair() {
        for (hipEvent_t x : ev)
            if (x) soft(hipEventDestroy(x), "hipEventDestroy");
    }
};

size_t run_state_bytes(size_t n_views, size_t n_items) {
    return align256(n_views * sizeof(GeomDev)) + align256(n_items * sizeof(Item)) + 256;
}

// Systems per workgroup of each cells-per-lane launch class (Wc[c], c = 1..4
// = ceil(nx / 64)) over these meshes; the same rule for the workspace size
// and the solve.  A class takes opts.waves_by_class[c - 1], else
// waves_per_group, else the automatic choice; in 3D every wave of a group
// needs nz rows of LDS, which bounds the class's W.
obte_status resolve_waves(const obte_mesh* const* meshes, int n, const obte_solve_opts* o, int* Wc) {
    int base = o->waves_per_group;
    if (base == 0) {
        base = auto_waves(meshes[0]);
        for (int i = 1; i < n; ++i)
            if (auto_waves(meshes[i]) != base)
                return fail(OBTE_ERR_ARG, "meshes differ in their automatic waves_per_group; set it explicitly");
    }
    int nzm = 1;
    bool present[5] = {false, false, false, false, false};
    for (int i = 0; i < n; ++i) {
        nzm = std::max(nzm, meshes[i]->nz);
        present[(meshes[i]->nx + 63) / 64] = true;
    }
    const size_t cap = 64 * 1024, tsz = o->precision == OBTE_FP32 ? 4 : 8;
    for (int c = 1; c <= 4; ++c) {
        const int set = o->waves_by_class[c - 1];
        int W = set ? set : base;
        // 3D: one row per z-plane in the compute type (2D keeps its rows in
        // registers and needs no LDS)
        const size_t per_wave = nzm > 1 ? (size_t)nzm * 64 * c * tsz : 0;
        if (present[c] && per_wave > cap)
            return fail(OBTE_ERR_ARG, "a wave needs %zu bytes of LDS (nx, nz too large; limit %zu)", per_wave, cap);
        // 2D FP64 rows of 3 or 4 cells per lane (and the FP64 persistent
        // launch, which holds every class body) run at most 4 waves per
        // group: the kernels' register budget
        if (present[c] && nzm == 1 && o->precision == OBTE_FP64 && (c >= 3 || o->dispatch == 2) && W > 4) {
            if (set || o->waves_per_group)
                return fail(OBTE_ERR_ARG, "FP64 sweeps of %d cells per lane take at most 4 systems per workgroup", c);
            W = 4;
        }
        const int wmax = per_wave > 0 ? (int)(cap / per_wave) : 8;
        if (present[c] && W > wmax) {
            if (set || o->waves_per_group)
                return fail(OBTE_ERR_ARG, "%d systems per workgroup need more than 64 KiB of LDS (max %d)", W, wmax);
            W = wmax;
        }
        Wc[c] = std::max(1, W);
    }
    Wc[0] = Wc[1];
    return OBTE_OK;
}

obte_status build_run(Run& R, obte_mesh* const* meshes, int n, const obte_solve_opts* o,
                      char* ws, std::vector<size_t>* offsets) {
    R.meshes.assign(meshes, meshes + n);
    R.precision = o->precision;
    R.accel = o->accel;
    for (int i = 0; i < n; ++i) R.gauge |= meshes[i]->n_modes > 0 ? 1 : 0;
    int Wc[5];
    obte_status s = resolve_waves(meshes, n, o, Wc);
    if (s != OBTE_OK) return s;
    for (int c = 0; c < 5; ++c) R.cls_waves[c] = Wc[c];
    size_t off = 0;
    std::vector<Item> by_cls[5];
    for (int gi = 0; gi < n; ++gi) {
        obte_mesh* m = meshes[gi];
        const int c = (m->nx + 63) / 64;
        const int W = Wc[c];
        if (m->nx != 64 * c) R.cls_full[c] = 0;
        Layout L = make_layout(m, o, W);
        if (offsets) offsets->push_back(off);
        GeomDev v = make_view(m, ws + off, L, W, o->accel);
        const int ng = n_groups(m, W);
        // longest MFPs first: their systems take the most wrap iterations, so
        // the shorter ones dispatched after them fill in behind (a shorter
        // makespan than direction-major order; the results do not depend on it)
        for (int gp = ng - 1; gp >= 0; --gp)
            for (int l = 0; l < m->n_dir; ++l) {
                Item it;
                it.geom = gi;
                it.l = l;
                it.m0 = gp * W;
                it.nm = std::min(W, m->n_mfp - gp * W);
                by_cls[c].push_back(it);
            }
        R.views.push_back(v);
        R.nzmax = std::max(R.nzmax, m->nz);
        R.max_cells = std::max(R.max_cells, m->ncells);
        R.max_solid = std::max(R.max_solid, m->nsolid);
        R.max_walls = std::max(R.max_walls, m->nwalls);
        off += align256(L.total);
    }
    for (int gi = 0; gi < n; ++gi)
        if ((meshes[gi]->nz > 1) != (R.nzmax > 1))
            return fail(OBTE_ERR_ARG, "a batch cannot mix 2D and 3D meshes");
    const size_t tsz = o->precision == OBTE_FP32 ? 4 : 8;
    R.queue = o->dispatch == 2 && R.nzmax == 1;
    if (R.queue) {
        // one list over every class, longest-MFP groups of every geometry
        // first; a group has as many waves as the widest class needs
        std::vector<Item> all;
        for (int c = 1; c <= 4; ++c) {
            all.insert(all.end(), by_cls[c].begin(), by_cls[c].end());
            if (!by_cls[c].empty()) R.queue_waves = std::max(R.queue_waves, Wc[c]);
            by_cls[c].clear();
        }
        std::stable_sort(all.begin(), all.end(), [](const Item& a, const Item& b) { return a.m0 > b.m0; });
        by_cls[0] = std::move(all);
        R.cls_first[0] = 0;
        R.cls_count[0] = (int)by_cls[0].size();
        R.items = by_cls[0];
    }
    for (int c = 1; c <= 4; ++c) {
        // dispatch = 1 (and 2 in 3D): the longest-MFP groups of every geometry
        // first (the order is stable, so geometries and directions keep theirs)
        if (o->dispatch == 1 || (o->dispatch == 2 && !R.queue))
            std::stable_sort(by_cls[c].begin(), by_cls[c].end(),
                             [](const Item& a, const Item& b) { return a.m0 > b.m0; });
        R.cls_first[c] = (int)R.items.size();
        R.cls_count[c] = (int)by_cls[c].size();
        R.items.insert(R.items.end(), by_cls[c].begin(), by_cls[c].end());
        R.cls_lds[c] = R.nzmax > 1 ? (size_t)Wc[c] * R.nzmax * 64 * c * tsz : 0;
    }
    R.state_off = off;
    R.state_bytes = run_state_bytes(R.views.size(), R.items.size());
    return OBTE_OK;
}

// Place the run's device state in the workspace (after the size check).
// With a staging mesh (its pinned buffer) and a stream, the views and items
// go through pinned memory with copies queued on the stream (the host does
// not wait for them); else plain synchronous copies (obte_solve_noalloc).
obte_status upload_run(Run& R, char* ws, hipStream_t st = nullptr, obte_mesh* stage = nullptr) {
    char* p = ws + R.state_off;
    R.d_views = (GeomDev*)p;
    p += align256(R.views.size() * sizeof(GeomDev));
    R.d_items = (Item*)p;
    p += align256(R.items.size() * sizeof(Item));
    R.d_pending = (int*)p;
    R.d_queue = R.d_pending + 16;       // within the state's last 256 bytes
    const size_t vb = R.views.size() * sizeof(GeomDev), ib = R.items.size() * sizeof(Item);
    if (st && stage) {
        obte_status s = ensure_stage(stage, STAGE_LOOP + align256(vb) + ib);
        if (s != OBTE_OK) return s;
        char* h = stage->h_stage + STAGE_LOOP;
        std::memcpy(h, R.views.data(), vb);
        std::memcpy(h + align256(vb), R.items.data(), ib);
        HIPCHK(hipMemcpyAsync(R.d_views, h, vb, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(R.d_items, h + align256(vb), ib, hipMemcpyHostToDevice, st));
        R.h_views = reinterpret_cast<const GeomDev*>(h);
        return OBTE_OK;
    }
    HIPCHK(hipMemcpy(R.d_views, R.views.data(), vb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(R.d_items, R.items.data(), ib, hipMemcpyHostToDevice));
    return OBTE_OK;
}

// The pass kernel over every item, one launch per cells-per-lane class.
// (start: an event recorded after the 2D input packing, so that it and the
// end event bracket the pass kernels alone)
obte_status launch_sweeps(const Run& R, const PassParams& pp, hipStream_t st, hipEvent_t start = nullptr) {
    if (R.nzmax == 1)
        HIPCHK(launch_pack_rows(R.precision, R.d_views, (int)R.views.size(), R.max_cells, pp, st,
                                R.queue ? R.d_queue : nullptr));
    else
        HIPCHK(launch_pack3(R.precision, R.d_views, (int)R.views.size(), R.max_cells, pp, st));
    if (start) HIPCHK(hipEventRecord(start, st));
    if (R.queue) {
        HIPCHK(launch_sweep_queue(R.precision, R.d_views, R.d_items, R.cls_count[0], R.queue_waves, pp, st,
                                  R.d_queue));
        return OBTE_OK;
    }
    for (int c = 1; c <= 4; ++c)
        if (R.cls_count[c] > 0)
            HIPCHK(launch_sweep_pass(R.precision, c, R.nzmax, R.d_views, R.d_items + R.cls_first[c],
                                     R.cls_count[c], R.cls_waves[c], pp, R.cls_lds[c], st, R.cls_full[c]));
    return OBTE_OK;
}

obte_status enqueue_pass(const Run& R, const PassParams& pp, hipStream_t st, Timer* tm, int k) {
    obte_status s = launch_sweeps(R, pp, st, (tm && tm->on) ? tm->ev[4 * k] : nullptr);
    if (s != OBTE_OK) return s;
    if (tm && tm->on) HIPCHK(hipEventRecord(tm->ev[4 * k + 1], st));
    if (tm && tm->on) HIPCHK(hipEventRecord(tm->ev[4 * k + 2], st));
    HIPCHK(launch_reduce_pass(R.precision, R.d_views, (int)R.views.size(), R.max_solid, pp, st));
    if (R.gauge && !pp.adjoint) HIPCHK(launch_gauge(R.d_views, (int)R.views.size(), R.max_cells + R.max_walls, st));
    if (R.accel > 0) HIPCHK(launch_anderson(R.d_views, (int)R.views.size(), R.max_cells + R.max_walls, pp, st));
    HIPCHK(launch_finalize(R.d_views, (int)R.views.size(), pp, st));
    if (tm && tm->on) HIPCHK(hipEventRecord(tm->ev[4 * k + 3], st));
    return OBTE_OK;
}

// Fourier first guess of every geometry: CG iterations replayed as HIP graphs
// of KF iterations (with the count of geometries still iterating at the end)
// until none is left; direct launches when there is no stream to capture.
obte_status run_fourier(const Run& R, const obte_solve_opts* o, hipStream_t st, GraphSlot* slot,
                        bool use_graph = true) {
    const int n = (int)R.views.size();
    constexpr int KF = 8;     // even: an iteration's parity is its position in the graph
    HIPCHK(launch_fourier_init(R.d_views, n, R.max_cells, st));
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int j = 0; j < KF && e == hipSuccess; ++j)
            e = launch_fourier_iter(R.d_views, n, R.max_cells, j & 1, o->fourier_tol, o->max_fourier, st);
        if (e == hipSuccess) e = launch_fourier_pending(R.d_views, n, R.d_pending, st);
        return e;
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (st && use_graph) {
        const auto key = graph_key(R.d_views, R.d_pending, n, R.max_cells, o->fourier_tol, o->max_fourier, KF);
        obte_status s = slot_graph(slot, key, st, [&]() -> obte_status {
            const hipError_t e = enqueue();
            return e == hipSuccess ? OBTE_OK : fail(OBTE_ERR_HIP, "Fourier graph capture: %s", hipGetErrorString(e));
        }, &exec, &graph);
        if (s != OBTE_OK) return s;
    }
    obte_status out = OBTE_OK;
    EventPair evp;
    if (exec && R.h_pin) {
        // speculative: the next graph is queued before the previous one's
        // count is read, so the GPU does not idle on the host round trip; a
        // graph queued after convergence runs as early exits
        hipError_t e = evp.create();
        int* slot2[2] = {R.h_pin, R.h_pin + 1};
        auto launch = [&](int b) -> hipError_t {
            hipError_t e2 = hipGraphLaunch(exec, st);
            if (e2 == hipSuccess) e2 = hipMemcpyAsync(slot2[b], R.d_pending, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e2 == hipSuccess) e2 = hipEventRecord(evp.ev[b], st);
            return e2;
        };
        int it = KF, cur = 0;
        if (e == hipSuccess) e = launch(cur);
        while (e == hipSuccess) {
            const bool more = it <= o->max_fourier + KF;
            if (more) {
                e = launch(cur ^ 1);
                it += KF;
                if (e != hipSuccess) break;
            }
            e = hipEventSynchronize(evp.ev[cur]);
            if (e != hipSuccess || *slot2[cur] == 0 || !more) break;
            cur ^= 1;
        }
        if (e != hipSuccess) out = fail(OBTE_ERR_HIP, "Fourier iterations: %s", hipGetErrorString(e));
    } else {
        int pending = 1;
        for (int it = 0; pending > 0 && it <= o->max_fourier + KF; it += KF) {
            const hipError_t e = exec ? hipGraphLaunch(exec, st) : enqueue();
            if (e != hipSuccess) { out = fail(OBTE_ERR_HIP, "Fourier iterations: %s", hipGetErrorString(e)); break; }
            hipError_t e2 = hipMemcpyAsync(&pending, R.d_pending, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
            if (e2 != hipSuccess) { out = fail(OBTE_ERR_HIP, "Fourier readback: %s", hipGetErrorString(e2)); break; }
        }
    }
    if (graph) {      // not kept by a slot: a queued graph ends first
        soft(hipStreamSynchronize(st), "hipStreamSynchronize");
        soft(hipGraphExecDestroy(exec), "hipGraphExecDestroy");
        soft(hipGraphDestroy(graph), "hipGraphDestroy");
    }
    if (out != OBTE_OK) return out;
    HIPCHK(launch_fourier_finish(R.d_views, n, R.max_cells, st));
    return OBTE_OK;
}

// Replays graphs of K passes until every geometry reports done.
obte_status outer_loop(const Run& R, const PassParams& pp, int K, hipStream_t st, int max_outer,
                       Timer* tm, GraphSlot* slot) {
    const int n = (int)R.views.size();
    std::vector<int> ctrl(CTRL_N);
    if (tm && tm->on && tm->K < K) return fail(OBTE_ERR_STATE, "timer sized for fewer passes");
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    if (K > 1) {
        const auto key = graph_key(R.d_views, R.d_items, (int)R.views.size(), R.cls_first, R.cls_count, R.cls_lds,
                                   R.cls_waves, R.precision, R.nzmax, R.max_cells, R.max_walls, R.gauge, R.accel,
                                   R.queue, R.queue_waves, pp, K, tm && tm->on);
        obte_status s = slot_graph(slot, key, st, [&]() -> obte_status {
            obte_status sk = OBTE_OK;
            for (int k = 0; k < K && sk == OBTE_OK; ++k) sk = enqueue_pass(R, pp, st, tm, k);
            return sk;
        }, &exec, &graph);
        if (s != OBTE_OK) return s;
    }
    obte_status out = OBTE_OK;
    int launched = 0;
    if (exec && n == 1 && !(tm && tm->on) && R.h_pin) {
        // speculative, as the Fourier loop: one graph of K passes queued
        // ahead; passes after convergence exit at once (the done flag)
        EventPair evp;
        hipError_t e = evp.create();
        int* slot2[2] = {R.h_pin + 4, R.h_pin + 4 + CTRL_N};
        auto launch = [&](int b) -> hipError_t {
            hipError_t e2 = hipGraphLaunch(exec, st);
            if (e2 == hipSuccess)
                e2 = hipMemcpyAsync(slot2[b], R.views[0].ctrl, CTRL_N * sizeof(int), hipMemcpyDeviceToHost, st);
            if (e2 == hipSuccess) e2 = hipEventRecord(evp.ev[b], st);
            return e2;
        };
        int cur = 0;
        if (e == hipSuccess) e = launch(cur);
        launched = K;
        bool done = false;
        while (e == hipSuccess) {
            const bool more = launched <= max_outer + K;
            if (more) {
                e = launch(cur ^ 1);
                launched += K;
                if (e != hipSuccess) break;
            }
            e = hipEventSynchronize(evp.ev[cur]);
            if (e != hipSuccess) break;
            done = slot2[cur][CTRL_DONE] != 0;
            if (done || !more) break;
            cur ^= 1;
        }
        if (e != hipSuccess) out = fail(OBTE_ERR_HIP, "graph launch / readback: %s", hipGetErrorString(e));
        else if (!done) out = fail(OBTE_ERR_STATE, "outer loop did not terminate");
        if (graph) {      // not kept by a slot: the queued graph ends first
            soft(hipStreamSynchronize(st), "hipStreamSynchronize");
            soft(hipGraphExecDestroy(exec), "hipGraphExecDestroy");
            soft(hipGraphDestroy(graph), "hipGraphDestroy");
        }
        return out;
    }
    while (true) {
        if (exec) {
            hipError_t e = hipGraphLaunch(exec, st);
            if (e != hipSuccess) { out = fail(OBTE_ERR_HIP, "graph launch: %s", hipGetErrorString(e)); break; }
            launched += K;
        } else {
            out = enqueue_pass(R, pp, st, tm, 0);
            if (out != OBTE_OK) break;
            launched += 1;
        }
        bool all_done = true;
        for (int i = 0; i < n && all_done; ++i) {
            hipError_t e = hipMemcpyAsync(ctrl.data(), R.views[i].ctrl, CTRL_N * sizeof(int),
                                          hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) { out = fail(OBTE_ERR_HIP, "readback: %s", hipGetErrorString(e)); all_done = true; break; }
            if (!ctrl[CTRL_DONE]) all_done = false;
        }
        if (tm && tm->on && out == OBTE_OK) tm->collect(exec ? K : 1);
        if (out != OBTE_OK || all_done) break;
        if (launched > max_outer + K + 2) { out = fail(OBTE_ERR_STATE, "outer loop did not terminate"); break; }
    }
    if (graph) {      // not kept by a slot
        soft(hipGraphExecDestroy(exec), "hipGraphExecDestroy");
        soft(hipGraphDestroy(graph), "hipGraphDestroy");
    }
    return out;
}

PassParams base_params(const obte_solve_opts* o) {
    PassParams pp{};
    pp.inner_tol = o->inner_tol;
    pp.max_inner = o->max_inner;
    pp.mode = 0;
    pp.max_outer = o->max_outer;
    pp.outer_tol = o->outer_tol;
    pp.lag_wrap = o->lag_wrap;
    pp.inner_rtol = o->inner_rtol;
    pp.wrap_tol = o->wrap_tol > 0.0 ? o->wrap_tol : std::max(o->inner_tol, 0.2 * o->outer_tol);
    pp.stop_rule = o->stop_rule;
    return pp;
}

// noalloc: no graph capture, no pinned staging, no events (the entry point
// for callers that cannot allocate); every launch goes directly on `stream`.
obte_status solve_impl(obte_mesh* const* meshes, int n, const obte_solve_opts* o,
                       const double* const* sigma, void* workspace, size_t ws_bytes, void* stream,
                       double* T_L_out, double* J_out, double* kappa_out, obte_stats* stats,
                       bool keep_T, bool noalloc = false) {
    obte_status s = check_opts(o);
    if (s != OBTE_OK) return s;
    if (!meshes || n < 1) return fail(OBTE_ERR_ARG, "no meshes");
    if (!workspace) return fail(OBTE_ERR_ARG, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(OBTE_ERR_ARG, "workspace must be 256-byte aligned");
    for (int i = 0; i < n; ++i) {
        if (!meshes[i]) return fail(OBTE_ERR_ARG, "mesh %d is NULL", i);
        if (!meshes[i]->has_material) return fail(OBTE_ERR_STATE, "mesh %d has no material", i);
    }
    hipStream_t st = (hipStream_t)stream;
    Run R;
    std::vector<size_t> offs;
    s = build_run(R, meshes, n, o, (char*)workspace, &offs);
    if (s != OBTE_OK) return s;
    {
        const size_t need = R.state_off + R.state_bytes;
        if (ws_bytes < need)
            return fail(OBTE_ERR_NOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, need);
        if ((s = upload_run(R, (char*)workspace, st, noalloc ? nullptr : meshes[0])) != OBTE_OK) return s;
        if (!noalloc) {
            if ((s = ensure_stage(meshes[0], STAGE_LOOP)) != OBTE_OK) return s;
            R.h_pin = (int*)meshes[0]->h_stage;
        }
    }
    for (int i = 0; i < n; ++i) {
        obte_mesh* m = meshes[i];
        Layout L = make_layout(m, o, R.cls_waves[1]);
        char* ws = (char*)workspace + offs[i];
        if (R.h_views)
            HIPCHK(hipMemcpyAsync(m->d_geom, R.h_views + i, sizeof(GeomDev), hipMemcpyHostToDevice, st));
        else
            HIPCHK(hipMemcpy(m->d_geom, &R.views[i], sizeof(GeomDev), hipMemcpyHostToDevice));
        m->host_view = R.views[i];
        HIPCHK(launch_prep_sigma(m->d_geom, m->ncells, sigma ? sigma[i] : nullptr, st));
        if (o->init == 0) {
            const size_t tsz = o->precision == OBTE_FP32 ? 4 : 8;
            HIPCHK(hipMemsetAsync(ws + L.U, 0, 2 * (size_t)m->n_sys * m->nx * m->nz * tsz, st));
        }
        HIPCHK(hipMemsetAsync(ws + L.iters, 0, 2 * (size_t)m->n_sys * 8, st));
        HIPCHK(hipMemsetAsync(ws + L.wres, 0, (size_t)m->n_sys * 8, st));
    }
    Timer tm;
    // events recorded inside a captured graph cannot be timed: timing runs
    // launch the pass kernels directly
    const int K = (o->passes_per_graph <= 1 || !st || o->timing || noalloc) ? 1 : o->passes_per_graph;
    if (o->timing) {
        s = tm.init(K);
        if (s != OBTE_OK) return s;
    }
    if (o->init == 0) {
        if (tm.on) HIPCHK(hipEventRecord(tm.f0, st));
        s = run_fourier(R, o, st, n == 1 ? &meshes[0]->g_fourier : nullptr, !noalloc);
        if (s != OBTE_OK) return s;
        if (tm.on) HIPCHK(hipEventRecord(tm.f1, st));
    } else {
        // resume: clear the done / converged flags, keep the pass count; the
        // mixing history restarts from the stored iterate
        for (int i = 0; i < n; ++i) {
            int zero2[2] = {0, 0};
            HIPCHK(hipMemcpyAsync(R.views[i].ctrl + CTRL_DONE, zero2, sizeof(int), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(R.views[i].ctrl + CTRL_CONVERGED, zero2, sizeof(int), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemsetAsync(R.views[i].actl, 0, 8 * sizeof(int), st));
        }
    }
    if (!o->only_fourier) {
        PassParams pp = base_params(o);
        pp.sigma1 = 1;
        for (int i = 0; i < n; ++i)
            if (sigma && sigma[i]) pp.sigma1 = 0;
        s = outer_loop(R, pp, K, st, o->max_outer, &tm, n == 1 ? &meshes[0]->g_pass : nullptr);
        if (s != OBTE_OK) return s;
        // energy balance of the last pass, from its stored solutions
        for (int i = 0; i < n; ++i)
            HIPCHK(launch_energy(meshes[i]->d_geom, R.precision, meshes[i]->nsolid, st));
        // replay the last pass's final sweep for the flux map / stored state
        if ((J_out || keep_T) && n == 1) {
            PassParams rp = pp;
            rp.mode = 1;
            rp.store_T = keep_T ? 1 : 0;
            s = launch_sweeps(R, rp, st);
            if (s != OBTE_OK) return s;
        }
    }
    if (n == 1 && (T_L_out || J_out)) HIPCHK(launch_output(meshes[0]->d_geom, R.precision, meshes[0]->ncells, T_L_out, o->only_fourier ? nullptr : J_out, nullptr, st));
    if (n == 1 && J_out && o->only_fourier) HIPCHK(hipMemsetAsync(J_out, 0, sizeof(double) * meshes[0]->ncells * meshes[0]->ndim, st));
    // results
    obte_status ret = OBTE_OK;
    for (int i = 0; i < n; ++i) {
        obte_mesh* m = meshes[i];
        const GeomDev& v = R.views[i];
        std::vector<int> ctrl(CTRL_N);
        double fs[5];
        HIPCHK(hipMemcpyAsync(ctrl.data(), v.ctrl, CTRL_N * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(fs, v.fscal, sizeof fs, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const int passes = o->only_fourier ? 0 : ctrl[CTRL_PASS];
        std::vector<double> hist(passes + 1, 0.0), histf(passes + 1, 0.0), ks(m->n_sys), kfs(m->n_sys),
            wrh(passes + 1, 0.0);
        std::vector<long long> its(m->n_sys), sws(m->n_sys);
        if (passes > 0 && noalloc) {
            // plain copies into the host vectors (no pinned staging)
            const size_t hb = (size_t)passes * sizeof(double), sb = (size_t)m->n_sys * 8;
            HIPCHK(hipMemcpy(hist.data(), v.hist, hb, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(histf.data(), v.hist_face, hb, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(wrh.data(), v.wres_hist, hb, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(ks.data(), v.ksys, sb, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(its.data(), v.iters, sb, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(sws.data(), v.sweeps, sb, hipMemcpyDeviceToHost));
        } else if (passes > 0) {
            // one wait for the six read-backs: asynchronous copies into pinned memory
            const size_t hb = (size_t)passes * sizeof(double), sb = (size_t)m->n_sys * 8;
            obte_status se = ensure_stage(m, STAGE_LOOP + 3 * hb + 3 * sb);
            if (se != OBTE_OK) return se;
            char* hs = m->h_stage + STAGE_LOOP;
            const void* src[6] = {v.hist, v.hist_face, v.wres_hist, v.ksys, v.iters, v.sweeps};
            void* dst[6] = {hist.data(), histf.data(), wrh.data(), ks.data(), its.data(), sws.data()};
            const size_t len[6] = {hb, hb, hb, sb, sb, sb};
            size_t off = 0;
            for (int k = 0; k < 6; ++k) {
                HIPCHK(hipMemcpyAsync(hs + off, src[k], len[k], hipMemcpyDeviceToHost, st));
                off += len[k];
            }
            HIPCHK(hipStreamSynchronize(st));
            off = 0;
            for (int k = 0; k < 6; ++k) {
                std::memcpy(dst[k], hs + off, len[k]);
                off += len[k];
            }
        }
        m->kappa_fourier = fs[0];
        m->kappa = passes > 0 ? hist[passes - 1] : fs[0];
        m->kappa_face = passes > 0 ? histf[passes - 1] : fs[0];
        m->kappa_per_mfp.assign(m->n_mfp, 0.0);
        for (int sys = 0; sys < m->n_sys; ++sys) m->kappa_per_mfp[sys / m->n_dir] += ks[sys];
        m->sys_iters = its;
        m->sys_sweeps = sws;
        m->modes_solved = false;
        if (m->n_modes > 0 && passes > 0) {
            // mode-resolved kappa: gather of the per-system sums (kernel)
            const double pref = m->L[m->grad_axis] / (m->dT * (double)m->ncells);
            HIPCHK(launch_kappa_modes(m->d_mode_sys, m->d_mode_w, m->d_mode_Sg, m->n_modes, MODE_TERMS,
                                      m->d_D, m->n_sys, v.kraw, pref, m->d_kmode, st));
            m->kappa_mode.assign(m->n_modes, 0.0);
            HIPCHK(hipMemcpyAsync(m->kappa_mode.data(), m->d_kmode, (size_t)m->n_modes * sizeof(double),
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            m->modes_solved = true;
        }
        m->solved = true;
        m->adj_ready = keep_T && !o->only_fourier && ctrl[CTRL_CONVERGED];
        m->last_ws = workspace;
        m->last_sigma = sigma ? sigma[i] : nullptr;
        m->last_precision = o->precision;
        m->last_waves = R.cls_waves[(m->nx + 63) / 64];
        for (int c = 0; c < 4; ++c) m->last_waves_cls[c] = R.cls_waves[c + 1];
        m->last_dispatch = o->dispatch;
        m->last_max_outer = o->max_outer;
        m->last_keep = o->keep_state;
        obte_status si = OBTE_OK;
        if (ctrl[CTRL_NONFINITE]) si = fail(OBTE_ERR_NUMERIC, "non-finite kappa in mesh %d", i);
        else if (!o->only_fourier && !ctrl[CTRL_CONVERGED])
            si = fail(OBTE_ERR_NOT_CONVERGED, "mesh %d: no convergence in %d passes", i, passes);
        if (stats) {
            obte_stats& S = stats[i];
            S.outer_iters = passes;
            S.inner_iters = 0;
            S.sweeps = 0;
            for (int sys = 0; sys < m->n_sys; ++sys) { S.inner_iters += its[sys]; S.sweeps += sws[sys]; }
            S.fourier_iters = (int)fs[1];
            S.kappa = m->kappa;
            S.kappa_face = m->kappa_face;
            S.kappa_fourier = fs[0];
            S.last_rel_change = passes >= 2 ? std::fabs(hist[passes - 1] - hist[passes - 2]) /
                                                  std::fabs(hist[passes - 1])
                                            : 0.0;
            S.status = si;
            S.wrap_residual = passes > 0 ? wrh[passes - 1] : 0.0;
            S.sweep_launches = tm.launches;
            S.sweep_ms = tm.sweep_ms;
            S.reduce_ms = tm.reduce_ms;
            S.fourier_ms = 0.0;
            S.energy_residual = passes > 0 ? fs[4] : 0.0;
            if (tm.on && o->init == 0) {
                float f = 0;
                hipError_t e = hipEventElapsedTime(&f, tm.f0, tm.f1);
                if (e == hipSuccess) S.fourier_ms = f;
                else soft(e, "hipEventElapsedTime");
            }
        }
        if (kappa_out) kappa_out[i] = m->kappa;
        if (si != OBTE_OK && ret == OBTE_OK) ret = si;
    }
    return ret;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// the unstructured-mesh driver reports through the same per-thread message
void obte_set_error(const char* msg) { g_err = msg; }

extern "C" {

const char* obte_last_error(void) { return g_err.c_str(); }

void obte_default_opts(obte_solve_opts* o) {
    if (!o) return;
    o->precision = OBTE_FP64;
    o->outer_tol = 1e-8;
    o->max_outer = 1000;
    o->inner_tol = 1e-12;
    o->max_inner = 64;
    o->init = 0;
    o->only_fourier = 0;
    o->passes_per_graph = 8;
    o->waves_per_group = 0;
    o->fourier_tol = 1e-13;
    o->max_fourier = 20000;
    o->keep_state = 0;
    o->lag_wrap = 0;
    o->inner_rtol = 0.0;
    o->wrap_tol = 0.0;
    o->timing = 0;
    o->stop_rule = 0;
    o->accel = 0;
    for (int c = 0; c < 4; ++c) o->waves_by_class[c] = 0;
    o->dispatch = 0;
}

obte_status obte_mesh_create(const obte_mesh_desc* d, obte_mesh** out) {
    if (!out) return fail(OBTE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!d) return fail(OBTE_ERR_ARG, "desc is NULL");
    if (d->ndim != 2 && d->ndim != 3) return fail(OBTE_ERR_ARG, "ndim must be 2 or 3");
    const int nz = d->ndim == 3 ? d->n[2] : 1;
    for (int a = 0; a < d->ndim; ++a) {
        if (d->n[a] < 2) return fail(OBTE_ERR_ARG, "n[%d] must be >= 2", a);
        if (!(d->L[a] > 0.0) || !std::isfinite(d->L[a])) return fail(OBTE_ERR_ARG, "L[%d] must be > 0", a);
        if (d->periodic[a] != 0 && d->periodic[a] != 1) return fail(OBTE_ERR_ARG, "periodic[%d] must be 0/1", a);
    }
    if (d->n[0] > 256) return fail(OBTE_ERR_ARG, "n[0] must be <= 256");
    if (d->ndim == 3) {
        // one wave keeps a row per z-plane in LDS (checked against the LDS
        // budget per solve, which depends on the precision)
        if (nz > 128) return fail(OBTE_ERR_ARG, "3D meshes need n[2] <= 128");
        if (d->periodic[2]) return fail(OBTE_ERR_ARG, "periodic z is not supported (diffuse top/bottom)");
    }
    if (d->grad_axis < 0 || d->grad_axis > 1) return fail(OBTE_ERR_ARG, "grad_axis must be 0 or 1");
    if (!d->periodic[d->grad_axis]) return fail(OBTE_ERR_ARG, "the gradient axis must be periodic");
    if (!(d->dT_ext != 0.0) || !std::isfinite(d->dT_ext)) return fail(OBTE_ERR_ARG, "dT_ext must be finite and non-zero");
    if (!d->solid) return fail(OBTE_ERR_ARG, "solid mask is NULL");
    const long long nc = (long long)d->n[0] * d->n[1] * nz;
    if (nc > (1LL << 26)) return fail(OBTE_ERR_ARG, "mesh too large");
    obte_mesh* m = new (std::nothrow) obte_mesh();
    if (!m) return fail(OBTE_ERR_NOMEM, "host allocation failed");
    m->ndim = d->ndim;
    m->nx = d->n[0]; m->ny = d->n[1]; m->nz = nz;
    m->nf = 2 * d->ndim;
    m->ncells = (int)nc;
    for (int a = 0; a < 3; ++a) {
        m->L[a] = (a < d->ndim) ? d->L[a] : 1.0;
        m->periodic[a] = (a < d->ndim) ? d->periodic[a] : 0;
        m->h[a] = m->L[a] / (a == 0 ? m->nx : (a == 1 ? m->ny : m->nz));
    }
    m->grad_axis = d->grad_axis;
    m->dT = d->dT_ext;
    m->fc.assign(nc, 0);
    m->sidx.assign(nc, -1);
    m->wall_idx.assign(nc * m->nf, -1);
    const int n3[3] = {m->nx, m->ny, m->nz};
    for (long long c = 0; c < nc; ++c) {
        if (d->solid[c] > 1) { delete m; return fail(OBTE_ERR_ARG, "solid mask entries must be 0/1"); }
        if (!d->solid[c]) continue;
        m->sidx[c] = m->nsolid++;
        m->scell.push_back((int)c);
        const int q0[3] = {(int)(c % m->nx), (int)((c / m->nx) % m->ny), (int)(c / ((long long)m->nx * m->ny))};
        uint16_t w = 1;
        for (int a = 0; a < d->ndim; ++a)
            for (int side = 0; side < 2; ++side) {
                const int f = 2 * a + side;
                int q[3] = {q0[0], q0[1], q0[2]};
                q[a] += side ? 1 : -1;
                int cls = FC_INTERIOR;
                bool wrapped = false;
                if (q[a] < 0 || q[a] >= n3[a]) {
                    if (!m->periodic[a]) cls = FC_WALL;
                    q[a] = (q[a] + n3[a]) % n3[a];
                    wrapped = true;
                }
                if (cls != FC_WALL) {
                    const long long cc = q[0] + (long long)m->nx * (q[1] + (long long)m->ny * q[2]);
                    if (!d->solid[cc]) cls = FC_WALL;
                    else if (wrapped && a == m->grad_axis) cls = side == 0 ? FC_JUMP_P : FC_JUMP_M;
                }
                if (cls == FC_WALL) {
                    m->wall_idx[c * m->nf + f] = (int)m->wall_cell.size();
                    m->wall_cell.push_back((int)c);
                    m->wall_face.push_back(f);
                }
                w |= (uint16_t)(cls << (1 + 2 * f));
            }
        m->fc[c] = w;
    }
    m->nwalls = (int)m->wall_cell.size();
    if (m->nsolid == 0) { delete m; return fail(OBTE_ERR_ARG, "the mesh has no solid cell"); }
    *out = m;
    return OBTE_OK;
}

// Material on the (MFP, direction) grid: kappa_m kernel or a mode table
// interpolated onto it.
obte_status grid_material(obte_mesh* m, const obte_material_desc* d, bool modes) {
    if (d->n_mfp < 1 || d->n_dir < 2) return fail(OBTE_ERR_ARG, "need n_mfp >= 1 and n_dir >= 2");
    if (!d->mfp || !d->dirs || !d->dir_w || (!modes && !d->kappa_m)) return fail(OBTE_ERR_ARG, "NULL material array");
    const int nd = m->ndim;
    double wsum = 0.0;
    std::vector<double> ssum(3, 0.0);
    for (int l = 0; l < d->n_dir; ++l) {
        double nrm = 0.0;
        for (int a = 0; a < nd; ++a) nrm += d->dirs[l * nd + a] * d->dirs[l * nd + a];
        if (std::fabs(nrm - 1.0) > 1e-9) return fail(OBTE_ERR_ARG, "direction %d is not a unit vector", l);
        if (!(d->dir_w[l] > 0.0)) return fail(OBTE_ERR_ARG, "direction weight %d must be > 0", l);
        wsum += d->dir_w[l];
        for (int a = 0; a < nd; ++a) ssum[a] += d->dirs[l * nd + a] * d->dir_w[l];
    }
    if (std::fabs(wsum - 1.0) > 1e-9) return fail(OBTE_ERR_ARG, "direction weights must sum to 1");
    for (int a = 0; a < nd; ++a)
        if (std::fabs(ssum[a]) > 1e-9) return fail(OBTE_ERR_ARG, "direction set must be centrally symmetric");
    for (int mm = 0; mm < d->n_mfp; ++mm) {
        if (!(d->mfp[mm] > 0.0) || !std::isfinite(d->mfp[mm])) return fail(OBTE_ERR_ARG, "mfp[%d] must be > 0", mm);
        if (!modes && (!(d->kappa_m[mm] >= 0.0) || !std::isfinite(d->kappa_m[mm])))
            return fail(OBTE_ERR_ARG, "kappa_m[%d] must be >= 0", mm);
    }
    m->n_mfp = d->n_mfp;
    m->n_dir = d->n_dir;
    m->n_sys = d->n_mfp * d->n_dir;
    m->mfp.assign(d->mfp, d->mfp + d->n_mfp);
    if (modes) m->kappa_m.assign(d->n_mfp, 0.0);
    else m->kappa_m.assign(d->kappa_m, d->kappa_m + d->n_mfp);
    m->dir_w.assign(d->dir_w, d->dir_w + d->n_dir);
    m->dirs3.assign(3 * d->n_dir, 0.0);
    for (int l = 0; l < d->n_dir; ++l)
        for (int a = 0; a < nd; ++a) m->dirs3[l * 3 + a] = d->dirs[l * nd + a];
    // alpha_ml = kappa_m w_l / (Lambda_m^2 mu_g), mu_g = sum w s_g^2
    const int g = m->grad_axis;
    double mu = 0.0;
    for (int l = 0; l < m->n_dir; ++l) mu += m->dir_w[l] * m->dirs3[l * 3 + g] * m->dirs3[l * 3 + g];
    if (!(mu > 0.0)) return fail(OBTE_ERR_ARG, "directions have no component along the gradient axis");
    m->n_modes = 0;
    if (modes) {
        obte_status sm = mode_weights(m, d);
        if (sm != OBTE_OK) { m->n_modes = 0; return sm; }
    } else {
        m->alpha.assign(m->n_sys, 0.0);
        double asum = 0.0;
        for (int mm = 0; mm < m->n_mfp; ++mm)
            for (int l = 0; l < m->n_dir; ++l) {
                const double a = m->kappa_m[mm] * m->dir_w[l] / (m->mfp[mm] * m->mfp[mm] * mu);
                m->alpha[mm * m->n_dir + l] = a;
                asum += a;
            }
        if (!(asum > 0.0)) return fail(OBTE_ERR_ARG, "kappa_m is all zero");
        m->Dw.assign(m->n_sys, 0.0);
        m->S.assign(3 * m->n_sys, 0.0);
        m->kappa_axis.assign(3, 0.0);
        for (int mm = 0; mm < m->n_mfp; ++mm)
            for (int l = 0; l < m->n_dir; ++l) {
                const int sys = mm * m->n_dir + l;
                const double a = m->alpha[sys];
                m->Dw[sys] = a / asum;
                for (int ax = 0; ax < 3; ++ax) {
                    m->S[sys * 3 + ax] = a * m->mfp[mm] * m->dirs3[l * 3 + ax];
                    m->kappa_axis[ax] += a * m->mfp[mm] * m->mfp[mm] * m->dirs3[l * 3 + ax] * m->dirs3[l * 3 + ax];
                }
            }
    }
    return OBTE_OK;
}

// Eq. iter3 without interpolation: one system per moving mode, its
// vectorial MFP as the transport vector (stored as a direction with the
// single MFP node 1).
obte_status exact_modes(obte_mesh* m, const obte_material_desc* d) {
    const int nd = m->ndim, nm = d->n_modes;
    const int md = d->mode_dim > 0 ? d->mode_dim : nd;
    if (!(md == nd || (md == 3 && nd == 2)))
        return fail(OBTE_ERR_ARG, "mode_dim %d does not fit a %dD mesh", d->mode_dim, nd);
    std::vector<int> moving;
    double asum = 0.0, net[3] = {0.0, 0.0, 0.0}, scale = 0.0;
    for (int mu = 0; mu < nm; ++mu) {
        const double a = d->mode_alpha[mu];
        if (!(a >= 0.0) || !std::isfinite(a)) return fail(OBTE_ERR_ARG, "mode_alpha[%d] must be >= 0", mu);
        double lam2 = 0.0;
        for (int ax = 0; ax < md; ++ax) {
            const double f = d->mode_F[mu * md + ax];
            if (!std::isfinite(f)) return fail(OBTE_ERR_ARG, "mode_F[%d] is not finite", mu);
            if (ax >= nd) continue;
            lam2 += f * f;
            net[ax] += a * f;
            scale += a * std::fabs(f);
        }
        if (lam2 > 0.0) { moving.push_back(mu); asum += a; }
    }
    if (!(asum > 0.0) || moving.size() < 2) return fail(OBTE_ERR_ARG, "no mode with a nonzero MFP and weight");
    for (int ax = 0; ax < nd; ++ax)
        if (std::fabs(net[ax]) > 1e-9 * scale) return fail(OBTE_ERR_ARG, "mode table carries a net flux along axis %d", ax);
    const int n = (int)moving.size(), g = m->grad_axis;
    m->n_mfp = 1;
    m->n_dir = n;
    m->n_sys = n;
    m->mfp.assign(1, 1.0);
    m->kappa_m.assign(1, 0.0);
    m->dir_w.assign(n, 0.0);
    m->dirs3.assign(3 * (size_t)n, 0.0);
    m->alpha.assign(n, 0.0);
    m->Dw.assign(n, 0.0);
    m->S.assign(3 * (size_t)n, 0.0);
    m->kappa_axis.assign(3, 0.0);
    for (int k = 0; k < n; ++k) {
        const int mu = moving[k];
        const double a = d->mode_alpha[mu];
        m->alpha[k] = a;
        m->Dw[k] = a / asum;
        m->dir_w[k] = a / asum;
        for (int ax = 0; ax < nd; ++ax) {
            const double f = d->mode_F[mu * md + ax];
            m->dirs3[k * 3 + ax] = f;
            m->S[k * 3 + ax] = a * f;
            m->kappa_axis[ax] += a * f * f;
        }
    }
    if (!(m->kappa_axis[g] > 0.0)) return fail(OBTE_ERR_ARG, "no mode moves along the gradient axis");
    m->n_modes = nm;
    m->mode_sys.assign((size_t)nm * MODE_TERMS, 0);
    m->mode_w.assign((size_t)nm * MODE_TERMS, 0.0);
    m->mode_Sg.assign(nm, 0.0);
    for (int k = 0; k < n; ++k) {
        const int mu = moving[k];
        m->mode_sys[(size_t)mu * MODE_TERMS] = k;
        m->mode_w[(size_t)mu * MODE_TERMS] = 1.0;
        m->mode_Sg[mu] = m->S[k * 3 + g];
    }
    return OBTE_OK;
}

obte_status obte_material_set(obte_mesh* m, const obte_material_desc* d) {
    if (!m || !d) return fail(OBTE_ERR_ARG, "NULL argument");
    if (d->n_modes < 0) return fail(OBTE_ERR_ARG, "n_modes must be >= 0");
    const bool modes = d->n_modes > 0;
    if (modes && (!d->mode_F || !d->mode_alpha)) return fail(OBTE_ERR_ARG, "NULL mode table array");
    m->n_modes = 0;
    const obte_status sm = (modes && d->modes_exact) ? exact_modes(m, d) : grid_material(m, d, modes);
    if (sm != OBTE_OK) {
        m->n_modes = 0;
        m->has_material = false;
        return sm;
    }
    // outgoing wall weights per face orientation
    m->wout.assign((size_t)m->nf * m->n_sys, 0.0);
    for (int f = 0; f < m->nf; ++f) {
        const int ax = f >> 1;
        const double sg = (f & 1) ? 1.0 : -1.0;
        double tot = 0.0;
        for (int sys = 0; sys < m->n_sys; ++sys) tot += std::max(0.0, m->S[sys * 3 + ax] * sg);
        for (int sys = 0; sys < m->n_sys; ++sys)
            m->wout[(size_t)f * m->n_sys + sys] = tot > 0.0 ? std::max(0.0, m->S[sys * 3 + ax] * sg) / tot : 0.0;
    }
    // device tables
    free_dev(m);
    HIPCHK(hipGetDevice(&m->device));
    obte_status s;
    if ((s = upload(&m->d_fc, m->fc)) != OBTE_OK) return s;
    if ((s = upload(&m->d_sidx, m->sidx)) != OBTE_OK) return s;
    if ((s = upload(&m->d_scell, m->scell)) != OBTE_OK) return s;
    if ((s = upload(&m->d_wall_cell, m->wall_cell)) != OBTE_OK) return s;
    if ((s = upload(&m->d_wall_face, m->wall_face)) != OBTE_OK) return s;
    if ((s = upload(&m->d_wall_idx, m->wall_idx)) != OBTE_OK) return s;
    if ((s = upload(&m->d_mfp, m->mfp)) != OBTE_OK) return s;
    if ((s = upload(&m->d_dirs, m->dirs3)) != OBTE_OK) return s;
    if ((s = upload(&m->d_D, m->Dw)) != OBTE_OK) return s;
    if ((s = upload(&m->d_S, m->S)) != OBTE_OK) return s;
    if ((s = upload(&m->d_wout, m->wout)) != OBTE_OK) return s;
    if ((s = upload(&m->d_kax, m->kappa_axis)) != OBTE_OK) return s;
    if (m->n_modes > 0) {
        if ((s = upload(&m->d_mode_sys, m->mode_sys)) != OBTE_OK) return s;
        if ((s = upload(&m->d_mode_w, m->mode_w)) != OBTE_OK) return s;
        if ((s = upload(&m->d_mode_Sg, m->mode_Sg)) != OBTE_OK) return s;
        HIPCHK(hipMalloc((void**)&m->d_kmode, (size_t)m->n_modes * sizeof(double)));
    }
    m->modes_solved = false;
    HIPCHK(hipMalloc((void**)&m->d_geom, sizeof(GeomDev)));
    GeomDev v = make_view(m, nullptr, Layout{}, 0, 0);
    HIPCHK(hipMemcpy(m->d_geom, &v, sizeof v, hipMemcpyHostToDevice));
    m->host_view = v;
    m->has_material = true;
    m->solved = false;
    m->adj_ready = false;
    return OBTE_OK;
}

obte_status obte_workspace_size(const obte_mesh* m, const obte_solve_opts* o, size_t* bytes) {
    return obte_workspace_size_batch(&m, 1, o, bytes);
}

obte_status obte_workspace_size_batch(const obte_mesh* const* meshes, int n, const obte_solve_opts* o,
                                      size_t* bytes) {
    if (!meshes || n < 1 || !bytes) return fail(OBTE_ERR_ARG, "NULL argument or no meshes");
    obte_status s = check_opts(o);
    if (s != OBTE_OK) return s;
    for (int i = 0; i < n; ++i) {
        if (!meshes[i]) return fail(OBTE_ERR_ARG, "mesh %d is NULL", i);
        if (!meshes[i]->has_material) return fail(OBTE_ERR_STATE, "material not set on mesh %d", i);
    }
    int Wc[5];
    s = resolve_waves(meshes, n, o, Wc);
    if (s != OBTE_OK) return s;
    size_t total = 0, items = 0;
    for (int i = 0; i < n; ++i) {
        const int W = Wc[(meshes[i]->nx + 63) / 64];
        total += align256(make_layout(meshes[i], o, W).total);
        items += (size_t)meshes[i]->n_dir * n_groups(meshes[i], W);
    }
    *bytes = total + run_state_bytes(n, items);
    return OBTE_OK;
}

obte_status obte_solve(obte_mesh* m, const obte_solve_opts* o, const double* sigma_dev,
                       void* workspace, size_t ws_bytes, void* stream, double* T_L_dev,
                       double* J_dev, obte_stats* stats) {
    if (!m) return fail(OBTE_ERR_ARG, "mesh is NULL");
    const double* sg[1] = {sigma_dev};
    return solve_impl(&m, 1, o, sg, workspace, ws_bytes, stream, T_L_dev, J_dev, nullptr, stats,
                      o && o->keep_state);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Workspace of obte_solve_noalloc: a file-scope device array, one copy per
// device.  Host code never passes the array's name to a kernel or a copy: it
// uses the device address taken once per device with hipGetSymbolAddress.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t NOALLOC_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEV] = {};

// The current device's copy of the array (its address is looked up on the
// first call on each device, with that device current).
obte_status scratch_on_current_device(void** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) return fail(OBTE_ERR_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(OBTE_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return OBTE_OK;
}
}  // namespace

extern "C" {

size_t obte_noalloc_scratch_bytes(void) { return NOALLOC_BYTES; }

obte_status obte_solve_noalloc(obte_mesh* m, const obte_solve_opts* o, const double* sigma_dev, void* stream,
                               double* T_L_dev, double* J_dev, obte_stats* stats) {
    if (!m) return fail(OBTE_ERR_ARG, "mesh is NULL");
    if (!o) return fail(OBTE_ERR_ARG, "opts is NULL");
    if (o->init != 0) return fail(OBTE_ERR_ARG, "obte_solve_noalloc starts from the Fourier guess (init = 0)");
    if (o->keep_state) return fail(OBTE_ERR_ARG, "obte_solve_noalloc keeps no adjoint state (keep_state = 0)");
    if (o->timing) return fail(OBTE_ERR_ARG, "obte_solve_noalloc records no events (timing = 0)");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (m->has_material && m->device != dev)
        return fail(OBTE_ERR_ARG, "the mesh tables are on device %d, the current device is %d", m->device, dev);
    size_t need = 0;
    obte_status s = obte_workspace_size(m, o, &need);
    if (s != OBTE_OK) return s;
    if (need > NOALLOC_BYTES)
        return fail(OBTE_ERR_NOMEM, "this solve needs %zu bytes of scratch; obte_solve_noalloc has %zu "
                                    "(use obte_solve with a caller workspace)", need, NOALLOC_BYTES);
    void* ws = nullptr;
    if ((s = scratch_on_current_device(&ws)) != OBTE_OK) return s;
    const double* sg[1] = {sigma_dev};
    return solve_impl(&m, 1, o, sg, ws, NOALLOC_BYTES, stream, T_L_dev, J_dev, nullptr, stats, false, true);
}

obte_status obte_solve_batch(obte_mesh* const* meshes, int n, const obte_solve_opts* o,
                             const double* const* sigma_dev, void* workspace, size_t ws_bytes,
                             void* stream, double* kappa_out, obte_stats* stats) {
    if (o && o->keep_state) return fail(OBTE_ERR_ARG, "keep_state is not supported by the batch entry point");
    return solve_impl(meshes, n, o, sigma_dev, workspace, ws_bytes, stream, nullptr, nullptr, kappa_out,
                      stats, false);
}

obte_status obte_kappa_modes(const obte_mesh* m, double* kappa_mode) {
    if (!m || !kappa_mode) return fail(OBTE_ERR_ARG, "NULL argument");
    if (m->n_modes <= 0) return fail(OBTE_ERR_STATE, "the material has no mode table");
    if (!m->modes_solved) return fail(OBTE_ERR_STATE, "no solve with passes has completed on this mesh");
    for (int i = 0; i < m->n_modes; ++i) kappa_mode[i] = m->kappa_mode[i];
    return OBTE_OK;
}

obte_status obte_kappa(const obte_mesh* m, double* kappa_eff, double* kappa_per_mfp) {
    if (!m) return fail(OBTE_ERR_ARG, "mesh is NULL");
    if (!m->solved) return fail(OBTE_ERR_STATE, "no solve has completed on this mesh");
    if (kappa_eff) *kappa_eff = m->kappa;
    if (kappa_per_mfp)
        for (int i = 0; i < m->n_mfp; ++i) kappa_per_mfp[i] = m->kappa_per_mfp[i];
    return OBTE_OK;
}

obte_status obte_system_counts(const obte_mesh* m, long long* inner_iters, long long* sweeps) {
    if (!m) return fail(OBTE_ERR_ARG, "mesh is NULL");
    if (!m->solved) return fail(OBTE_ERR_STATE, "no solve has completed on this mesh");
    if ((int)m->sys_sweeps.size() != m->n_sys) return fail(OBTE_ERR_STATE, "the last solve ran no passes");
    for (int i = 0; i < m->n_sys; ++i) {
        if (inner_iters) inner_iters[i] = m->sys_iters[i];
        if (sweeps) sweeps[i] = m->sys_sweeps[i];
    }
    return OBTE_OK;
}

obte_status obte_adjoint(obte_mesh* m, const obte_solve_opts* o, const double* sigma_dev,
                         void* workspace, size_t ws_bytes, void* stream, double* grad_dev,
                         obte_stats* stats) {
    if (!m) return fail(OBTE_ERR_ARG, "mesh is NULL");
    obte_status s = check_opts(o);
    if (s != OBTE_OK) return s;
    if (!grad_dev) return fail(OBTE_ERR_ARG, "gradient output is NULL");
    if (!m->adj_ready || m->last_ws != workspace || m->last_sigma != sigma_dev ||
        m->last_precision != o->precision)
        return fail(OBTE_ERR_STATE, "obte_adjoint needs a converged obte_solve with keep_state = 1 "
                                    "and the same sigma, precision and workspace");
    hipStream_t st = (hipStream_t)stream;
    Run R;
    obte_solve_opts oo = *o;
    oo.waves_per_group = m->last_waves;
    for (int c = 0; c < 4; ++c) oo.waves_by_class[c] = m->last_waves_cls[c];
    oo.dispatch = m->last_dispatch;
    oo.keep_state = 1;
    obte_mesh* mp = m;
    s = build_run(R, &mp, 1, &oo, (char*)workspace, nullptr);
    if (s != OBTE_OK) return s;
    Layout L = make_layout(m, &oo, R.cls_waves[1]);
    if (ws_bytes < R.state_off + R.state_bytes)
        return fail(OBTE_ERR_NOMEM, "workspace too small for the adjoint (accel deeper than the forward solve's?)");
    if ((s = upload_run(R, (char*)workspace)) != OBTE_OK) return s;
    if ((s = ensure_stage(m, STAGE_LOOP)) != OBTE_OK) return s;
    R.h_pin = (int*)m->h_stage;
    char* ws = (char*)workspace;
    // lambda^(0) = 0: Psi = Phi = 0, no warm start, fresh counters
    HIPCHK(hipMemsetAsync(ws + L.lam_psi, 0, 2 * (size_t)m->ncells * 8, st));
    HIPCHK(hipMemsetAsync(ws + L.lam_phi, 0, 2 * (size_t)std::max(m->nwalls, 1) * 8, st));
    const size_t tsz = o->precision == OBTE_FP32 ? 4 : 8;
    const size_t half = (size_t)m->n_sys * m->nx * m->nz * tsz;
    HIPCHK(hipMemsetAsync(ws + L.U + half, 0, half, st));
    HIPCHK(hipMemsetAsync(ws + L.bnd + 2 * (size_t)m->nf * m->ncells * 8, 0,
                          2 * (size_t)m->nf * m->ncells * 8, st));
    HIPCHK(hipMemsetAsync(ws + L.iters, 0, 2 * (size_t)m->n_sys * 8, st));
    HIPCHK(hipMemsetAsync(ws + L.wres, 0, (size_t)m->n_sys * 8, st));
    HIPCHK(hipMemsetAsync(ws + L.ctrl, 0, CTRL_N * sizeof(int), st));
    HIPCHK(hipMemsetAsync(ws + L.ax, 0, ((size_t)m->ncells + m->nwalls) * 8, st));
    HIPCHK(hipMemsetAsync(ws + L.actl, 0, 8 * sizeof(int), st));
    PassParams pp = base_params(o);
    pp.adjoint = 1;
    pp.sigma1 = sigma_dev ? 0 : 1;
    const int K = (o->passes_per_graph <= 1 || !st || o->timing) ? 1 : o->passes_per_graph;
    Timer tm;
    if (o->timing && (s = tm.init(K)) != OBTE_OK) return s;
    s = outer_loop(R, pp, K, st, o->max_outer, &tm, &m->g_adj);
    if (s != OBTE_OK) return s;
    HIPCHK(launch_output(m->d_geom, R.precision, m->ncells, nullptr, nullptr, grad_dev, st));
    std::vector<int> ctrl(CTRL_N);
    HIPCHK(hipMemcpyAsync(ctrl.data(), R.views[0].ctrl, CTRL_N * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int passes = ctrl[CTRL_PASS];
    std::vector<double> hist(std::max(passes, 1));
    if (passes > 0) HIPCHK(hipMemcpy(hist.data(), R.views[0].hist, passes * sizeof(double), hipMemcpyDeviceToHost));
    if (stats) {
        std::vector<long long> its(m->n_sys), sws(m->n_sys);
        HIPCHK(hipMemcpy(its.data(), R.views[0].iters, m->n_sys * 8, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(sws.data(), R.views[0].sweeps, m->n_sys * 8, hipMemcpyDeviceToHost));
        stats->outer_iters = passes;
        stats->inner_iters = 0;
        stats->sweeps = 0;
        for (int i = 0; i < m->n_sys; ++i) { stats->inner_iters += its[i]; stats->sweeps += sws[i]; }
        stats->fourier_iters = 0;
        stats->kappa = passes > 0 ? hist[passes - 1] : 0.0;   // p^T lambda
        stats->kappa_face = 0.0;
        stats->kappa_fourier = m->kappa_fourier;
        stats->last_rel_change = passes >= 2 ? std::fabs(hist[passes - 1] - hist[passes - 2]) / std::fabs(hist[passes - 1]) : 0.0;
        stats->status = ctrl[CTRL_CONVERGED] ? OBTE_OK : OBTE_ERR_NOT_CONVERGED;
        stats->sweep_launches = tm.launches;
        stats->sweep_ms = tm.sweep_ms;
        stats->reduce_ms = tm.reduce_ms;
        stats->fourier_ms = 0.0;
        stats->energy_residual = 0.0;
    }
    if (ctrl[CTRL_NONFINITE]) return fail(OBTE_ERR_NUMERIC, "non-finite adjoint functional");
    if (!ctrl[CTRL_CONVERGED]) return fail(OBTE_ERR_NOT_CONVERGED, "adjoint: no convergence in %d passes", passes);
    return OBTE_OK;
}

obte_status obte_upwind_apply(const obte_mesh* m, int precision, int transpose, const double* sigma_dev,
                              const int* sys_ids_dev, int n_sys, const void* x_dev, void* y_dev,
                              void* stream) {
    if (!m || !x_dev || !y_dev || !sys_ids_dev) return fail(OBTE_ERR_ARG, "NULL argument");
    if (!m->has_material) return fail(OBTE_ERR_STATE, "material not set");
    if (precision != 0 && precision != 1) return fail(OBTE_ERR_ARG, "precision must be 0 or 1");
    if (n_sys < 1 || n_sys > 65535) return fail(OBTE_ERR_ARG, "n_sys must be in 1..65535");
    HIPCHK(launch_apply(precision, transpose ? 1 : 0, m->d_geom, m->host_view, sigma_dev, sys_ids_dev,
                        n_sys, x_dev, y_dev, (hipStream_t)stream));
    return OBTE_OK;
}

obte_status obte_checkpoint_save(const obte_mesh* m, const void* workspace, const char* path) {
    if (!m || !workspace || !path) return fail(OBTE_ERR_ARG, "NULL argument");
    if (!m->solved) return fail(OBTE_ERR_STATE, "nothing to checkpoint");
    if (m->last_ws != workspace) return fail(OBTE_ERR_ARG, "workspace differs from the last solve's");
    // every check precedes the open: a rejected call leaves the file untouched
    FILE* f = fopen(path, "wb");
    if (!f) return fail(OBTE_ERR_ARG, "cannot open %s", path);
    // header: magic, sizes; body: ctrl, T_L, sT (2), Tw (2), U, hist
    const GeomDev& v = m->host_view;
    const int hdr[9] = {CKPT_MAGIC, m->ncells, m->nwalls, m->n_sys, m->nx * m->nz, m->last_precision,
                        m->last_waves, m->last_max_outer, m->last_keep};
    fwrite(hdr, sizeof hdr, 1, f);
    auto dump = [&](const void* dptr, size_t bytes) -> bool {
        std::vector<char> buf(bytes);
        if (hipMemcpy(buf.data(), dptr, bytes, hipMemcpyDeviceToHost) != hipSuccess) return false;
        return fwrite(buf.data(), 1, bytes, f) == bytes;
    };
    std::vector<int> ctrl(CTRL_N);
    bool ok = dump(v.ctrl, CTRL_N * sizeof(int));
    if (ok && hipMemcpy(ctrl.data(), v.ctrl, CTRL_N * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) ok = false;
    const size_t tsz = m->last_precision == OBTE_FP32 ? 4 : 8;
    ok = ok && dump(v.T_L, (size_t)m->ncells * 8) && dump(v.sT, 2 * (size_t)m->ncells * 8) &&
         dump(v.Tw, 2 * (size_t)std::max(m->nwalls, 1) * 8) &&
         dump(v.U, (size_t)m->n_sys * m->nx * m->nz * tsz) &&
         dump(v.bnd, 2 * (size_t)m->nf * m->ncells * 8) &&
         dump(v.ax, ((size_t)m->ncells + m->nwalls) * 8);
    const int passes = ctrl[CTRL_PASS];
    fwrite(&passes, sizeof passes, 1, f);
    ok = ok && (passes == 0 || dump(v.hist, (size_t)passes * 8)) && (passes == 0 || dump(v.hist_face, (size_t)passes * 8));
    fclose(f);
    if (!ok) return fail(OBTE_ERR_HIP, "checkpoint write failed");
    return OBTE_OK;
}

obte_status obte_checkpoint_load(obte_mesh* m, void* workspace, const char* path) {
    if (!m || !workspace || !path) return fail(OBTE_ERR_ARG, "NULL argument");
    if (!m->has_material) return fail(OBTE_ERR_STATE, "material not set");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(OBTE_ERR_ARG, "cannot open %s", path);
    int hdr[9];
    if (fread(hdr, sizeof hdr, 1, f) != 1 || hdr[0] != CKPT_MAGIC || hdr[1] != m->ncells ||
        hdr[2] != m->nwalls || hdr[3] != m->n_sys || hdr[4] != m->nx * m->nz) {
        fclose(f);
        return fail(OBTE_ERR_ARG, "checkpoint does not match this mesh / precision");
    }
    obte_solve_opts o;
    obte_default_opts(&o);
    o.precision = hdr[5];
    o.max_outer = hdr[7];
    o.keep_state = hdr[8];
    const GeomDev v = make_view(m, (char*)workspace, make_layout(m, &o, hdr[6]), hdr[6], 0);
    auto load = [&](void* dptr, size_t bytes) -> bool {
        std::vector<char> buf(bytes);
        if (fread(buf.data(), 1, bytes, f) != bytes) return false;
        return hipMemcpy(dptr, buf.data(), bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    const size_t tsz = hdr[5] == OBTE_FP32 ? 4 : 8;
    bool ok = load(v.ctrl, CTRL_N * sizeof(int)) && load(v.T_L, (size_t)m->ncells * 8) &&
              load(v.sT, 2 * (size_t)m->ncells * 8) && load(v.Tw, 2 * (size_t)std::max(m->nwalls, 1) * 8) &&
              load(v.U, (size_t)m->n_sys * m->nx * m->nz * tsz) &&
              load(v.bnd, 2 * (size_t)m->nf * m->ncells * 8) &&
              load(v.ax, ((size_t)m->ncells + m->nwalls) * 8);
    int passes = 0;
    ok = ok && fread(&passes, sizeof passes, 1, f) == 1;
    ok = ok && (passes == 0 || load(v.hist, (size_t)passes * 8)) && (passes == 0 || load(v.hist_face, (size_t)passes * 8));
    fclose(f);
    if (!ok) return fail(OBTE_ERR_ARG, "checkpoint read failed");
    m->last_precision = hdr[5];
    m->last_waves = hdr[6];
    m->last_max_outer = hdr[7];
    m->last_keep = hdr[8];
    return OBTE_OK;
}

void obte_mesh_destroy(obte_mesh* m) {
    if (!m) return;
    free_dev(m);
    if (m->h_stage) soft(hipHostFree(m->h_stage), "hipHostFree(stage)");
    delete m;
}

int obte_mesh_n_cells(const obte_mesh* m) { return m ? m->ncells : -1; }
int obte_mesh_n_solid(const obte_mesh* m) { return m ? m->nsolid : -1; }
int obte_mesh_n_walls(const obte_mesh* m) { return m ? m->nwalls : -1; }
int obte_mesh_n_systems(const obte_mesh* m) { return m ? m->n_sys : -1; }
int obte_mesh_n_modes(const obte_mesh* m) { return m ? m->n_modes : -1; }

}  // extern "C"
