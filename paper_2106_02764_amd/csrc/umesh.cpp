// Host driver of the unstructured-mesh path: polygon geometry and face
// lists, material weights, the per-direction upwind order, the tables of
// the non-orthogonal heat-conduction solve, and Algorithm 1's outer loop.
//
// Geometry (plain definitions): polygon area by the shoelace formula, the
// area centroid, edge length and the outward unit normal (dy, -dx) / |e| of
// each counter-clockwise edge.  An interior face joins two solid cells; d
// runs from the first cell's centroid to the centroid of the second cell's
// periodic image, and that image carries T + delta dT with
// T(x + L_g) = T(x) - dT (delta = minus the image shift along the gradient
// axis).  Faces towards pore cells are diffuse walls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/obte.h"
#include "obte_internal.h"
#include "umesh_internal.h"

namespace {

obte_status ufail(obte_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    obte_set_error(buf);
    return st;
}

#define UHIP(call)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ufail(OBTE_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

constexpr int MAX_SOLID = 8192;     // with the wrap slots: one workgroup's 64 KiB of LDS
static_assert(MAX_SOLID <= 256 * UF_MAXB, "heat-conduction partials: one slot per block of 256 cells");

}  // namespace

struct obte_umesh {
    double L[2] = {0, 0}, dT = 1.0;
    int ga = 0;
    int n_cells = 0, ns = 0, nf = 0, nw = 0;
    std::vector<int> scell, sid;
    std::vector<double> V, xc;                 // ns, 2 ns
    std::vector<int> fi, fj, fper;             // interior faces; fper: 1 across a periodic boundary
    std::vector<double> fA, fn, fd, fdel, fw;  // fn, fd: 2 per face
    std::vector<int> wcell;
    std::vector<double> wA, wn;
    std::vector<std::vector<int>> cfaces;      // per solid cell: 2 f (+1 if second cell), or -(w + 1)
    // material
    bool has_material = false;
    int n_mfp = 0, n_dir = 0, n_sys = 0;
    std::vector<double> mfp, dirs, Dw, S, wout;
    double kax[2] = {0, 0};
    std::vector<int> nlev;
    int wmax = 0;
    // device
    std::vector<void*> dev;
    UGeomDev gh{};
    UGeomDev* gd = nullptr;
    UFourierDev fh{};
    UFourierDev* fdv = nullptr;
    double* sigma1 = nullptr;
    int* scell_d = nullptr;
    int* wcell_d = nullptr;
    double* h_fsc = nullptr;                   // pinned: the heat-conduction loop scalars read back
};

namespace {

void free_dev(obte_umesh* m) {
    for (void* p : m->dev) (void)hipFree(p);
    m->dev.clear();
    if (m->h_fsc) (void)hipHostFree(m->h_fsc);
    m->h_fsc = nullptr;
    m->gd = nullptr;
    m->fdv = nullptr;
    (void)hipGetLastError();
}

template <typename T>
obte_status upload(obte_umesh* m, T** dst, const std::vector<T>& v) {
    const size_t n = std::max<size_t>(v.size(), 1);
    void* p = nullptr;
    UHIP(hipMalloc(&p, n * sizeof(T)));
    m->dev.push_back(p);
    if (!v.empty()) UHIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *dst = (T*)p;
    return OBTE_OK;
}

template <typename T>
obte_status alloc(obte_umesh* m, T** dst, size_t n) {
    void* p = nullptr;
    UHIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
    m->dev.push_back(p);
    UHIP(hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(T)));
    *dst = (T*)p;
    return OBTE_OK;
}

__global__ void k_uscatter(int ns, const int* __restrict__ scell, const double* __restrict__ src,
                           double* __restrict__ dst, double shift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns) dst[scell[i]] = src[i] - shift;
}

__global__ void k_ugather(int n, const int* __restrict__ idx, const double* __restrict__ src, double* __restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

}  // namespace

extern "C" {

obte_status obte_umesh_create(const double* nodes, int n_nodes, const int* cells, const int* shifts, int n_cells,
                              int nv, const unsigned char* solid, double Lx, double Ly, int grad_axis, double dT,
                              obte_umesh** out) {
    if (!out) return ufail(OBTE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!nodes || !cells || !shifts || !solid) return ufail(OBTE_ERR_ARG, "NULL mesh array");
    if (n_nodes < 3 || n_cells < 1) return ufail(OBTE_ERR_ARG, "need at least 3 nodes and 1 cell");
    if (nv != 3 && nv != 4) return ufail(OBTE_ERR_ARG, "cells must be triangles or quadrilaterals (nv 3 or 4)");
    if (!(Lx > 0.0) || !(Ly > 0.0) || !std::isfinite(Lx) || !std::isfinite(Ly))
        return ufail(OBTE_ERR_ARG, "Lx and Ly must be > 0");
    if (grad_axis != 0 && grad_axis != 1) return ufail(OBTE_ERR_ARG, "grad_axis must be 0 or 1");
    if (!(dT > 0.0) || !std::isfinite(dT)) return ufail(OBTE_ERR_ARG, "dT must be > 0");
    for (long long q = 0; q < (long long)n_cells * nv; ++q)
        if (cells[q] < 0 || cells[q] >= n_nodes) return ufail(OBTE_ERR_ARG, "cell node id out of range");
    obte_umesh* m = new obte_umesh();
    m->L[0] = Lx;
    m->L[1] = Ly;
    m->dT = dT;
    m->ga = grad_axis;
    m->n_cells = n_cells;
    // corner positions in each cell's own frame, areas and centroids
    std::vector<double> P((size_t)n_cells * nv * 2), area(n_cells), cen(2 * (size_t)n_cells);
    for (int c = 0; c < n_cells; ++c) {
        for (int k = 0; k < nv; ++k) {
            const size_t q = (size_t)c * nv + k;
            P[2 * q] = nodes[2 * cells[q]] + shifts[2 * q] * Lx;
            P[2 * q + 1] = nodes[2 * cells[q] + 1] + shifts[2 * q + 1] * Ly;
        }
        double a = 0.0, cx = 0.0, cy = 0.0;
        for (int k = 0; k < nv; ++k) {
            const size_t q0 = (size_t)c * nv + k, q1 = (size_t)c * nv + (k + 1) % nv;
            const double x0 = P[2 * q0], y0 = P[2 * q0 + 1], x1 = P[2 * q1], y1 = P[2 * q1 + 1];
            const double cr = x0 * y1 - x1 * y0;
            a += cr;
            cx += (x0 + x1) * cr;
            cy += (y0 + y1) * cr;
        }
        a *= 0.5;
        if (!(a > 0.0)) {
            delete m;
            return ufail(OBTE_ERR_ARG, "cell %d is clockwise or degenerate", c);
        }
        area[c] = a;
        cen[2 * c] = cx / (6.0 * a);
        cen[2 * c + 1] = cy / (6.0 * a);
    }
    // edges keyed by their node ids and the relative image shift
    using Key = std::array<long long, 4>;
    auto key_of = [&](int c, int k) {
        const size_t q0 = (size_t)c * nv + k, q1 = (size_t)c * nv + (k + 1) % nv;
        const long long a = cells[q0], b = cells[q1];
        if (a < b) return Key{a, b, shifts[2 * q1] - shifts[2 * q0], shifts[2 * q1 + 1] - shifts[2 * q0 + 1]};
        return Key{b, a, shifts[2 * q0] - shifts[2 * q1], shifts[2 * q0 + 1] - shifts[2 * q1 + 1]};
    };
    std::map<Key, std::vector<std::pair<int, int>>> edges;
    for (int c = 0; c < n_cells; ++c)
        for (int k = 0; k < nv; ++k) {
            const Key kk = key_of(c, k);
            if (kk[0] == kk[1]) {
                delete m;
                return ufail(OBTE_ERR_ARG, "cell %d has an edge from a node to itself", c);
            }
            edges[kk].push_back({c, k});
        }
    for (const auto& e : edges)
        if (e.second.size() != 2) {
            delete m;
            return ufail(OBTE_ERR_ARG, "an edge of cell %d is shared by %zu cells (need 2)", e.second[0].first,
                         e.second.size());
        }
    m->sid.assign(n_cells, -1);
    for (int c = 0; c < n_cells; ++c)
        if (solid[c]) {
            m->sid[c] = m->ns++;
            m->scell.push_back(c);
        }
    if (m->ns == 0) {
        delete m;
        return ufail(OBTE_ERR_ARG, "the mesh has no solid cell");
    }
    if (m->ns > MAX_SOLID) {
        const int ns = m->ns;
        delete m;
        return ufail(OBTE_ERR_ARG, "%d solid cells: the unstructured path takes at most %d", ns, MAX_SOLID);
    }
    for (int i = 0; i < m->ns; ++i) {
        const int c = m->scell[i];
        m->V.push_back(area[c]);
        m->xc.push_back(cen[2 * c]);
        m->xc.push_back(cen[2 * c + 1]);
    }
    m->cfaces.assign(m->ns, {});
    std::map<Key, int> face_of;
    for (int i = 0; i < m->ns; ++i) {
        const int c = m->scell[i];
        for (int k = 0; k < nv; ++k) {
            const Key kk = key_of(c, k);
            const auto& occ = edges[kk];
            const std::pair<int, int> other = occ[0] == std::make_pair(c, k) ? occ[1] : occ[0];
            const int c2 = other.first;
            const size_t q0 = (size_t)c * nv + k, q1 = (size_t)c * nv + (k + 1) % nv;
            const double ex = P[2 * q1] - P[2 * q0], ey = P[2 * q1 + 1] - P[2 * q0 + 1];
            const double len = std::hypot(ex, ey);
            const double nx = ey / len, ny = -ex / len;
            if (!solid[c2]) {
                m->cfaces[i].push_back(-(m->nw + 1));
                m->wcell.push_back(i);
                m->wA.push_back(len);
                m->wn.push_back(nx);
                m->wn.push_back(ny);
                ++m->nw;
                continue;
            }
            const auto it = face_of.find(kk);
            if (it != face_of.end()) {
                m->cfaces[i].push_back(2 * it->second + 1);
                continue;
            }
            // image offset bringing c2 into c's frame, from the shared nodes
            const int a = cells[q0], b = cells[q1];
            bool found = false;
            long long ox = 0, oy = 0;
            for (int qa = 0; qa < nv && !found; ++qa) {
                if (cells[(size_t)c2 * nv + qa] != a) continue;
                const long long cx_ = shifts[2 * q0] - shifts[2 * ((size_t)c2 * nv + qa)];
                const long long cy_ = shifts[2 * q0 + 1] - shifts[2 * ((size_t)c2 * nv + qa) + 1];
                for (int qb = 0; qb < nv; ++qb) {
                    const size_t r = (size_t)c2 * nv + qb;
                    if (cells[r] == b && shifts[2 * q1] - shifts[2 * r] == cx_ && shifts[2 * q1 + 1] - shifts[2 * r + 1] == cy_) {
                        ox = cx_;
                        oy = cy_;
                        found = true;
                        break;
                    }
                }
            }
            if (!found) {
                delete m;
                return ufail(OBTE_ERR_ARG, "inconsistent periodic shifts on an edge of cell %d", c);
            }
            const int f = m->nf++;
            face_of[kk] = f;
            m->cfaces[i].push_back(2 * f);
            const double dx = cen[2 * c2] + ox * Lx - cen[2 * c], dy = cen[2 * c2 + 1] + oy * Ly - cen[2 * c + 1];
            m->fi.push_back(i);
            m->fj.push_back(m->sid[c2]);
            m->fper.push_back(ox != 0 || oy != 0);
            m->fA.push_back(len);
            m->fn.push_back(nx);
            m->fn.push_back(ny);
            m->fd.push_back(dx);
            m->fd.push_back(dy);
            m->fdel.push_back(-(double)(grad_axis == 0 ? ox : oy));
            // fraction of d at which the centroid line crosses the face
            const double nd = dx * nx + dy * ny;
            m->fw.push_back(((P[2 * q0] - cen[2 * c]) * nx + (P[2 * q0 + 1] - cen[2 * c + 1]) * ny) / nd);
        }
    }
    *out = m;
    return OBTE_OK;
}

obte_status obte_umesh_material_set(obte_umesh* m, const double* mfp, int n_mfp, const double* dirs,
                                    const double* dir_w, int n_dir, const double* kappa_m) {
    if (!m) return ufail(OBTE_ERR_ARG, "mesh is NULL");
    if (!mfp || !dirs || !dir_w || !kappa_m) return ufail(OBTE_ERR_ARG, "NULL material array");
    if (n_mfp < 1 || n_dir < 2) return ufail(OBTE_ERR_ARG, "need n_mfp >= 1 and n_dir >= 2");
    double wsum = 0.0, sx = 0.0, sy = 0.0;
    for (int l = 0; l < n_dir; ++l) {
        const double x = dirs[2 * l], y = dirs[2 * l + 1];
        if (std::fabs(x * x + y * y - 1.0) > 1e-9) return ufail(OBTE_ERR_ARG, "direction %d is not a unit vector", l);
        if (!(dir_w[l] > 0.0)) return ufail(OBTE_ERR_ARG, "direction weight %d must be > 0", l);
        wsum += dir_w[l];
        sx += x * dir_w[l];
        sy += y * dir_w[l];
    }
    if (std::fabs(wsum - 1.0) > 1e-9) return ufail(OBTE_ERR_ARG, "direction weights must sum to 1");
    if (std::fabs(sx) > 1e-9 || std::fabs(sy) > 1e-9)
        return ufail(OBTE_ERR_ARG, "direction set must be centrally symmetric");
    for (int k = 0; k < n_mfp; ++k) {
        if (!(mfp[k] > 0.0) || !std::isfinite(mfp[k])) return ufail(OBTE_ERR_ARG, "mfp[%d] must be > 0", k);
        if (!(kappa_m[k] >= 0.0) || !std::isfinite(kappa_m[k])) return ufail(OBTE_ERR_ARG, "kappa_m[%d] must be >= 0", k);
    }
    free_dev(m);
    m->has_material = false;
    const int ns = m->ns, nw = m->nw, nf = m->nf, ga = m->ga;
    m->n_mfp = n_mfp;
    m->n_dir = n_dir;
    m->n_sys = n_mfp * n_dir;
    m->mfp.assign(mfp, mfp + n_mfp);
    m->dirs.assign(dirs, dirs + 2 * n_dir);
    // alpha_ml = kappa_m w_l / (Lambda_m^2 mu_g), D = alpha / sum alpha,
    // S = alpha Lambda s (section Model, Appendix A)
    double mu = 0.0;
    for (int l = 0; l < n_dir; ++l) mu += dir_w[l] * dirs[2 * l + ga] * dirs[2 * l + ga];
    if (!(mu > 0.0)) return ufail(OBTE_ERR_ARG, "directions have no component along the gradient axis");
    std::vector<double> alpha(m->n_sys);
    double asum = 0.0;
    for (int k = 0; k < n_mfp; ++k)
        for (int l = 0; l < n_dir; ++l) {
            alpha[k * n_dir + l] = kappa_m[k] * dir_w[l] / (mfp[k] * mfp[k] * mu);
            asum += alpha[k * n_dir + l];
        }
    if (!(asum > 0.0)) return ufail(OBTE_ERR_ARG, "kappa_m is all zero");
    m->Dw.assign(m->n_sys, 0.0);
    m->S.assign(2 * (size_t)m->n_sys, 0.0);
    m->kax[0] = m->kax[1] = 0.0;
    for (int k = 0; k < n_mfp; ++k)
        for (int l = 0; l < n_dir; ++l) {
            const int sys = k * n_dir + l;
            m->Dw[sys] = alpha[sys] / asum;
            for (int a = 0; a < 2; ++a) {
                m->S[2 * sys + a] = alpha[sys] * mfp[k] * dirs[2 * l + a];
                m->kax[a] += alpha[sys] * mfp[k] * mfp[k] * dirs[2 * l + a] * dirs[2 * l + a];
            }
        }
    // outgoing weights of each wall face: ReLu(S . n) / sum ReLu(S . n)
    m->wout.assign((size_t)nw * m->n_sys, 0.0);
    for (int w = 0; w < nw; ++w) {
        double tot = 0.0;
        for (int sys = 0; sys < m->n_sys; ++sys)
            tot += std::max(0.0, m->S[2 * sys] * m->wn[2 * w] + m->S[2 * sys + 1] * m->wn[2 * w + 1]);
        for (int sys = 0; sys < m->n_sys; ++sys) {
            const double r = std::max(0.0, m->S[2 * sys] * m->wn[2 * w] + m->S[2 * sys + 1] * m->wn[2 * w + 1]);
            m->wout[(size_t)w * m->n_sys + sys] = tot > 0.0 ? r / tot : 0.0;
        }
    }
    // ---- per-direction upwind order (periodic faces cut) and wrap slots
    std::vector<int> ord((size_t)n_dir * ns), lbase(n_dir), lptr, nwrap(n_dir, 0);
    std::vector<int> inc((size_t)n_dir * ns * UFACES, UNONE);
    std::vector<double> dout((size_t)n_dir * ns, 0.0), inv((size_t)n_dir * ns * UFACES, 0.0);
    std::vector<std::vector<int>> wup_l(n_dir);
    std::vector<std::vector<double>> wdel_l(n_dir);
    m->nlev.assign(n_dir, 0);
    for (int l = 0; l < n_dir; ++l) {
        const double s0 = dirs[2 * l], s1 = dirs[2 * l + 1];
        std::vector<double> dcell(ns, 0.0);
        std::vector<std::array<int, UFACES>> icode(ns);
        std::vector<std::array<double, UFACES>> icoef(ns);
        std::vector<int> indeg(ns, 0), nin(ns, 0);
        std::vector<std::vector<int>> down(ns);
        for (int i = 0; i < ns; ++i) {
            icode[i].fill(UNONE);
            icoef[i].fill(0.0);
            for (int code : m->cfaces[i]) {
                double nx, ny, A;
                int j = -1, w = -1, f = -1;
                bool second = false;
                if (code < 0) {
                    w = -code - 1;
                    nx = m->wn[2 * w];
                    ny = m->wn[2 * w + 1];
                    A = m->wA[w];
                } else {
                    f = code >> 1;
                    second = code & 1;
                    const double sg = second ? -1.0 : 1.0;
                    nx = sg * m->fn[2 * f];
                    ny = sg * m->fn[2 * f + 1];
                    A = m->fA[f];
                    j = second ? m->fi[f] : m->fj[f];
                }
                const double sn = s0 * nx + s1 * ny;
                if (sn > 0.0) {
                    dcell[i] += sn * A / m->V[i];
                } else if (sn < 0.0) {
                    const int q = nin[i]++;
                    icoef[i][q] = -sn * A / m->V[i];
                    if (w >= 0) {
                        icode[i][q] = UWALL0 - w;
                    } else if (m->fper[f]) {
                        const int slot = nwrap[l]++;
                        wup_l[l].push_back(j);
                        wdel_l[l].push_back((second ? -m->fdel[f] : m->fdel[f]) * m->dT);
                        icode[i][q] = ns + slot;
                    } else {
                        icode[i][q] = j;
                        ++indeg[i];
                        down[j].push_back(i);
                    }
                }
            }
        }
        // levels: a cell follows every upwind neighbour it reads
        std::vector<int> level(ns, 0), queue;
        queue.reserve(ns);
        for (int i = 0; i < ns; ++i)
            if (indeg[i] == 0) queue.push_back(i);
        for (size_t h = 0; h < queue.size(); ++h) {
            const int u = queue[h];
            for (int v : down[u]) {
                level[v] = std::max(level[v], level[u] + 1);
                if (--indeg[v] == 0) queue.push_back(v);
            }
        }
        if ((int)queue.size() != ns)
            return ufail(OBTE_ERR_ARG, "the upwind graph of direction %d has a cycle (non-convex cells?)", l);
        std::vector<int> byl(ns);
        for (int i = 0; i < ns; ++i) byl[i] = i;
        std::stable_sort(byl.begin(), byl.end(), [&](int a, int b) { return level[a] < level[b]; });
        const int nl = ns ? level[byl[ns - 1]] + 1 : 0;
        m->nlev[l] = nl;
        lbase[l] = (int)lptr.size();
        int p = 0;
        for (int k = 0; k < nl; ++k) {
            lptr.push_back(p);
            while (p < ns && level[byl[p]] == k) ++p;
        }
        lptr.push_back(ns);
        for (int p2 = 0; p2 < ns; ++p2) {
            const int i = byl[p2];
            const size_t pl = (size_t)l * ns + p2;
            ord[pl] = i;
            dout[pl] = dcell[i];
            for (int q = 0; q < UFACES; ++q) {
                inc[pl * UFACES + q] = icode[i][q];
                inv[pl * UFACES + q] = icoef[i][q];
            }
        }
    }
    int wmax = 0;
    for (int l = 0; l < n_dir; ++l) wmax = std::max(wmax, nwrap[l]);
    if (wmax > UWPL_MAX * 64) return ufail(OBTE_ERR_ARG, "%d periodic faces in one direction (at most %d)", wmax, UWPL_MAX * 64);
    if ((size_t)(ns + wmax) * 8 > 65536)
        return ufail(OBTE_ERR_ARG, "%d solid cells and %d periodic faces exceed one workgroup's LDS", ns, wmax);
    m->wmax = std::max(wmax, 1);
    std::vector<int> wup((size_t)n_dir * m->wmax, 0);
    std::vector<double> wdel((size_t)n_dir * m->wmax, 0.0);
    for (int l = 0; l < n_dir; ++l)
        for (int q = 0; q < nwrap[l]; ++q) {
            wup[(size_t)l * m->wmax + q] = wup_l[l][q];
            wdel[(size_t)l * m->wmax + q] = wdel_l[l][q];
        }
    // ---- heat conduction tables (Appendix B, volume-scaled): per cell its
    // neighbour entries with the primary coefficient a = A n.K n / (n.d),
    // the jump of the neighbour's image and the least-squares weights
    const double Kx = m->kax[0], Ky = m->kax[1];
    std::vector<int> nb_ptr(ns + 1, 0), nb_j, nb_f;
    std::vector<double> nb_a, nb_del, nb_w, P(ns, 0.0);
    std::vector<double> fa(nf), fc(2 * (size_t)nf);
    for (int f = 0; f < nf; ++f) {
        const double nx = m->fn[2 * f], ny = m->fn[2 * f + 1], dx = m->fd[2 * f], dy = m->fd[2 * f + 1];
        const double nKn = nx * nx * Kx + ny * ny * Ky, nd = nx * dx + ny * dy;
        fa[f] = m->fA[f] * nKn / nd;
        fc[2 * f] = m->fA[f] * (dx * nKn / nd - Kx * nx);
        fc[2 * f + 1] = m->fA[f] * (dy * nKn / nd - Ky * ny);
    }
    for (int i = 0; i < ns; ++i) {
        std::vector<std::array<double, 2>> dl;
        const size_t k0 = nb_j.size();
        for (int code : m->cfaces[i]) {
            if (code < 0) continue;
            const int f = code >> 1;
            const bool second = code & 1;
            const double sg = second ? -1.0 : 1.0;
            nb_j.push_back(second ? m->fi[f] : m->fj[f]);
            nb_a.push_back(fa[f]);
            const double del = sg * m->fdel[f];
            nb_del.push_back(del);
            nb_f.push_back(code);
            dl.push_back({sg * m->fd[2 * f], sg * m->fd[2 * f + 1]});
            P[i] -= fa[f] * del * m->dT;
        }
        nb_ptr[i + 1] = (int)nb_j.size();
        // least squares: g = (M^T M)^+ M^T q, M's rows the d's
        double a11 = 0.0, a12 = 0.0, a22 = 0.0;
        for (const auto& d : dl) {
            a11 += d[0] * d[0];
            a12 += d[0] * d[1];
            a22 += d[1] * d[1];
        }
        const double tr = a11 + a22, det = a11 * a22 - a12 * a12;
        double i11, i12, i22;
        if (dl.empty()) {
            i11 = i12 = i22 = 0.0;
        } else if (det > 1e-12 * tr * tr) {
            i11 = a22 / det;
            i12 = -a12 / det;
            i22 = a11 / det;
        } else {
            // rank one: the pseudo-inverse keeps the dominant eigenpair
            const double lam = 0.5 * tr + std::sqrt(std::max(0.0, 0.25 * (a11 - a22) * (a11 - a22) + a12 * a12));
            double vx = a12, vy = lam - a11;
            if (std::fabs(vx) + std::fabs(vy) == 0.0) {
                vx = lam - a22;
                vy = a12;
            }
            if (std::fabs(vx) + std::fabs(vy) == 0.0) {
                vx = 1.0;
                vy = 0.0;
            }
            const double nn = vx * vx + vy * vy;
            i11 = vx * vx / (nn * lam);
            i12 = vx * vy / (nn * lam);
            i22 = vy * vy / (nn * lam);
        }
        for (size_t k = 0; k < dl.size(); ++k) {
            nb_w.push_back(i11 * dl[k][0] + i12 * dl[k][1]);
            nb_w.push_back(i12 * dl[k][0] + i22 * dl[k][1]);
        }
        (void)k0;
    }
    // cut faces (across the periodic plane of the gradient axis), oriented
    // from the cell on the + side
    std::vector<int> cut_f, cut_s, cut_i, cut_j;
    std::vector<double> cut_K, cut_d, cut_A, cut_An;
    for (int f = 0; f < nf; ++f) {
        if (m->fdel[f] == 0.0) continue;
        const double sg = m->fdel[f] > 0.0 ? 1.0 : -1.0;
        const double nx = sg * m->fn[2 * f], ny = sg * m->fn[2 * f + 1];
        const double dx = sg * m->fd[2 * f], dy = sg * m->fd[2 * f + 1];
        cut_f.push_back(f);
        cut_s.push_back(sg > 0 ? 1 : -1);
        cut_i.push_back(sg > 0 ? m->fi[f] : m->fj[f]);
        cut_j.push_back(sg > 0 ? m->fj[f] : m->fi[f]);
        cut_K.push_back((nx * nx * Kx + ny * ny * Ky) / (nx * dx + ny * dy));
        cut_K.push_back(Kx * nx);
        cut_K.push_back(Ky * ny);
        cut_d.push_back(dx);
        cut_d.push_back(dy);
        cut_A.push_back(m->fA[f]);
        cut_An.push_back(m->fA[f] * nx);
        cut_An.push_back(m->fA[f] * ny);
    }
    // ---- device tables and buffers
    obte_status s = OBTE_OK;
    UGeomDev g{};
    g.ns = ns;
    g.nwalls = nw;
    g.n_sys = m->n_sys;
    g.n_dir = n_dir;
    g.n_mfp = n_mfp;
    g.grad_axis = ga;
    g.wmax = m->wmax;
    g.ncut = (int)cut_f.size();
    g.dT = m->dT;
    g.Lg = m->L[ga];
    g.Vbox = m->L[0] * m->L[1];
    g.Aperp = m->L[1 - ga];
    std::vector<double> ones(ns, 1.0);
#define UP(dst, v) \
    if ((s = upload(m, dst, v)) != OBTE_OK) { free_dev(m); return s; }
#define AL(dst, n) \
    if ((s = alloc(m, dst, n)) != OBTE_OK) { free_dev(m); return s; }
    UP((double**)&g.V, m->V);
    UP((double**)&g.mfp, m->mfp);
    UP((double**)&g.Dw, m->Dw);
    UP((double**)&g.S, m->S);
    UP((double**)&g.wout, m->wout);
    UP((int**)&g.wcell, m->wcell);
    UP((int**)&g.ord, ord);
    UP((int**)&g.lbase, lbase);
    UP((int**)&g.nlev, m->nlev);
    UP((int**)&g.lptr, lptr);
    UP((double**)&g.dout, dout);
    UP((int**)&g.inc, inc);
    UP((double**)&g.inv, inv);
    UP((int**)&g.nwrap, nwrap);
    UP((int**)&g.wup, wup);
    UP((double**)&g.wdel, wdel);
    UP((int**)&g.cut_i, cut_i);
    UP((int**)&g.cut_j, cut_j);
    UP((double**)&g.cut_An, cut_An);
    UP(&m->sigma1, ones);
    UP(&m->scell_d, m->scell);
    m->wcell_d = (int*)g.wcell;
    AL((double**)&g.sigma, ns);
    AL(&g.T_L, ns);
    AL(&g.T_w, nw);
    AL(&g.U, (size_t)m->n_sys * m->wmax);
    AL(&g.X, (size_t)m->n_sys * ns);
    AL(&g.ksys, m->n_sys);
    AL(&g.kfsys, m->n_sys);
    AL(&g.iters, m->n_sys);
    AL(&g.kap, 4);
    AL(&g.wres, m->n_sys);
    AL(&g.psg, (size_t)n_dir * ns);
    AL(&g.pb0, (size_t)n_dir * ns);
    AL(&g.pbw, (size_t)n_dir * ns);
    UFourierDev fdv{};
    fdv.ns = ns;
    fdv.nfaces = nf;
    fdv.grad_axis = ga;
    fdv.ncut = (int)cut_f.size();
    fdv.dT = m->dT;
    fdv.Lg = m->L[ga];
    fdv.Aperp = m->L[1 - ga];
    UP((int**)&fdv.nb_ptr, nb_ptr);
    UP((int**)&fdv.nb_j, nb_j);
    UP((double**)&fdv.nb_a, nb_a);
    UP((double**)&fdv.nb_del, nb_del);
    UP((double**)&fdv.nb_w, nb_w);
    UP((int**)&fdv.nb_f, nb_f);
    UP((int**)&fdv.fi, m->fi);
    UP((int**)&fdv.fj, m->fj);
    UP((double**)&fdv.fw, m->fw);
    UP((double**)&fdv.fc, fc);
    UP((double**)&fdv.P, P);
    UP((int**)&fdv.cut_f, cut_f);
    UP((int**)&fdv.cut_s, cut_s);
    UP((double**)&fdv.cut_K, cut_K);
    UP((double**)&fdv.cut_d, cut_d);
    UP((double**)&fdv.cut_A, cut_A);
    AL(&fdv.T, ns);
    AL(&fdv.r, ns);
    AL(&fdv.p, ns);
    AL(&fdv.q, ns);
    AL(&fdv.b, ns);
    AL(&fdv.g, 2 * (size_t)ns);
    AL(&fdv.bf, nf);
    AL(&fdv.out, 4);
    AL(&fdv.r1, ns);
    AL(&fdv.w0, ns);
    AL(&fdv.w1, ns);
    AL(&fdv.s0, ns);
    AL(&fdv.s1, ns);
    AL(&fdv.tp, ns);
    AL(&fdv.dg, ns);
    AL(&fdv.fpart, (size_t)UF_SLOTS * UF_MAXB);
    AL(&fdv.fsc, UF_SCALARS);
    if (hipHostMalloc((void**)&m->h_fsc, UF_SCALARS * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        m->h_fsc = nullptr;
        free_dev(m);
        return ufail(OBTE_ERR_HIP, "hipHostMalloc failed");
    }
    std::vector<UGeomDev> gv{g};
    std::vector<UFourierDev> fv{fdv};
    UP(&m->gd, gv);
    UP(&m->fdv, fv);
#undef UP
#undef AL
    m->gh = g;
    m->fh = fdv;
    m->has_material = true;
    return OBTE_OK;
}

obte_status obte_umesh_fourier(obte_umesh* m, double tol, int max_outer, double cg_tol, void* stream,
                               double* T_dev, double* kappa_F, int* outer_iters) {
    if (!m) return ufail(OBTE_ERR_ARG, "mesh is NULL");
    if (!m->has_material) return ufail(OBTE_ERR_STATE, "material not set");
    if (!(tol >= 0.0) || !(cg_tol > 0.0) || max_outer < 1) return ufail(OBTE_ERR_ARG, "need tol >= 0, cg_tol > 0, max_outer >= 1");
    hipStream_t st = (hipStream_t)stream;
    UHIP(hipMemsetAsync(m->fh.T, 0, sizeof(double) * m->ns, st));
    UHIP(hipMemsetAsync(m->fh.fsc, 0, sizeof(double) * UF_SCALARS, st));
    // conjugate gradients end in at most n steps in exact arithmetic; twice
    // that caps a solve whose tolerance sits below the rounding floor
    const int max_cg = 2 * m->ns + 50;
    constexpr int CG_CHUNK = 16;        // CG iterations queued per read of the stop flag (even)
    double* h = m->h_fsc;               // pinned: the loop scalars read back
    for (int outer = 1; outer <= max_outer; ++outer) {
        UHIP(ulaunch_fourier_start(m->fdv, m->ns, m->nf, st));
        for (int done = 0; !done;) {
            UHIP(ulaunch_fourier_cg(m->fdv, m->ns, CG_CHUNK, cg_tol, max_cg, st));
            UHIP(hipMemcpyAsync(h, m->fh.fsc, sizeof(double) * UF_SCALARS, hipMemcpyDeviceToHost, st));
            UHIP(hipStreamSynchronize(st));
            done = h[0] != 0.0;
        }
        UHIP(ulaunch_fourier_end(m->fdv, m->ns, tol, st));
        UHIP(hipMemcpyAsync(h, m->fh.fsc, sizeof(double) * UF_SCALARS, hipMemcpyDeviceToHost, st));
        UHIP(hipStreamSynchronize(st));
        if (h[5] != 0.0 || !std::isfinite(h[4])) break;
    }
    UHIP(ulaunch_fourier_kappa(m->fdv, m->ns, st));
    double out[4];
    UHIP(hipMemcpyAsync(out, m->fh.out, sizeof out, hipMemcpyDeviceToHost, st));
    if (T_dev) {
        UHIP(hipMemsetAsync(T_dev, 0, sizeof(double) * m->n_cells, st));
        hipLaunchKernelGGL(k_uscatter, dim3((m->ns + 255) / 256), dim3(256), 0, st, m->ns, m->scell_d, m->fh.T, T_dev, 0.0);
        UHIP(hipGetLastError());
    }
    UHIP(hipStreamSynchronize(st));
    if (kappa_F) *kappa_F = out[0];
    if (outer_iters) *outer_iters = (int)out[1];
    if (!std::isfinite(out[0])) return ufail(OBTE_ERR_NUMERIC, "non-finite heat-conduction solution");
    if ((int)out[1] >= max_outer && out[3] > tol)
        return ufail(OBTE_ERR_NOT_CONVERGED, "heat conduction: no convergence in %d outer iterations", max_outer);
    return OBTE_OK;
}

obte_status obte_umesh_solve(obte_umesh* m, const obte_solve_opts* o, const double* sigma_dev, void* stream,
                             double* T_L_dev, obte_stats* stats) {
    if (!m || !o) return ufail(OBTE_ERR_ARG, "NULL argument");
    if (!m->has_material) return ufail(OBTE_ERR_STATE, "material not set");
    if (o->precision != OBTE_FP64) return ufail(OBTE_ERR_ARG, "the unstructured path runs in FP64 (precision 0)");
    if (o->init != 0) return ufail(OBTE_ERR_ARG, "the unstructured path starts from the Fourier guess (init 0)");
    if (o->accel != 0) return ufail(OBTE_ERR_ARG, "the unstructured path runs Algorithm 1 (accel 0)");
    if (o->max_outer < 1 || !(o->outer_tol >= 0.0) || !(o->inner_tol > 0.0) || o->max_inner < 1 ||
        !(o->inner_rtol >= 0.0 && o->inner_rtol < 1.0) ||
        !(o->fourier_tol >= 0.0) || o->max_fourier < 1)
        return ufail(OBTE_ERR_ARG, "invalid tolerances or iteration caps");
    hipStream_t st = (hipStream_t)stream;
    const int ns = m->ns, nw = m->nw;
    UGeomDev& g = m->gh;
    // sigma over the solid cells
    if (sigma_dev) {
        hipLaunchKernelGGL(k_ugather, dim3((ns + 255) / 256), dim3(256), 0, st, ns, m->scell_d, sigma_dev, (double*)g.sigma);
        UHIP(hipGetLastError());
    } else {
        UHIP(hipMemcpyAsync((double*)g.sigma, m->sigma1, sizeof(double) * ns, hipMemcpyDeviceToDevice, st));
    }
    // first guess: T_L = T_F, T_w = T_F of the wall's cell
    double kF = 0.0;
    int fit = 0;
    // each conjugate-gradient solve to a hundredth of the outer tolerance
    const double cg_tol = std::max(1e-14, 1e-2 * o->fourier_tol);
    obte_status sf = obte_umesh_fourier(m, o->fourier_tol, o->max_fourier, cg_tol, stream, nullptr, &kF, &fit);
    if (sf != OBTE_OK && sf != OBTE_ERR_NOT_CONVERGED) return sf;
    UHIP(hipMemcpyAsync(g.T_L, m->fh.T, sizeof(double) * ns, hipMemcpyDeviceToDevice, st));
    if (nw > 0) {
        hipLaunchKernelGGL(k_ugather, dim3((nw + 255) / 256), dim3(256), 0, st, nw, m->wcell_d, m->fh.T, g.T_w);
        UHIP(hipGetLastError());
    }
    UHIP(hipMemsetAsync(g.U, 0, sizeof(double) * (size_t)m->n_sys * m->wmax, st));
    UHIP(hipMemsetAsync(g.iters, 0, sizeof(long long) * m->n_sys, st));
    int wpl = 1;
    while (wpl * 64 < m->wmax) wpl *= 2;
    const size_t lds = sizeof(double) * ((size_t)ns + m->wmax);
    std::vector<double> hist;
    double kap[4] = {0, 0, 0, 0};
    const double wrap_tol = o->wrap_tol > 0.0 ? o->wrap_tol : std::max(o->inner_tol, 0.2 * o->outer_tol);
    bool converged = false;
    int passes = 0;
    for (passes = 1; passes <= o->max_outer; ++passes) {
        UHIP(ulaunch_pass(m->gd, m->n_sys, m->n_dir * ns, wpl, lds, o->inner_tol, o->inner_rtol, o->max_inner, st));
        UHIP(ulaunch_reduce(m->gd, ns, nw, st));
        UHIP(hipMemcpyAsync(kap, g.kap, sizeof kap, hipMemcpyDeviceToHost, st));
        UHIP(hipStreamSynchronize(st));
        if (!std::isfinite(kap[0])) return ufail(OBTE_ERR_NUMERIC, "non-finite kappa in pass %d", passes);
        hist.push_back(kap[0]);
        // Algorithm 1's test, and every wrap solved to wrap_tol (a forcing
        // term leaves part of the periodic coupling to later passes)
        if (hist.size() >= 2 && std::fabs(kap[0] - hist[hist.size() - 2]) <= o->outer_tol * std::fabs(kap[0]) &&
            kap[2] <= wrap_tol) {
            converged = true;
            break;
        }
    }
    if (passes > o->max_outer) passes = o->max_outer;
    if (T_L_dev) {
        std::vector<double> tl(ns);
        UHIP(hipMemcpy(tl.data(), g.T_L, sizeof(double) * ns, hipMemcpyDeviceToHost));
        double mean = 0.0;
        for (double v : tl) mean += v;
        mean /= ns;
        UHIP(hipMemsetAsync(T_L_dev, 0, sizeof(double) * m->n_cells, st));
        hipLaunchKernelGGL(k_uscatter, dim3((ns + 255) / 256), dim3(256), 0, st, ns, m->scell_d, g.T_L, T_L_dev, mean);
        UHIP(hipGetLastError());
        UHIP(hipStreamSynchronize(st));
    }
    if (stats) {
        std::vector<long long> its(m->n_sys);
        UHIP(hipMemcpy(its.data(), g.iters, sizeof(long long) * m->n_sys, hipMemcpyDeviceToHost));
        obte_stats S{};
        S.outer_iters = passes;
        for (long long v : its) S.inner_iters += v;
        S.fourier_iters = fit;
        S.kappa = kap[0];
        S.kappa_face = kap[1];
        S.kappa_fourier = kF;
        S.wrap_residual = kap[2];
        S.last_rel_change = hist.size() >= 2 ? std::fabs(hist.back() - hist[hist.size() - 2]) / std::fabs(hist.back()) : 0.0;
        S.status = converged ? OBTE_OK : OBTE_ERR_NOT_CONVERGED;
        *stats = S;
    }
    if (!converged) return ufail(OBTE_ERR_NOT_CONVERGED, "no convergence in %d passes", o->max_outer);
    return OBTE_OK;
}

void obte_umesh_destroy(obte_umesh* m) {
    if (!m) return;
    free_dev(m);
    delete m;
}

int obte_umesh_n_solid(const obte_umesh* m) { return m ? m->ns : -1; }
int obte_umesh_n_faces(const obte_umesh* m) { return m ? m->nf : -1; }
int obte_umesh_n_walls(const obte_umesh* m) { return m ? m->nw : -1; }
int obte_umesh_n_levels(const obte_umesh* m, int l) {
    if (!m || !m->has_material || l < 0 || l >= m->n_dir) return -1;
    return m->nlev[l];
}

}  // extern "C"
