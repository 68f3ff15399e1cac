// C ABI of libqh (declarations and contracts in include/qh.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include <random>

#include "qh_internal.h"
#include "qh_spmv.h"

int qh_fail(qh_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

// ----------------------------------------------------------------------------- timing
int qh_tbeg(qh_ctx *c) {
    if (!c->timing) return -1;
    int slot = (int)c->pending.size() * 2;
    while ((int)c->ev_pool.size() < slot + 2) {
        // timing only, read after the stream is synchronised: no system-scope fence on record
        // (the fence writes back and invalidates the caches, which would slow the next kernel)
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
        c->ev_pool.push_back(e);
    }
    (void)hipEventRecord(c->ev_pool[slot], c->stream);
    return slot;
}

void qh_tend(qh_ctx *c, int slot, int kernel) {
    if (slot < 0) return;
    (void)hipEventRecord(c->ev_pool[slot + 1], c->stream);
    c->pending.push_back({slot, kernel});
}

void qh_tflush(qh_ctx *c) {
    if (c->pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto &p : c->pending) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, c->ev_pool[p.slot], c->ev_pool[p.slot + 1]);
        c->t_ms[p.kernel] += ms;
        c->t_cnt[p.kernel] += 1;
    }
    c->pending.clear();
}

namespace {

template <class T>
int upload(qh_ctx *c, T **dst, const T *src, size_t n) {
    int rc = qh_alloc(c, dst, n);
    if (rc) return rc;
    QH_HIP(c, hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return QH_OK;
}

int upload_csr(qh_ctx *c, DevCsr &d, const HostCsr &h, bool two) {
    d.n = (int32_t)h.nrow;
    d.nnz = (int64_t)h.col.size();
    int rc;
    if ((rc = upload(c, &d.ptr, h.ptr.data(), h.ptr.size()))) return rc;
    if ((rc = upload(c, &d.col, h.col.data(), h.col.size()))) return rc;
    if ((rc = upload(c, two ? &d.val2 : &d.val, h.val.data(), h.val.size()))) return rc;
    std::vector<int2> tiles;
    if (!qh_make_tiles(h.ptr.data(), d.n, tiles)) return qh_fail(c, QH_EINVAL, "matrix row longer than a product tile");
    d.ntiles = (int32_t)tiles.size() - 1;
    if ((rc = upload(c, &d.tiles, tiles.data(), tiles.size()))) return rc;
    std::vector<int4> tbase;
    std::vector<uint16_t> col16;
    d.nnz_c16 = qh_compact_cols(h.col.data(), tiles, tbase, col16);
    if ((rc = upload(c, &d.tbase, tbase.data(), tbase.size()))) return rc;
    if ((rc = upload(c, &d.col16, col16.data(), col16.size()))) return rc;
    return QH_OK;
}

void free_all(qh_ctx *c) {
    for (void *p : c->allocations) (void)hipFree(p);
    c->allocations.clear();
}

int sync(qh_ctx *c) {
    QH_HIP(c, hipStreamSynchronize(c->stream));
    return QH_OK;
}

// Assemble on the host and upload the matrices once mesh and physics are both known.
int ensure_assembled(qh_ctx *c) {
    if (!c->have_mesh || !c->have_phys) return QH_OK;
    int rc;
    if (c->host_only) {
        if (!c->assembled) qh_assemble(c->hm, c->phys.eps0, c->phys.mu0, c->hA, c->hCMb, c->hGtM, c->hK);
        c->assembled = true;
        return QH_OK;
    }
    if (!c->assembled) {
        qh_assemble(c->hm, c->phys.eps0, c->phys.mu0, c->hA, c->hCMb, c->hGtM, c->hK);
        // A: val2 = [*eps], A_S = S, val = [*eps] + tau S (device)
        if ((rc = upload_csr(c, c->A, c->hA, true))) return rc;
        if ((rc = upload(c, &c->A_S, c->hA.val2.data(), c->hA.val2.size()))) return rc;
        if ((rc = qh_alloc(c, &c->A.val, c->A.nnz))) return rc;
        if ((rc = qh_alloc(c, &c->A_rhs, c->A.nnz))) return rc;
        if ((rc = upload_csr(c, c->CMb, c->hCMb, false))) return rc;
        if ((rc = upload_csr(c, c->GtM, c->hGtM, false))) return rc;
        if ((rc = upload_csr(c, c->K, c->hK, false))) return rc;
        if ((rc = qh_cg_alloc(c, c->cge, c->A.n))) return rc;
        if ((rc = qh_cg_alloc(c, c->cgn, c->K.n))) return rc;
        if ((rc = qh_alloc(c, &c->e_old, std::max<int64_t>(1, c->A.n)))) return rc;
        if ((rc = qh_alloc(c, &c->e_prev, std::max<int64_t>(1, c->A.n)))) return rc;
        if ((rc = qh_alloc(c, &c->g_prev, c->hm.Ne))) return rc;
        if ((rc = qh_alloc(c, &c->e_star, std::max<int64_t>(1, c->A.n)))) return rc;
        if ((rc = qh_alloc(c, &c->rho, std::max<int64_t>(1, c->K.n)))) return rc;
        QH_HIP(c, launch_diag_inv(c, c->K, c->cgn.dinv));
        c->assembled = true;
        c->tau_assembled = -1.0;
        // cge.x mirrors e on the interior edges
        std::vector<double> e_h(c->hm.Ne, 0.0), x(c->A.n);
        QH_HIP(c, hipMemcpyAsync(e_h.data(), c->e, sizeof(double) * c->hm.Ne, hipMemcpyDeviceToHost, c->stream));
        QH_HIP(c, hipStreamSynchronize(c->stream));
        for (int32_t i = 0; i < c->A.n; ++i) x[i] = e_h[c->hm.int_edges[i]];
        QH_HIP(c, hipMemcpyAsync(c->cge.x, x.data(), sizeof(double) * x.size(), hipMemcpyHostToDevice, c->stream));
    }
    double tau = 0.25 * c->phys.dt * c->phys.dt;
    if (tau != c->tau_assembled) {
        QH_HIP(c, launch_assemble_A(c, tau));
        QH_HIP(c, launch_diag_inv(c, c->A, c->cge.dinv));
        c->tau_assembled = tau;
    }
    return sync(c);
}

int check_divb_host(qh_ctx *c, const int64_t *b) {
    const HostMesh &m = c->hm;
    for (int64_t t = 0; t < m.Nt; ++t) {
        const int32_t *f = &m.tf[4 * t];
        int64_t s = b[f[0]] - b[f[1]] + b[f[2]] - b[f[3]];
        if (s != 0) return qh_fail(c, QH_EINVAL, "D b != 0 in tet " + std::to_string(t));
    }
    return QH_OK;
}

int set_fields(qh_ctx *c, const double *e, const int64_t *b) {
    const HostMesh &m = c->hm;
    int rc = check_divb_host(c, b);
    if (rc) return rc;
    std::vector<double> eh(e, e + m.Ne);
    for (int64_t i = 0; i < m.Ne; ++i)
        if (m.wall_edge[i] && !m.neumann) eh[i] = 0.0;
    QH_HIP(c, hipMemcpyAsync(c->e, eh.data(), sizeof(double) * m.Ne, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, hipMemcpyAsync(c->b, b, sizeof(int64_t) * m.Nf, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, hipMemsetAsync(c->divb0, 0, sizeof(int64_t) * m.Nt, c->stream));
    if (c->assembled) {
        std::vector<double> x(m.int_edges.size());
        for (size_t i = 0; i < x.size(); ++i) x[i] = eh[m.int_edges[i]];
        QH_HIP(c, hipMemcpyAsync(c->cge.x, x.data(), sizeof(double) * x.size(), hipMemcpyHostToDevice, c->stream));
    }
    c->have_fields = true;
    c->fields_dirty = true;
    c->wave_hist = false;
    if (c->dbnd) QH_HIP(c, hipMemsetAsync(c->dbnd, 0, sizeof(double) * m.Nn, c->stream));
    return sync(c);
}

// Seeds of point location: a uniform grid of about Nt/2 buckets over the bounding box; each
// bucket holds a tet whose centroid lies in it, or (buckets without one) a neighbour's.
int build_locator(qh_ctx *c) {
    const HostMesh &m = c->hm;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < m.Nn; ++v)
        for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], m.xyz[3 * v + d]), hi[d] = std::max(hi[d], m.xyz[3 * v + d]);
    const double target = std::max<double>(1.0, std::min<double>(0.5 * (double)m.Nt, 16777216.0));
    const double ext[3] = {std::max(hi[0] - lo[0], 1e-300), std::max(hi[1] - lo[1], 1e-300), std::max(hi[2] - lo[2], 1e-300)};
    const double h = std::cbrt(ext[0] * ext[1] * ext[2] / target);
    int64_t total = 1;
    for (int d = 0; d < 3; ++d) {
        c->loc_n[d] = (int32_t)std::max<double>(1.0, std::min<double>(4096.0, std::ceil(ext[d] / h)));
        c->loc_lo[d] = (float)lo[d];
        c->loc_inv[d] = (float)(c->loc_n[d] / ext[d]);
        total *= c->loc_n[d];
    }
    const int nx = c->loc_n[0], ny = c->loc_n[1], nz = c->loc_n[2];
    std::vector<int32_t> seed(total, -1);
    auto bucket = [&](const double *p) {
        int b[3];
        for (int d = 0; d < 3; ++d)
            b[d] = std::min(std::max((int)((p[d] - lo[d]) * (c->loc_n[d] / ext[d])), 0), c->loc_n[d] - 1);
        return ((int64_t)b[2] * ny + b[1]) * nx + b[0];
    };
    std::vector<int64_t> queue;
    for (int64_t t = 0; t < m.Nt; ++t) {
        const int64_t b = bucket(&m.cen[3 * t]);
        if (seed[b] < 0) seed[b] = (int32_t)t, queue.push_back(b);
    }
    for (size_t q = 0; q < queue.size(); ++q) {  // breadth first into the empty buckets
        const int64_t b = queue[q];
        const int64_t bx = b % nx, by = (b / nx) % ny, bz = b / ((int64_t)nx * ny);
        const int64_t nbs[6][3] = {{bx - 1, by, bz}, {bx + 1, by, bz}, {bx, by - 1, bz}, {bx, by + 1, bz}, {bx, by, bz - 1}, {bx, by, bz + 1}};
        for (auto &u : nbs) {
            if (u[0] < 0 || u[0] >= nx || u[1] < 0 || u[1] >= ny || u[2] < 0 || u[2] >= nz) continue;
            const int64_t w = (u[2] * ny + u[1]) * nx + u[0];
            if (seed[w] < 0) seed[w] = seed[b], queue.push_back(w);
        }
    }
    return upload(c, &c->loc_seed, seed.data(), seed.size());
}

// Locates n particles of a species from index `first` on the device (their positions are in
// place) into s.tet; QH_EINVAL naming the first point outside the mesh.
int locate_species(qh_ctx *c, Species &s, int64_t first, int64_t n) {
    QH_HIP(c, launch_locate(c, n, s.x + first, s.y + first, s.zz + first, s.tet + first));
    std::vector<int32_t> t(n);
    QH_HIP(c, hipMemcpyAsync(t.data(), s.tet + first, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; ++i)
        if (t[i] < 0) return qh_fail(c, QH_EINVAL, "particle " + std::to_string(i) + " lies outside the mesh");
    return QH_OK;
}

int recompute_charge(qh_ctx *c) {
    QH_HIP(c, hipMemsetAsync(c->Q, 0, sizeof(int64_t) * c->hm.Nn, c->stream));
    for (auto &s : c->species) QH_HIP(c, launch_charge_deposit(c, s));
    QH_HIP(c, hipMemcpyAsync(c->Q_old, c->Q, sizeof(int64_t) * c->hm.Nn, hipMemcpyDeviceToDevice, c->stream));
    return sync(c);
}

}  // namespace

extern "C" {

int qh_create(qh_ctx **out, int device, void *stream) {
    if (!out) return QH_EINVAL;
    *out = nullptr;
    if (device < 0) {
        qh_ctx *c = new qh_ctx();
        c->host_only = true;
        *out = c;
        return QH_OK;
    }
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return QH_EHIP;
    if (device < 0 || device >= n) return QH_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return QH_EHIP;
    qh_ctx *c = new qh_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    unsigned long long *cnt = nullptr;
    if (qh_alloc(c, &cnt, 4 * QH_COUNTER_SLOTS + QH_CNT_ALL) != QH_OK) {
        delete c;
        return QH_ENOMEM;
    }
    c->counters = cnt;
    if (qh_alloc(c, &c->scratch_d, 16) != QH_OK) {
        free_all(c);
        delete c;
        return QH_ENOMEM;
    }
    // the address of this device's static scratch array (qh_deposit_noalloc); a failure is kept
    // in the context's message and reported by that call
    (void)qh_static_scratch_init(c);
    *out = c;
    return QH_OK;
}

void qh_destroy(qh_ctx *c) {
    if (!c) return;
    if (c->host_only) {
        delete c;
        return;
    }
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    free_all(c);
    delete c;
}

const char *qh_last_error(const qh_ctx *c) { return c ? c->err.c_str() : "null context"; }

int qh_set_boundary(qh_ctx *c, int32_t mode) {
    if (!c) return QH_EINVAL;
    if (mode != QH_BC_PEC && mode != QH_BC_NEUMANN) return qh_fail(c, QH_EINVAL, "boundary mode");
    if (c->have_mesh) return qh_fail(c, QH_ESTATE, "the boundary condition is set before the mesh");
    c->bc = mode;
    return QH_OK;
}

int qh_set_plane_wave(qh_ctx *c, double E0, double f0, double bandwidth, double t0) {
    if (!c) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh || !c->have_phys) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    if (c->bc != QH_BC_NEUMANN)
        return qh_fail(c, QH_ESTATE, "a plane wave enters through a natural boundary (QH_BC_NEUMANN)");
    if (E0 == 0.0) {
        c->pw_on = false;
        return QH_OK;
    }
    if (!std::isfinite(E0) || !std::isfinite(t0) || !(f0 > 0) || !(bandwidth > 0))
        return qh_fail(c, QH_EINVAL, "plane wave: E0, t0 finite, f0 and bandwidth positive");
    const HostMesh &m = c->hm;
    // Dunavant's degree-4 rule on a triangle (barycentric points, weights summing to 1)
    static const double kP[6][3] = {{0.108103018168070, 0.445948490915965, 0.445948490915965},
                                    {0.445948490915965, 0.108103018168070, 0.445948490915965},
                                    {0.445948490915965, 0.445948490915965, 0.108103018168070},
                                    {0.816847572980459, 0.091576213509771, 0.091576213509771},
                                    {0.091576213509771, 0.816847572980459, 0.091576213509771},
                                    {0.091576213509771, 0.091576213509771, 0.816847572980459}};
    static const double kW[6] = {0.223381589678011, 0.223381589678011, 0.223381589678011,
                                 0.109951743655322, 0.109951743655322, 0.109951743655322};
    static const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    struct Pt {
        int32_t e;
        double coef, x;
    };
    std::vector<Pt> pts;
    for (int64_t t = 0; t < m.Nt; ++t)
        for (int k = 0; k < 4; ++k) {
            if (!m.wall_face[m.tf[4 * t + k]]) continue;
            int v[3], nv = 0;
            for (int i = 0; i < 4; ++i)
                if (i != k) v[nv++] = i;
            const double *g = &m.grad[12 * t];
            const double gn = std::sqrt(g[3 * k] * g[3 * k] + g[3 * k + 1] * g[3 * k + 1] + g[3 * k + 2] * g[3 * k + 2]);
            const double n[3] = {-g[3 * k] / gn, -g[3 * k + 1] / gn, -g[3 * k + 2] / gn};  // outward
            const double nxy[3] = {-n[2], 0.0, n[0]};                                           // n x y-hat
            const double *P[3];
            for (int j = 0; j < 3; ++j) P[j] = &m.xyz[3 * (int64_t)m.tn[4 * t + v[j]]];
            const double u[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
            const double w[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
            const double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
            const double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            for (int q = 0; q < 6; ++q) {
                double lam[4] = {0.0, 0.0, 0.0, 0.0};
                double x = 0.0;
                for (int j = 0; j < 3; ++j) {
                    lam[v[j]] = kP[q][j];
                    x += kP[q][j] * P[j][0];
                }
                for (int j = 0; j < 6; ++j) {
                    const int a = LE[j][0], b = LE[j][1];
                    if (a == k || b == k) continue;  // the edge is not on this face
                    double dotv = 0.0;                // W1_ab = lam_a grad lam_b - lam_b grad lam_a
                    for (int d = 0; d < 3; ++d) dotv += (lam[a] * g[3 * b + d] - lam[b] * g[3 * a + d]) * nxy[d];
                    pts.push_back({m.int_edge_of[m.te[6 * t + j]], kW[q] * area * dotv, x});
                }
            }
        }
    std::stable_sort(pts.begin(), pts.end(), [](const Pt &p, const Pt &q) { return p.e < q.e; });
    std::vector<int32_t> ptr(1, 0), edge;
    std::vector<double> coef(pts.size()), xq(pts.size());
    for (size_t k = 0; k < pts.size(); ++k) {
        if (k == 0 || pts[k].e != pts[k - 1].e) {
            if (k) ptr.push_back((int32_t)k);
            edge.push_back(pts[k].e);
        }
        coef[k] = pts[k].coef;
        xq[k] = pts[k].x;
    }
    ptr.push_back((int32_t)pts.size());
    const int32_t nb = (int32_t)edge.size();
    // the incident field depends on x only: s' is evaluated once per distinct x of the points
    std::vector<double> xs(xq);
    std::sort(xs.begin(), xs.end());
    xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
    std::vector<int32_t> xi(xq.size());
    for (size_t k = 0; k < xq.size(); ++k) xi[k] = (int32_t)(std::lower_bound(xs.begin(), xs.end(), xq[k]) - xs.begin());
    // boundary nodes: per node, its boundary edges with the sign of G (head +1, tail -1)
    std::vector<std::vector<int32_t>> lists(m.Nn);
    for (int32_t i = 0; i < nb; ++i) {
        const int32_t ge = m.int_edges[edge[i]];
        lists[m.edges[2 * ge + 1]].push_back(i << 1);
        lists[m.edges[2 * ge]].push_back(i << 1 | 1);
    }
    std::vector<int32_t> nptr(1, 0), nlist, node;
    for (int64_t v = 0; v < m.Nn; ++v)
        if (!lists[v].empty()) {
            node.push_back((int32_t)v);
            nlist.insert(nlist.end(), lists[v].begin(), lists[v].end());
            nptr.push_back((int32_t)nlist.size());
        }
    QH_HIP(c, hipStreamSynchronize(c->stream));  // a second call replaces the first one's tables
    qh_release(c, c->pw_ptr), qh_release(c, c->pw_edge), qh_release(c, c->pw_coef), qh_release(c, c->pw_xi);
    qh_release(c, c->pw_xs), qh_release(c, c->pw_tab);
    qh_release(c, c->pw_nptr), qh_release(c, c->pw_nlist), qh_release(c, c->pw_node);
    qh_release(c, c->pw_hsum);
    c->pw_on = false;
    int rc;
    if ((rc = upload(c, &c->pw_ptr, ptr.data(), ptr.size())) || (rc = upload(c, &c->pw_edge, edge.data(), edge.size())) ||
        (rc = upload(c, &c->pw_coef, coef.data(), coef.size())) || (rc = upload(c, &c->pw_xi, xi.data(), xi.size())) ||
        (rc = upload(c, &c->pw_xs, xs.data(), xs.size())) || (rc = qh_alloc(c, &c->pw_tab, 3 * xs.size())) ||
        (rc = upload(c, &c->pw_nptr, nptr.data(), nptr.size())) ||
        (rc = upload(c, &c->pw_nlist, nlist.data(), nlist.size())) || (rc = upload(c, &c->pw_node, node.data(), node.size())) ||
        (rc = qh_alloc(c, &c->pw_hsum, std::max<int32_t>(1, nb))))
        return rc;
    if (!c->dbnd) {  // the flux already brought in stays in the Gauss-law target
        if ((rc = qh_alloc(c, &c->dbnd, m.Nn))) return rc;
        QH_HIP(c, hipMemsetAsync(c->dbnd, 0, sizeof(double) * m.Nn, c->stream));
    }
    c->pw_nb = nb;
    c->pw_nn = (int32_t)node.size();
    c->pw_nu = (int32_t)xs.size();
    c->pw_amp = E0 / std::sqrt(c->phys.mu0 / c->phys.eps0);
    c->pw_c = 1.0 / std::sqrt(c->phys.eps0 * c->phys.mu0);
    c->pw_f0 = f0;
    c->pw_sig = 1.0 / (2.0 * M_PI * bandwidth);
    c->pw_t0 = t0;
    c->pw_on = true;
    return sync(c);
}

int qh_mesh_upload(qh_ctx *c, int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tet_nodes) {
    if (!c) return QH_EINVAL;
    if (c->have_mesh) return qh_fail(c, QH_ESTATE, "mesh already uploaded (one mesh per context)");
    c->hm.neumann = c->bc == QH_BC_NEUMANN;
    std::string msg = qh_build_mesh(c->hm, n_nodes, xyz, n_tets, tet_nodes);
    if (!msg.empty()) return qh_fail(c, QH_EINVAL, msg);
    HostMesh &m = c->hm;
    int rc;
    if (c->host_only) {
        c->have_mesh = true;
        return ensure_assembled(c);
    }
    // FP32 geometry records: (grad l_i, centroid component)
    std::vector<float4> geo(3 * m.Nt);
    for (int64_t t = 0; t < m.Nt; ++t)
        for (int i = 1; i <= 3; ++i) {
            const double *g = &m.grad[12 * t + 3 * i];
            geo[3 * t + i - 1] = make_float4((float)g[0], (float)g[1], (float)g[2], (float)m.cen[3 * t + i - 1]);
        }
    std::vector<int32_t> te8(8 * m.Nt, -1);
    for (int64_t t = 0; t < m.Nt; ++t)
        for (int k = 0; k < 6; ++k) te8[8 * t + k] = m.te[6 * t + k];
    if ((rc = upload(c, &c->geo, geo.data(), geo.size()))) return rc;
    if ((rc = upload(c, &c->tnodes, (const int4 *)m.tn.data(), m.Nt))) return rc;
    if ((rc = upload(c, &c->tedges, te8.data(), te8.size()))) return rc;
    if ((rc = upload(c, &c->tnbr, (const int4 *)m.nbr.data(), m.Nt))) return rc;
    if ((rc = upload(c, &c->wall_node_d, m.wall_node.data(), m.wall_node.size()))) return rc;
    if ((rc = build_locator(c))) return rc;
    if ((rc = upload(c, &c->tfaces, m.tf.data(), m.tf.size()))) return rc;
    if ((rc = upload(c, &c->tsign, m.tsign.data(), m.tsign.size()))) return rc;
    if ((rc = upload(c, &c->face_edges, m.face_edges.data(), m.face_edges.size()))) return rc;
    if ((rc = upload(c, &c->int_edges, m.int_edges.data(), std::max<size_t>(1, m.int_edges.size())))) return rc;
    if ((rc = upload(c, &c->int_nodes, m.int_nodes.data(), std::max<size_t>(1, m.int_nodes.size())))) return rc;
    if ((rc = upload(c, &c->int_node_of, m.int_node_of.data(), m.int_node_of.size()))) return rc;
    if ((rc = upload(c, &c->edge_nodes, m.edges.data(), m.edges.size()))) return rc;
    if ((rc = upload(c, &c->n2e_ptr, m.n2e_ptr.data(), m.n2e_ptr.size()))) return rc;
    if ((rc = upload(c, &c->n2e, m.n2e.data(), m.n2e.size()))) return rc;
    if ((rc = upload(c, &c->e2t_ptr, m.e2t_ptr.data(), m.e2t_ptr.size()))) return rc;
    if ((rc = upload(c, &c->e2t, m.e2t.data(), m.e2t.size()))) return rc;
    if ((rc = upload(c, &c->n2t_ptr, m.n2t_ptr.data(), m.n2t_ptr.size()))) return rc;
    if ((rc = upload(c, &c->n2t, m.n2t.data(), m.n2t.size()))) return rc;
    if ((rc = qh_alloc(c, &c->acc_tet, 10 * m.Nt))) return rc;
    {
        const int64_t nmail = (m.Nt + kMailTets - 1) / kMailTets;
        if ((rc = qh_alloc(c, &c->mail_cnt, nmail)) || (rc = qh_alloc(c, &c->mail, nmail * kMailCap * kMailWords))) return rc;
    }
    if ((rc = qh_alloc(c, &c->frec, 3 * m.Nt))) return rc;
    if ((rc = qh_alloc(c, &c->e, m.Ne)) || (rc = qh_alloc(c, &c->b, m.Nf)) || (rc = qh_alloc(c, &c->g, m.Ne)) ||
        (rc = qh_alloc(c, &c->Q, m.Nn)) || (rc = qh_alloc(c, &c->Q_old, m.Nn)) || (rc = qh_alloc(c, &c->Q_bg, m.Nn)) ||
        (rc = qh_alloc(c, &c->divb0, m.Nt)) || (rc = qh_alloc(c, &c->u_int, m.Ne)) ||
        (rc = qh_alloc(c, &c->hist, m.Nt + 1)) || (rc = qh_alloc(c, &c->cursor, m.Nt + 1)) ||
        (rc = qh_alloc(c, &c->scan_tmp, (m.Nt + 1023) / 1024 + 1)))
        return rc;
    QH_HIP(c, hipMemsetAsync(c->e, 0, sizeof(double) * m.Ne, c->stream));
    QH_HIP(c, hipMemsetAsync(c->b, 0, sizeof(int64_t) * m.Nf, c->stream));
    QH_HIP(c, hipMemsetAsync(c->g, 0, sizeof(int64_t) * m.Ne, c->stream));
    QH_HIP(c, hipMemsetAsync(c->Q, 0, sizeof(int64_t) * m.Nn, c->stream));
    QH_HIP(c, hipMemsetAsync(c->Q_old, 0, sizeof(int64_t) * m.Nn, c->stream));
    QH_HIP(c, hipMemsetAsync(c->Q_bg, 0, sizeof(int64_t) * m.Nn, c->stream));
    QH_HIP(c, hipMemsetAsync(c->divb0, 0, sizeof(int64_t) * m.Nt, c->stream));
    QH_HIP(c, hipMemsetAsync(c->u_int, 0, sizeof(int64_t) * m.Ne, c->stream));
    c->have_mesh = true;
    if ((rc = sync(c))) return rc;
    return ensure_assembled(c);
}

int qh_mesh_info(const qh_ctx *c, qh_mesh_info_t *out) {
    if (!c || !out) return QH_EINVAL;
    if (!c->have_mesh) return QH_ESTATE;
    const HostMesh &m = c->hm;
    out->n_nodes = m.Nn;
    out->n_edges = m.Ne;
    out->n_faces = m.Nf;
    out->n_tets = m.Nt;
    out->n_int_nodes = (int64_t)m.int_nodes.size();
    out->n_int_edges = (int64_t)m.int_edges.size();
    out->nnz_edge = (int64_t)c->hA.col.size();
    out->nnz_node = (int64_t)c->hK.col.size();
    out->nnz_edge_c16 = c->A.nnz_c16;
    out->nnz_factor = c->lp.built ? c->lp.nnz : 0;
    out->nnz_factor_c16 = c->lp.built ? c->lp.nnz_c16 : 0;
    qh_ctx *mc = const_cast<qh_ctx *>(c);
    if (mc->cfl_lambda < 0.0) mc->cfl_lambda = qh_cfl_lambda_geo(m);
    const double eps0 = c->have_phys ? c->phys.eps0 : 8.8541878128e-12, mu0 = c->have_phys ? c->phys.mu0 : 1.25663706212e-6;
    out->dt_cfl = mc->cfl_lambda > 0.0 ? 2.0 * std::sqrt(eps0 * mu0 / mc->cfl_lambda) : 0.0;
    return QH_OK;
}

int qh_mesh_topology(const qh_ctx *c, int32_t *edges, int32_t *faces, int32_t *tet_nodes, int32_t *tet_edges,
                     int32_t *tet_faces, int32_t *tet_nbr, uint8_t *wall_edge, uint8_t *wall_node) {
    if (!c) return QH_EINVAL;
    if (!c->have_mesh) return QH_ESTATE;
    const HostMesh &m = c->hm;
    if (edges) std::copy(m.edges.begin(), m.edges.end(), edges);
    if (faces) std::copy(m.faces.begin(), m.faces.end(), faces);
    if (tet_nodes) std::copy(m.tn.begin(), m.tn.end(), tet_nodes);
    if (tet_edges) std::copy(m.te.begin(), m.te.end(), tet_edges);
    if (tet_faces) std::copy(m.tf.begin(), m.tf.end(), tet_faces);
    if (tet_nbr) std::copy(m.nbr.begin(), m.nbr.end(), tet_nbr);
    if (wall_edge) std::copy(m.wall_edge.begin(), m.wall_edge.end(), wall_edge);
    if (wall_node) std::copy(m.wall_node.begin(), m.wall_node.end(), wall_node);
    return QH_OK;
}

int qh_set_physics(qh_ctx *c, const qh_phys_t *p) {
    if (!c || !p) return QH_EINVAL;
    if (!(p->eps0 > 0) || !(p->mu0 > 0) || !(p->dt > 0) || !(p->u_q > 0) || !(p->u_b > 0))
        return qh_fail(c, QH_EINVAL, "physics: eps0, mu0, dt, u_q, u_b must be positive");
    if (c->have_phys && (p->eps0 != c->phys.eps0 || p->mu0 != c->phys.mu0) && c->assembled)
        return qh_fail(c, QH_ESTATE, "eps0/mu0 cannot change after assembly");
    bool ub_changed = c->have_phys && p->u_b != c->phys.u_b;
    if (ub_changed && c->have_fields) return qh_fail(c, QH_ESTATE, "u_b cannot change once fields are set");
    c->phys = *p;
    c->have_phys = true;
    c->fields_dirty = true;
    c->wave_hist = false;
    return ensure_assembled(c);
}

int qh_fields_upload(qh_ctx *c, const double *e, const int64_t *b) {
    if (!c || !e || !b) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    return set_fields(c, e, b);
}

int qh_fields_download(const qh_ctx *cc, double *e, int64_t *b) {
    qh_ctx *c = const_cast<qh_ctx *>(cc);
    if (!c) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (e) QH_HIP(c, hipMemcpyAsync(e, c->e, sizeof(double) * c->hm.Ne, hipMemcpyDeviceToHost, c->stream));
    if (b) QH_HIP(c, hipMemcpyAsync(b, c->b, sizeof(int64_t) * c->hm.Nf, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int qh_fields_init_synthetic(qh_ctx *c, const double *we, const double *wa, double sigma_e, double bz,
                             double sigma_b) {
    if (!c || !we || !wa) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh || !c->have_phys) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    const HostMesh &m = c->hm;
    std::vector<double> e(m.Ne, 0.0);
    std::vector<int64_t> a(m.Ne), b(m.Nf);
    const double k = sigma_b / (2.0 * std::sqrt(3.0));
    for (int64_t i = 0; i < m.Ne; ++i) {
        const double *pa = &m.xyz[3 * (int64_t)m.edges[2 * i]], *pb = &m.xyz[3 * (int64_t)m.edges[2 * i + 1]];
        double d[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
        double ell = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (m.neumann || !m.wall_edge[i]) e[i] = ell * sigma_e * we[i];
        double av = bz * 0.5 * (pa[0] + pb[0]) * d[1] + k * ell * ell * wa[i];
        a[i] = (int64_t)std::llrint(av / c->phys.u_b);
    }
    for (int64_t f = 0; f < m.Nf; ++f) {
        const int32_t *fe = &m.face_edges[3 * f];
        b[f] = a[fe[2]] - a[fe[1]] + a[fe[0]];
    }
    return set_fields(c, e.data(), b.data());
}

int qh_species_add(qh_ctx *c, double q_over_m, int32_t z, int32_t *sid) {
    if (!c || !sid) return QH_EINVAL;
    if (z == 0 || std::abs(z) > 64) return qh_fail(c, QH_EINVAL, "charge number must be in [-64, 64], nonzero");
    Species s;
    s.qm = q_over_m;
    s.z = z;
    c->species.push_back(s);
    *sid = (int32_t)c->species.size() - 1;
    return QH_OK;
}

// Storage of a species for at least cap particles, all or nothing: every new array is
// allocated before any is swapped in, so a failed allocation leaves the species (its count, its
// particles and its arrays) as it was. The first `keep` particles and the tet ranges of their
// blocks are copied into the new arrays; the sort scratch needs no copy.
static int reserve_species(qh_ctx *c, Species &s, int64_t cap, int64_t keep) {
    if (cap <= s.cap) return QH_OK;
    float **fs[12] = {&s.x, &s.y, &s.zz, &s.vx, &s.vy, &s.vz, &s.sx, &s.sy, &s.sz, &s.svx, &s.svy, &s.svz};
    int32_t **is[4] = {&s.tet, &s.id, &s.stet, &s.sid};
    float *nf[12] = {};
    int32_t *ni[4] = {}, *nown = nullptr;
    uint16_t *novf = nullptr;
    auto drop_new = [&]() {
        for (auto &p : nf) qh_release(c, p);
        for (auto &p : ni) qh_release(c, p);
        qh_release(c, nown), qh_release(c, novf);
    };
    int rc;
    for (auto &p : nf)
        if ((rc = qh_alloc(c, &p, cap))) return drop_new(), rc;
    for (auto &p : ni)
        if ((rc = qh_alloc(c, &p, cap))) return drop_new(), rc;
    if ((rc = qh_alloc(c, &nown, qh_species_blocks(cap) + 1)) || (rc = qh_alloc(c, &novf, qh_species_blocks(cap) * QH_CHUNK)))
        return drop_new(), rc;
    hipError_t e = hipSuccess;
    if (keep > 0) {
        for (int k = 0; k < 6 && e == hipSuccess; ++k)
            e = hipMemcpyAsync(nf[k], *fs[k], sizeof(float) * keep, hipMemcpyDeviceToDevice, c->stream);
        for (int k = 0; k < 2 && e == hipSuccess; ++k)
            e = hipMemcpyAsync(ni[k], *is[k], sizeof(int32_t) * keep, hipMemcpyDeviceToDevice, c->stream);
        if (s.own && e == hipSuccess)
            e = hipMemcpyAsync(nown, s.own, sizeof(int32_t) * (qh_species_blocks(keep) + 1), hipMemcpyDeviceToDevice,
                               c->stream);
    }
    // the old arrays may still be read by queued work: released only after the stream has passed
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        drop_new();
        return qh_fail(c, QH_EHIP, std::string("species storage: ") + hipGetErrorString(e));
    }
    for (int k = 0; k < 12; ++k) qh_release(c, *fs[k]), *fs[k] = nf[k];
    for (int k = 0; k < 4; ++k) qh_release(c, *is[k]), *is[k] = ni[k];
    qh_release(c, s.own), s.own = nown;
    qh_release(c, s.ovf), s.ovf = novf;
    s.cap = cap;
    return QH_OK;
}

// Replaces a species' particles; ids: given (a checkpoint) or 0..n-1, next_id the next to give.
static int upload_species(qh_ctx *c, int32_t sid, int64_t n, const float *x, const float *v, const int32_t *tet,
                          const int32_t *ids_in, int64_t next_id);

int qh_particles_upload(qh_ctx *c, int32_t sid, int64_t n, const float *x, const float *v, const int32_t *tet) {
    return upload_species(c, sid, n, x, v, tet, nullptr, n);
}

static int upload_species(qh_ctx *c, int32_t sid, int64_t n, const float *x, const float *v, const int32_t *tet,
                          const int32_t *ids_in, int64_t next_id) {
    if (!c || sid < 0 || sid >= (int32_t)c->species.size() || n < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (n > 0 && (!x || !v)) return QH_EINVAL;
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (n >= ((int64_t)1 << 31)) return qh_fail(c, QH_EINVAL, "at most 2^31-1 particles per species");
    if (tet) {
        for (int64_t i = 0; i < n; ++i)
            if (tet[i] < 0 || tet[i] >= c->hm.Nt) return qh_fail(c, QH_EINVAL, "tet id out of range at particle " + std::to_string(i));
    } else {
        for (int64_t i = 0; i < 3 * n; ++i)
            if (!std::isfinite(x[i])) return qh_fail(c, QH_EINVAL, "non-finite position at particle " + std::to_string(i / 3));
    }
    Species &s = c->species[sid];
    int rc;
    if ((rc = reserve_species(c, s, n, 0))) return rc;
    // the species holds no particle until every array is in place: a failed copy or location
    // leaves it empty, never with unset tet ids
    s.n = 0;
    s.next_id = next_id;
    if (n > 0) {
        std::vector<float> comp(n);
        float *dst[6] = {s.x, s.y, s.zz, s.vx, s.vy, s.vz};
        for (int k = 0; k < 6; ++k) {
            const float *src = k < 3 ? x : v;
            int d = k % 3;
            for (int64_t i = 0; i < n; ++i) comp[i] = src[3 * i + d];
            QH_HIP(c, hipMemcpyAsync(dst[k], comp.data(), sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
            QH_HIP(c, hipStreamSynchronize(c->stream));
        }
        std::vector<int32_t> ids(n);
        if (ids_in) std::copy(ids_in, ids_in + n, ids.begin());
        else std::iota(ids.begin(), ids.end(), 0);
        if (tet) QH_HIP(c, hipMemcpyAsync(s.tet, tet, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
        else if ((rc = locate_species(c, s, 0, n))) return rc;
        QH_HIP(c, hipMemcpyAsync(s.id, ids.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipStreamSynchronize(c->stream));
        s.n = n;
        if ((rc = qh_sort_species(c, s))) return rc;
    }
    c->wave_hist = false;
    return recompute_charge(c);
}

int qh_particles_download(const qh_ctx *cc, int32_t sid, float *x, float *v, int32_t *tet) {
    qh_ctx *c = const_cast<qh_ctx *>(cc);
    if (!c || sid < 0 || sid >= (int32_t)c->species.size()) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    const Species &s = c->species[sid];
    int64_t n = s.n;
    if (n == 0) return QH_OK;
    std::vector<int32_t> ids(n), tt(n);
    std::vector<float> comp(6 * n);
    const float *src[6] = {s.x, s.y, s.zz, s.vx, s.vy, s.vz};
    for (int k = 0; k < 6; ++k)
        QH_HIP(c, hipMemcpyAsync(comp.data() + k * n, src[k], sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipMemcpyAsync(ids.data(), s.id, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipMemcpyAsync(tt.data(), s.tet, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    // rank of each particle by id (ids are unique; after injections and absorptions they are
    // not a permutation of 0..n-1)
    std::vector<int64_t> order(n), rank(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int64_t p, int64_t q) { return ids[p] < ids[q]; });
    for (int64_t r = 0; r < n; ++r) rank[order[r]] = r;
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = rank[i];
        if (x)
            for (int d = 0; d < 3; ++d) x[3 * j + d] = comp[d * n + i];
        if (v)
            for (int d = 0; d < 3; ++d) v[3 * j + d] = comp[(3 + d) * n + i];
        if (tet) tet[j] = tt[i];
    }
    return QH_OK;
}

int qh_particles_count(const qh_ctx *c, int32_t sid, int64_t *n) {
    if (!c || !n || sid < 0 || sid >= (int32_t)c->species.size()) return QH_EINVAL;
    *n = c->species[sid].n;
    return QH_OK;
}

int qh_particles_ids(const qh_ctx *cc, int32_t sid, int32_t *ids) {
    qh_ctx *c = const_cast<qh_ctx *>(cc);
    if (!c || !ids || sid < 0 || sid >= (int32_t)c->species.size()) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    const Species &s = c->species[sid];
    if (s.n == 0) return QH_OK;
    QH_HIP(c, hipMemcpyAsync(ids, s.id, sizeof(int32_t) * s.n, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    std::sort(ids, ids + s.n);
    return QH_OK;
}

int qh_set_walls(qh_ctx *c, int32_t mode) {
    if (!c) return QH_EINVAL;
    if (mode != QH_WALLS_REFLECT && mode != QH_WALLS_ABSORB) return qh_fail(c, QH_EINVAL, "walls: QH_WALLS_REFLECT or QH_WALLS_ABSORB");
    c->walls = mode;
    return QH_OK;
}

int qh_particles_inject(qh_ctx *c, int32_t sid, int64_t n, const float *x, const float *v, const int32_t *tet) {
    if (!c || sid < 0 || sid >= (int32_t)c->species.size() || n < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (n == 0) return QH_OK;
    if (!x || !v) return QH_EINVAL;
    if (tet) {
        for (int64_t i = 0; i < n; ++i)
            if (tet[i] < 0 || tet[i] >= c->hm.Nt) return qh_fail(c, QH_EINVAL, "tet id out of range at particle " + std::to_string(i));
    } else {
        for (int64_t i = 0; i < 3 * n; ++i)
            if (!std::isfinite(x[i])) return qh_fail(c, QH_EINVAL, "non-finite position at particle " + std::to_string(i / 3));
    }
    Species &s = c->species[sid];
    const int64_t n0 = s.n, n1 = n0 + n;
    if (n1 >= ((int64_t)1 << 31) || s.next_id + n >= ((int64_t)1 << 31))
        return qh_fail(c, QH_EINVAL, "at most 2^31-1 particles (and ids) per species");
    int rc;
    if (n1 > s.cap && (rc = reserve_species(c, s, std::max<int64_t>(std::max<int64_t>(2 * s.cap, n1), 4096), n0)))
        return rc;
    // components laid out one after another; the host buffers live until the sync at the end
    std::vector<float> comp(6 * n);
    float *dst[6] = {s.x, s.y, s.zz, s.vx, s.vy, s.vz};
    for (int k = 0; k < 6; ++k) {
        const float *src = k < 3 ? x : v;
        for (int64_t i = 0; i < n; ++i) comp[k * n + i] = src[3 * i + k % 3];
        QH_HIP(c, hipMemcpyAsync(dst[k] + n0, comp.data() + k * n, sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
    }
    std::vector<int32_t> ids(n);
    std::iota(ids.begin(), ids.end(), (int32_t)s.next_id);
    if (tet) QH_HIP(c, hipMemcpyAsync(s.tet + n0, tet, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
    else if ((rc = locate_species(c, s, n0, n))) return rc;  // s.n is still n0: nothing was added
    QH_HIP(c, hipMemcpyAsync(s.id + n0, ids.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
    s.next_id += n;
    s.n = n1;
    QH_HIP(c, launch_own_extend(c, s, (int32_t)qh_species_blocks(n0), (int32_t)qh_species_blocks(n1)));
    QH_HIP(c, launch_charge_deposit(c, s, n0));
    return sync(c);
}

int qh_locate(qh_ctx *c, int64_t n, const double *xyz, int32_t *tet) {
    if (!c || n < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (n == 0) return QH_OK;
    if (!xyz || !tet) return QH_EINVAL;
    std::vector<float> comp(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            if (!std::isfinite(xyz[3 * i + d])) return qh_fail(c, QH_EINVAL, "non-finite point " + std::to_string(i));
            comp[d * n + i] = (float)xyz[3 * i + d];
        }
    float *dx = nullptr;
    int32_t *dt = nullptr;
    int rc;
    if ((rc = qh_alloc(c, &dx, 3 * n)) || (rc = qh_alloc(c, &dt, n))) return rc;
    QH_HIP(c, hipMemcpyAsync(dx, comp.data(), sizeof(float) * 3 * n, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, launch_locate(c, n, dx, dx + n, dx + 2 * n, dt));
    QH_HIP(c, hipMemcpyAsync(tet, dt, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    qh_release(c, dx), qh_release(c, dt);
    return QH_OK;
}

int qh_probe_fields(qh_ctx *c, int64_t n, const double *xyz, const int32_t *tet, double *E, double *B) {
    if (!c || n < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh || !c->have_phys || !c->have_fields) return qh_fail(c, QH_ESTATE, "mesh, physics and fields first");
    if (n == 0) return QH_OK;
    if (!xyz || !tet) return QH_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (tet[i] < 0 || tet[i] >= c->hm.Nt) return qh_fail(c, QH_EINVAL, "tet id out of range at point " + std::to_string(i));
    double *dx = nullptr, *dE = nullptr, *dB = nullptr;
    int32_t *dt = nullptr;
    int rc;
    if ((rc = qh_alloc(c, &dx, 3 * n)) || (rc = qh_alloc(c, &dt, n)) || (rc = qh_alloc(c, &dE, 3 * n)) ||
        (rc = qh_alloc(c, &dB, 3 * n)))
        return rc;
    QH_HIP(c, hipMemcpyAsync(dx, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, hipMemcpyAsync(dt, tet, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
    launch_field_prep(c);  // the records of the present e and b
    QH_HIP(c, launch_probe(c, n, dx, dt, dE, dB));
    if (E) QH_HIP(c, hipMemcpyAsync(E, dE, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    if (B) QH_HIP(c, hipMemcpyAsync(B, dB, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    qh_release(c, dx), qh_release(c, dt), qh_release(c, dE), qh_release(c, dB);
    return QH_OK;
}

int qh_charge_background(qh_ctx *c, int32_t mode) {
    if (!c) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (mode == 0) QH_HIP(c, hipMemsetAsync(c->Q_bg, 0, sizeof(int64_t) * c->hm.Nn, c->stream));
    else if (mode == 1) QH_HIP(c, hipMemcpyAsync(c->Q_bg, c->Q, sizeof(int64_t) * c->hm.Nn, hipMemcpyDeviceToDevice, c->stream));
    else return qh_fail(c, QH_EINVAL, "background mode must be 0 or 1");
    return sync(c);
}

int qh_capture_segments(qh_ctx *c, int64_t cap) {
    if (!c || cap < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (cap > c->cap_segments) {
        int rc;
        if ((rc = qh_alloc(c, &c->seg_buf, 12 * cap))) return rc;
        if (!c->seg_count && (rc = qh_alloc(c, &c->seg_count, 1))) return rc;
        c->cap_segments = cap;
    }
    if (!c->seg_count) {
        int rc;
        if ((rc = qh_alloc(c, &c->seg_count, 1))) return rc;
    }
    QH_HIP(c, hipMemsetAsync(c->seg_count, 0, sizeof(unsigned long long), c->stream));
    c->capture_next = cap > 0;
    return sync(c);
}

int qh_segments_download(const qh_ctx *cc, int64_t *n_out, int32_t *pid, int32_t *sp, int32_t *seq, int32_t *tet,
                         int32_t *lam0, int32_t *lam1) {
    qh_ctx *c = const_cast<qh_ctx *>(cc);
    if (!c || !n_out) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->seg_count) {
        *n_out = 0;
        return QH_OK;
    }
    unsigned long long cnt = 0;
    QH_HIP(c, hipMemcpyAsync(&cnt, c->seg_count, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    *n_out = (int64_t)cnt;
    int64_t k = std::min<int64_t>((int64_t)cnt, c->cap_segments);
    std::vector<int32_t> buf(12 * std::max<int64_t>(k, 1));
    if (k > 0) QH_HIP(c, hipMemcpyAsync(buf.data(), c->seg_buf, sizeof(int32_t) * 12 * k, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < k; ++i) {
        const int32_t *o = &buf[12 * i];
        if (pid) pid[i] = o[0];
        if (sp) sp[i] = o[1];
        if (seq) seq[i] = o[2];
        if (tet) tet[i] = o[3];
        for (int q = 0; q < 4; ++q) {
            if (lam0) lam0[4 * i + q] = o[4 + q];
            if (lam1) lam1[4 * i + q] = o[8 + q];
        }
    }
    return QH_OK;
}

int qh_edge_system_download(const qh_ctx *cc, double *rhs, double *sol) {
    qh_ctx *c = const_cast<qh_ctx *>(cc);
    if (!c) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    if (rhs) QH_HIP(c, hipMemcpyAsync(rhs, c->cge.b, sizeof(double) * c->A.n, hipMemcpyDeviceToHost, c->stream));
    if (sol) QH_HIP(c, hipMemcpyAsync(sol, c->e_star, sizeof(double) * c->A.n, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int qh_fields_download_dev(qh_ctx *c, double *e, int64_t *b) {
    if (!c) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (e) QH_HIP(c, hipMemcpyAsync(e, c->e, sizeof(double) * c->hm.Ne, hipMemcpyDeviceToDevice, c->stream));
    if (b) QH_HIP(c, hipMemcpyAsync(b, c->b, sizeof(int64_t) * c->hm.Nf, hipMemcpyDeviceToDevice, c->stream));
    return QH_OK;
}

int qh_deposits_download_dev(qh_ctx *c, int64_t *g, int64_t *Q) {
    if (!c) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (g) QH_HIP(c, hipMemcpyAsync(g, c->g, sizeof(int64_t) * c->hm.Ne, hipMemcpyDeviceToDevice, c->stream));
    if (Q) QH_HIP(c, hipMemcpyAsync(Q, c->Q, sizeof(int64_t) * c->hm.Nn, hipMemcpyDeviceToDevice, c->stream));
    return QH_OK;
}

int qh_fields_upload_dev(qh_ctx *c, const double *e, const int64_t *b) {
    if (!c || !e || !b) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    const HostMesh &m = c->hm;
    // D b = 0 checked on the device before anything changes
    unsigned long long *bad = c->counters + 4 * QH_COUNTER_SLOTS + QH_CNT_DIVB, nbad = 0;
    QH_HIP(c, hipMemsetAsync(c->divb0, 0, sizeof(int64_t) * m.Nt, c->stream));
    QH_HIP(c, hipMemsetAsync(bad, 0, sizeof(unsigned long long), c->stream));
    QH_HIP(c, launch_divb_check(c, b, bad));
    QH_HIP(c, hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    if (nbad) return qh_fail(c, QH_EINVAL, "D b != 0 in " + std::to_string(nbad) + " tets");
    QH_HIP(c, hipMemsetAsync(c->e, 0, sizeof(double) * m.Ne, c->stream));  // PEC wall edges stay 0
    QH_HIP(c, launch_fields_in(c, e, c->assembled ? c->cge.x : nullptr));
    QH_HIP(c, hipMemcpyAsync(c->b, b, sizeof(int64_t) * m.Nf, hipMemcpyDeviceToDevice, c->stream));
    c->have_fields = true;
    c->fields_dirty = true;
    c->wave_hist = false;
    if (c->dbnd) QH_HIP(c, hipMemsetAsync(c->dbnd, 0, sizeof(double) * m.Nn, c->stream));
    return QH_OK;
}

int qh_deposits_download(const qh_ctx *cc, int64_t *g, int64_t *Q) {
    qh_ctx *c = const_cast<qh_ctx *>(cc);
    if (!c) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (g) QH_HIP(c, hipMemcpyAsync(g, c->g, sizeof(int64_t) * c->hm.Ne, hipMemcpyDeviceToHost, c->stream));
    if (Q) QH_HIP(c, hipMemcpyAsync(Q, c->Q, sizeof(int64_t) * c->hm.Nn, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int qh_deposit(qh_ctx *c, int64_t n_seg, const int32_t *seg_tet, const int32_t *lam0, const int32_t *lam1,
               const int32_t *seg_z, int64_t n_pt, const int32_t *pt_tet, const int32_t *pt_lam, const int32_t *pt_z,
               int64_t *g_out, int64_t *q_out) {
    if (!c || n_seg < 0 || n_pt < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (n_seg > 0 && (!seg_tet || !lam0 || !lam1 || !seg_z)) return QH_EINVAL;
    if (n_pt > 0 && (!pt_tet || !pt_lam || !pt_z)) return QH_EINVAL;
    const HostMesh &m = c->hm;
    for (int64_t s = 0; s < n_seg; ++s)
        if (seg_tet[s] < 0 || seg_tet[s] >= m.Nt) return qh_fail(c, QH_EINVAL, "segment tet out of range");
    for (int64_t p = 0; p < n_pt; ++p)
        if (pt_tet[p] < 0 || pt_tet[p] >= m.Nt) return qh_fail(c, QH_EINVAL, "point tet out of range");
    int32_t *d = nullptr;
    int64_t *gd = nullptr, *qd = nullptr;
    size_t ni = (size_t)(10 * n_seg + 6 * n_pt) + 1;  // st, l0, l1, sz | pt, pl, pz
    if (hipMalloc((void **)&d, ni * sizeof(int32_t)) != hipSuccess) return qh_fail(c, QH_ENOMEM, "deposit buffers");
    if (hipMalloc((void **)&gd, (m.Ne + m.Nn) * sizeof(int64_t)) != hipSuccess) {
        (void)hipFree(d);
        return qh_fail(c, QH_ENOMEM, "deposit buffers");
    }
    qd = gd + m.Ne;
    int32_t *st = d, *l0 = st + n_seg, *l1 = l0 + 4 * n_seg, *sz = l1 + 4 * n_seg;
    int32_t *pt = sz + n_seg, *pl = pt + n_pt, *pz = pl + 4 * n_pt;
    hipError_t e = hipSuccess;
    auto cp = [&](int32_t *dst, const int32_t *src, int64_t k) {
        if (k > 0 && e == hipSuccess) e = hipMemcpyAsync(dst, src, sizeof(int32_t) * k, hipMemcpyHostToDevice, c->stream);
    };
    cp(st, seg_tet, n_seg); cp(l0, lam0, 4 * n_seg); cp(l1, lam1, 4 * n_seg); cp(sz, seg_z, n_seg);
    cp(pt, pt_tet, n_pt); cp(pl, pt_lam, 4 * n_pt); cp(pz, pt_z, n_pt);
    if (e == hipSuccess) e = hipMemsetAsync(gd, 0, (m.Ne + m.Nn) * sizeof(int64_t), c->stream);
    if (e == hipSuccess) e = launch_deposit_lists(c, n_seg, st, l0, l1, sz, n_pt, pt, pl, pz, gd, qd);
    if (e == hipSuccess && g_out) e = hipMemcpyAsync(g_out, gd, sizeof(int64_t) * m.Ne, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && q_out) e = hipMemcpyAsync(q_out, qd, sizeof(int64_t) * m.Nn, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    (void)hipFree(gd);
    if (e != hipSuccess) return qh_fail(c, QH_EHIP, std::string("deposit: ") + hipGetErrorString(e));
    return QH_OK;
}

int qh_deposit_noalloc(qh_ctx *c, int64_t n_seg, const int32_t *seg_tet, const int32_t *lam0, const int32_t *lam1,
                       const int32_t *seg_z, int64_t n_pt, const int32_t *pt_tet, const int32_t *pt_lam,
                       const int32_t *pt_z, int64_t *g_out, int64_t *q_out) {
    if (!c || n_seg < 0 || n_pt < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh) return qh_fail(c, QH_ESTATE, "no mesh");
    if (n_seg > 0 && (!seg_tet || !lam0 || !lam1 || !seg_z)) return QH_EINVAL;
    if (n_pt > 0 && (!pt_tet || !pt_lam || !pt_z)) return QH_EINVAL;
    const HostMesh &m = c->hm;
    const size_t need = qh_static_deposit_bytes(m.Ne, m.Nn, n_seg, n_pt), have = qh_static_scratch_bytes();
    if (n_seg > ((int64_t)1 << 40) || n_pt > ((int64_t)1 << 40) || need > have)
        return qh_fail(c, QH_EINVAL, "deposit needs " + std::to_string(need) + " bytes of the static scratch array, which holds " +
                                         std::to_string(have) + " (8 bytes per edge and node, 40 per piece, 24 per point)");
    for (int64_t s = 0; s < n_seg; ++s)
        if (seg_tet[s] < 0 || seg_tet[s] >= m.Nt) return qh_fail(c, QH_EINVAL, "segment tet out of range");
    for (int64_t p = 0; p < n_pt; ++p)
        if (pt_tet[p] < 0 || pt_tet[p] >= m.Nt) return qh_fail(c, QH_EINVAL, "point tet out of range");
    return qh_static_deposit(c, n_seg, seg_tet, lam0, lam1, seg_z, n_pt, pt_tet, pt_lam, pt_z, g_out, q_out);
}

int qh_pic_step(qh_ctx *c, const qh_step_params_t *P, int32_t n_steps, qh_step_stats_t *stats) {
    if (!c || !P || n_steps < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->have_mesh || !c->have_phys || !c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    if (!c->have_fields) return qh_fail(c, QH_ESTATE, "fields first");
    if (P->field_mode != QH_FIELDS_FROZEN && P->field_mode != QH_FIELDS_SOLVE && P->field_mode != QH_FIELDS_WAVE)
        return qh_fail(c, QH_EINVAL, "field_mode");
    const bool solve = P->field_mode != QH_FIELDS_FROZEN;
    if (P->precond != QH_PC_JACOBI && P->precond != QH_PC_LEARNED) return qh_fail(c, QH_EINVAL, "precond");
    if (P->solver != QH_SOLVER_FP64 && P->solver != QH_SOLVER_MIXED) return qh_fail(c, QH_EINVAL, "solver");
    const bool learned = P->precond == QH_PC_LEARNED && solve;
    if (learned) {
        int rc = qh_learned_setup(c);
        if (rc) return rc;
        if (!c->lp.factor_valid && (rc = qh_learned_factor(c))) return rc;
    }
    const HostMesh &m = c->hm;
    int status = QH_OK;
    hipEvent_t ev[4];
    bool use_ev = stats != nullptr;
    if (use_ev)
        for (auto &x : ev) QH_HIP(c, hipEventCreateWithFlags(&x, hipEventDisableSystemFence));
    // totals of the whole call (fixed-point headroom overflows of the gathers, lost particles,
    // verification failures), kept whether or not stats are asked for; the per-step slots before
    // them are cleared every step
    unsigned long long *totals = c->counters + 4 * QH_COUNTER_SLOTS + QH_CNT_HEADROOM_CALL;
    constexpr int kTotals = QH_CNT_DIVB_CALL - QH_CNT_HEADROOM_CALL + 1;
    QH_HIP(c, hipMemsetAsync(totals, 0, sizeof(unsigned long long) * kTotals, c->stream));
    for (int32_t st = 0; st < n_steps; ++st) {
        bool capture = c->capture_next;
        c->capture_next = false;
        if (use_ev) QH_HIP(c, hipEventRecord(ev[0], c->stream));
        if (c->fields_dirty || solve) {
            int t0 = qh_tbeg(c);
            launch_field_prep(c);
            qh_tend(c, t0, QK_FIELD_PREP);
            c->fields_dirty = false;
        }
        std::swap(c->Q, c->Q_old);
        QH_HIP(c, hipMemsetAsync(c->Q, 0, sizeof(int64_t) * m.Nn, c->stream));
        QH_HIP(c, hipMemsetAsync(c->g, 0, sizeof(int64_t) * m.Ne, c->stream));
        QH_HIP(c, hipMemsetAsync(c->counters, 0, sizeof(unsigned long long) * (4 * QH_COUNTER_SLOTS + QH_CNT_STEP_END),
                                 c->stream));
        for (size_t k = 0; k < c->species.size(); ++k) {
            int t0 = qh_tbeg(c);
            QH_HIP(c, launch_particle_step(c, c->species[k], (int)k, capture));
            qh_tend(c, t0, QK_PARTICLE);
        }
        // absorbing walls: every step ends with a sort, which drops the absorbed particles
        if (c->walls == QH_WALLS_ABSORB || (P->sort_every > 0 && (c->step_index + 1) % P->sort_every == 0))
            for (auto &s : c->species) {
                int t0 = qh_tbeg(c);
                int rc = qh_sort_species(c, s);
                if (rc) return rc;
                qh_tend(c, t0, QK_SORT);
            }
        if (use_ev) QH_HIP(c, hipEventRecord(ev[1], c->stream));
        SolveResult se, sn;
        double gauss_out[4] = {0, 0, 0, 0};
        if (solve) {
            QH_HIP(c, hipMemcpyAsync(c->e_old, c->cge.x, sizeof(double) * c->A.n, hipMemcpyDeviceToDevice, c->stream));
            // the wave-equation right-hand side needs e^{n-1} and the previous current: without
            // them (first step in this mode) the step takes the trapezoidal update
            const bool wave = P->field_mode == QH_FIELDS_WAVE && c->wave_hist;
            int t0 = qh_tbeg(c);
            QH_HIP(c, wave ? launch_wave_rhs(c) : launch_edge_rhs(c));
            qh_tend(c, t0, QK_EDGE_RHS);
            if (c->pw_on) {
                t0 = qh_tbeg(c);
                QH_HIP(c, launch_plane_wave(c, wave));
                qh_tend(c, t0, QK_BOUNDARY);
            }
            const bool mixed = P->solver == QH_SOLVER_MIXED;
            int rc = mixed ? qh_cg_solve_mixed(c, c->A, c->cge, P->tol_edge, P->max_it_edge, P->check_every, se, learned)
                           : qh_cg_solve(c, c->A, c->cge, P->tol_edge, P->max_it_edge, P->check_every, se, nullptr,
                                         false, learned);
            if (rc) return rc;
            c->last_refinements = se.refinements;
            int fallbacks = 0;
            if ((learned || mixed) && !se.converged) {
                // FP64 Jacobi restart: from the iterate when it is finite (the stall rule, the
                // iteration cap stopped it), from e^n after non-finite values
                if (se.flag == 3)
                    QH_HIP(c, hipMemcpyAsync(c->cge.x, c->e_old, sizeof(double) * c->A.n, hipMemcpyDeviceToDevice,
                                             c->stream));
                SolveResult sj;
                rc = qh_cg_solve(c, c->A, c->cge, P->tol_edge, P->max_it_edge, P->check_every, sj, nullptr);
                if (rc) return rc;
                sj.iters += se.iters;
                se = sj;
                fallbacks = 1;
            }
            c->last_fallbacks = fallbacks;
            if (!se.converged) status = QH_ENOTCONV;
            QH_HIP(c, hipMemcpyAsync(c->e_star, c->cge.x, sizeof(double) * c->A.n, hipMemcpyDeviceToDevice, c->stream));
            // the (rhs, solution) pair of this step into the bank, while recording
            if (c->lp.pair_rec && (rc = qh_learned_record_pair(c, c->cge.b, c->e_star))) return rc;
            if (P->gauss) {
                t0 = qh_tbeg(c);
                QH_HIP(c, launch_gauss_rhs(c, c->scratch_d, P->tol_node));
                QH_HIP(c, hipMemsetAsync(c->cgn.x, 0, sizeof(double) * c->K.n, c->stream));
                qh_tend(c, t0, QK_GAUSS);
                rc = qh_cg_solve(c, c->K, c->cgn, P->tol_node, P->max_it_node, P->check_every, sn, c->scratch_d, true);
                if (rc) return rc;
                if (!sn.converged) status = QH_ENOTCONV;
                t0 = qh_tbeg(c);
                QH_HIP(c, launch_gauss_apply(c));
                qh_tend(c, t0, QK_GAUSS);
            }
            int t1 = qh_tbeg(c);
            QH_HIP(c, launch_faraday(c));
            qh_tend(c, t1, QK_FARADAY);
            if (P->field_mode == QH_FIELDS_WAVE) {
                QH_HIP(c, hipMemcpyAsync(c->e_prev, c->e_old, sizeof(double) * c->A.n, hipMemcpyDeviceToDevice,
                                         c->stream));
                QH_HIP(c, hipMemcpyAsync(c->g_prev, c->g, sizeof(int64_t) * m.Ne, hipMemcpyDeviceToDevice, c->stream));
            }
            c->wave_hist = P->field_mode == QH_FIELDS_WAVE;
            if (stats) {
                // Gauss residual after the update (reuses the node right-hand-side buffer)
                QH_HIP(c, launch_gauss_rhs(c, c->scratch_d + 4, P->tol_node));
                QH_HIP(c, hipMemcpyAsync(gauss_out, c->scratch_d + 4, sizeof(gauss_out), hipMemcpyDeviceToHost, c->stream));
            }
        }
        if (!solve) c->wave_hist = false;  // the fields did not follow this step's current
        if (P->verify) QH_HIP(c, launch_verify(c, true));
        if (use_ev) QH_HIP(c, hipEventRecord(ev[2], c->stream));
        if (stats) {
            std::vector<unsigned long long> raw(4 * QH_COUNTER_SLOTS + 8);
            QH_HIP(c, hipMemcpyAsync(raw.data(), c->counters, sizeof(unsigned long long) * raw.size(),
                                     hipMemcpyDeviceToHost, c->stream));
            QH_HIP(c, hipStreamSynchronize(c->stream));
            unsigned long long cnt[6] = {0, 0, 0, 0, 0, 0};
            for (int k = 0; k < QH_COUNTER_SLOTS; ++k) {
                for (int j = 0; j < 3; ++j) cnt[j] += raw[4 * k + j];
                cnt[5] += raw[4 * k + 3];
            }
            cnt[3] = raw[4 * QH_COUNTER_SLOTS + QH_CNT_CONT];
            cnt[4] = raw[4 * QH_COUNTER_SLOTS + QH_CNT_DIVB];
            qh_step_stats_t &S = stats[st];
            std::memset(&S, 0, sizeof(S));
            S.edge_iters = se.iters;
            S.node_iters = sn.iters;
            S.edge_res = se.res;
            S.node_res = sn.res;
            S.gauss_res = gauss_out[1] > 0 ? std::sqrt(gauss_out[2]) / gauss_out[1] : 0.0;
            S.gauss_res_rho = gauss_out[3] > 0 ? std::sqrt(gauss_out[2]) / gauss_out[3] : 0.0;
            S.crossings = (int64_t)cnt[0];
            S.wall_hits = (int64_t)cnt[1];
            S.lost = (int64_t)cnt[2];
            S.continuity_bad = P->verify ? (int64_t)cnt[3] : -1;
            S.divb_bad = P->verify ? (int64_t)cnt[4] : -1;
            S.foreign = (int64_t)cnt[5];
            S.fallbacks = solve ? c->last_fallbacks : 0;
            S.edge_refinements = solve ? c->last_refinements : 0;
            (void)hipEventElapsedTime(&S.ms_particles, ev[0], ev[1]);
            (void)hipEventElapsedTime(&S.ms_fields, ev[1], ev[2]);
        }
        qh_tflush(c);
        c->step_index++;
    }
    if (use_ev)
        for (auto &x : ev) (void)hipEventDestroy(x);
    unsigned long long tot[kTotals] = {};
    QH_HIP(c, hipMemcpyAsync(tot, totals, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    const unsigned long long nhead = tot[0], nlost = tot[QH_CNT_LOST_CALL - QH_CNT_HEADROOM_CALL],
                             ncont = tot[QH_CNT_CONT_CALL - QH_CNT_HEADROOM_CALL],
                             ndivb = tot[QH_CNT_DIVB_CALL - QH_CNT_HEADROOM_CALL];
    // the most serious failure of the call names the status: a broken invariant, then a solve
    // at its cap, lost particles, fixed-point headroom
    if (ncont || ndivb) {
        status = QH_EVERIFY;
        c->err = "verification: continuity G^T g = Q^{n+1} - Q^n failed at " + std::to_string(ncont) +
                 " node-steps, D b changed in " + std::to_string(ndivb) + " tet-steps";
    } else if (status == QH_ENOTCONV) {
        c->err = "a Krylov solve hit its iteration cap";
    } else if (nlost) {
        status = QH_ELOST;
        c->err = std::to_string(nlost) + " particle-steps hit the walk cap";
    } else if (nhead) {
        status = QH_EOVERFLOW;
        c->err = std::to_string(nhead) + " edge currents or node charges of a step beyond 2^60 (int64 headroom)";
    }
    return status;
}

int qh_fields_energy(qh_ctx *c, double *w_e, double *w_m) {
    if (!c || !w_e || !w_m) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled || !c->have_fields) return qh_fail(c, QH_ESTATE, "mesh, physics and fields first");
    int rc;
    const int32_t np = qh_energy_parts(c);
    if (!c->xyz_d && (rc = upload(c, &c->xyz_d, c->hm.xyz.data(), c->hm.xyz.size()))) return rc;
    if (!c->energy_d && (rc = qh_alloc(c, &c->energy_d, (size_t)np + 2))) return rc;
    QH_HIP(c, launch_field_energy(c, c->energy_d, c->energy_d + np));
    double out[2];
    QH_HIP(c, hipMemcpyAsync(out, c->energy_d + np, sizeof out, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    *w_e = out[0];
    *w_m = out[1];
    return QH_OK;
}

int qh_fields_decompose(qh_ctx *c, double tol, int32_t max_it, double *e_ns, double *e_s, double *rho_bar,
                        qh_solve_stats_t *stats) {
    if (!c || !(tol > 0) || max_it < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled || !c->have_fields) return qh_fail(c, QH_ESTATE, "mesh, physics and fields first");
    const HostMesh &m = c->hm;
    const int32_t ne = c->A.n, nn = c->K.n;
    int rc;
    if (!c->dec_e && (rc = qh_alloc(c, &c->dec_e, std::max<int32_t>(ne, 1)))) return rc;
    hipEvent_t e0, e1;
    QH_HIP(c, hipEventCreate(&e0));
    QH_HIP(c, hipEventCreate(&e1));
    QH_HIP(c, hipEventRecord(e0, c->stream));
    SolveResult sn;
    sn.converged = true;
    if (nn > 0) {
        // K delta = -G^T [*eps] e, so delta = -E_ns and E_s = e + G delta
        QH_HIP(c, launch_div_e(c, c->scratch_d, tol));
        QH_HIP(c, hipMemsetAsync(c->cgn.x, 0, sizeof(double) * nn, c->stream));
        if ((rc = qh_cg_solve(c, c->K, c->cgn, tol, max_it, 8, sn, c->scratch_d, true))) return rc;
    }
    QH_HIP(c, hipMemcpyAsync(c->dec_e, c->cge.x, sizeof(double) * ne, hipMemcpyDeviceToDevice, c->stream));
    if (nn > 0) QH_HIP(c, launch_grad_add(c, c->cgn.x, c->dec_e));
    QH_HIP(c, hipEventRecord(e1, c->stream));
    std::vector<double> es(ne), dl(nn), rg(nn);
    QH_HIP(c, hipMemcpyAsync(es.data(), c->dec_e, sizeof(double) * ne, hipMemcpyDeviceToHost, c->stream));
    if (nn > 0) {
        QH_HIP(c, hipMemcpyAsync(dl.data(), c->cgn.x, sizeof(double) * nn, hipMemcpyDeviceToHost, c->stream));
        QH_HIP(c, hipMemcpyAsync(rg.data(), c->cgn.b, sizeof(double) * nn, hipMemcpyDeviceToHost, c->stream));
    }
    QH_HIP(c, hipStreamSynchronize(c->stream));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e_s) {
        std::fill(e_s, e_s + m.Ne, 0.0);
        for (int32_t i = 0; i < ne; ++i) e_s[m.int_edges[i]] = es[i];
    }
    if (e_ns) {
        std::fill(e_ns, e_ns + m.Nn, 0.0);
        for (int32_t i = 0; i < nn; ++i) e_ns[m.int_nodes[i]] = -dl[i];
        if (m.neumann) {
            // the potential is fixed up to a constant: zero W0-weighted mean (alpha_i = integral of W0_i)
            std::vector<double> alpha(m.Nn, 0.0);
            for (int64_t t = 0; t < m.Nt; ++t)
                for (int k = 0; k < 4; ++k) alpha[m.tn[4 * t + k]] += 0.25 * m.vol[t];
            double sa = 0.0, sp = 0.0;
            for (int64_t v = 0; v < m.Nn; ++v) sa += alpha[v], sp += alpha[v] * e_ns[v];
            for (int64_t v = 0; v < m.Nn; ++v) e_ns[v] -= sp / sa;
        }
    }
    if (rho_bar) {
        std::fill(rho_bar, rho_bar + m.Nn, 0.0);
        for (int32_t i = 0; i < nn; ++i) rho_bar[m.int_nodes[i]] = -rg[i];
    }
    if (stats) {
        stats->iters = sn.iters;
        stats->res = sn.res;
        stats->fallback = 0;
        stats->ms = ms;
    }
    return sn.converged ? QH_OK : qh_fail(c, QH_ENOTCONV, "decomposition: node solve did not converge");
}

int qh_field_solve(qh_ctx *c, int32_t system, const double *rhs, double *x, double tol, int32_t max_it,
                   int32_t precond, int32_t solver, qh_solve_stats_t *stats) {
    if (!c || !rhs || !x || max_it < 0) return QH_EINVAL;
    if (solver != QH_SOLVER_FP64 && solver != QH_SOLVER_MIXED) return qh_fail(c, QH_EINVAL, "solver");
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    DevCsr *M = system == QH_SYS_EDGE ? &c->A : system == QH_SYS_NODE ? &c->K : nullptr;
    if (!M) return qh_fail(c, QH_EINVAL, "system must be QH_SYS_EDGE or QH_SYS_NODE");
    if (precond != QH_PC_JACOBI && !(precond == QH_PC_LEARNED && system == QH_SYS_EDGE))
        return qh_fail(c, QH_EINVAL, "the learned preconditioner exists for the edge system only");
    const bool learned = precond == QH_PC_LEARNED;
    int rc;
    if (learned) {
        if ((rc = qh_learned_setup(c))) return rc;
        if (!c->lp.factor_valid && (rc = qh_learned_factor(c))) return rc;
    }
    int32_t nmax = std::max(c->A.n, c->K.n);
    if (c->cgx.n < nmax && (rc = qh_cg_alloc(c, c->cgx, nmax))) return rc;
    const bool mixed = solver == QH_SOLVER_MIXED;
    if (mixed && (rc = qh_cg_alloc32(c, c->cgx, nmax))) return rc;
    CgWork w = c->cgx;
    w.n = M->n;
    QH_HIP(c, hipMemcpyAsync(w.b, rhs, sizeof(double) * w.n, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, hipMemcpyAsync(w.x, x, sizeof(double) * w.n, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, launch_diag_inv(c, *M, w.dinv));
    hipEvent_t e0, e1;
    QH_HIP(c, hipEventCreate(&e0));
    QH_HIP(c, hipEventCreate(&e1));
    QH_HIP(c, hipEventRecord(e0, c->stream));
    SolveResult r;
    rc = mixed ? qh_cg_solve_mixed(c, *M, w, tol, max_it, 8, r, learned)
               : qh_cg_solve(c, *M, w, tol, max_it, 8, r, nullptr, false, learned);
    if (rc) return rc;
    int fallback = 0;
    if ((learned || mixed) && !r.converged) {
        // FP64 Jacobi restart from the iterate, or from the initial guess after non-finite values
        if (r.flag == 3) QH_HIP(c, hipMemcpyAsync(w.x, x, sizeof(double) * w.n, hipMemcpyHostToDevice, c->stream));
        SolveResult rj;
        rc = qh_cg_solve(c, *M, w, tol, max_it, 8, rj, nullptr);
        if (rc) return rc;
        rj.iters += r.iters;
        r = rj;
        fallback = 1;
    }
    QH_HIP(c, hipEventRecord(e1, c->stream));
    QH_HIP(c, hipMemcpyAsync(x, w.x, sizeof(double) * w.n, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    qh_tflush(c);
    if (stats) {
        stats->iters = r.iters;
        stats->res = r.res;
        stats->fallback = fallback;
        (void)hipEventElapsedTime(&stats->ms, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r.converged ? QH_OK : qh_fail(c, QH_ENOTCONV, "iteration cap reached");
}

int qh_precond_set_weights(qh_ctx *c, const float *w, int64_t n) {
    if (!c || !w || n != QH_MLP_NPARAM) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(w[k])) c->err = "non-finite weights (the solve will fall back to Jacobi)";
    c->lp.have_weights = true;  // keep setup from overwriting
    int rc = qh_learned_setup(c);
    if (rc) return rc;
    QH_HIP(c, hipMemcpyAsync(c->lp.w, w, 4 * n, hipMemcpyHostToDevice, c->stream));
    c->lp.factor_valid = false;
    return sync(c);
}

int qh_precond_get_weights(qh_ctx *c, float *w, int64_t n) {
    if (!c || !w || n != QH_MLP_NPARAM) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    int rc = qh_learned_setup(c);
    if (rc) return rc;
    QH_HIP(c, hipMemcpyAsync(w, c->lp.w, 4 * n, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

namespace {
constexpr char kBlobMagic[8] = {'Q', 'H', 'P', 'R', 'E', 'C', 'N', 'D'};
constexpr uint32_t kBlobVersion = 1;
constexpr size_t kBlobSize = 8 + 4 + 4 + 4 * (size_t)QH_MLP_NPARAM + 4;
uint32_t fnv1a(const unsigned char *p, size_t n) {
    uint32_t h = 2166136261u;
    for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 16777619u;
    return h;
}
}  // namespace

// ---------------------------------------------------------------------------------------
// Checkpoints: the state of a run as one blob (see qh.h for the layout's contents).
extern "C++" {
namespace {
constexpr char kStateMagic[8] = {'Q', 'H', 'S', 'T', 'A', 'T', 'E', '1'};

struct Writer {
    unsigned char *p;
    size_t n = 0;
    void put(const void *src, size_t k) {
        if (p) std::memcpy(p + n, src, k);
        n += k;
    }
    template <class T> void val(T v) { put(&v, sizeof(T)); }
};

struct Reader {
    const unsigned char *p;
    size_t len, n = 0;
    bool ok = true;
    const unsigned char *take(size_t k) {
        if (!ok || n + k > len) { ok = false; return nullptr; }
        const unsigned char *r = p + n;
        n += k;
        return r;
    }
    template <class T> T val() {
        T v{};
        if (const unsigned char *q = take(sizeof(T))) std::memcpy(&v, q, sizeof(T));
        return v;
    }
};

// Writes (or, with w.p null, sizes) the state; device arrays are copied through host buffers.
int state_write(qh_ctx *c, Writer &w) {
    const HostMesh &m = c->hm;
    const int64_t ni = c->A.n;
    const bool has_d = c->dbnd != nullptr;
    w.put(kStateMagic, 8);
    w.val<uint32_t>(1);
    w.val<uint32_t>((c->wave_hist ? 1u : 0u) | (has_d ? 2u : 0u));
    for (int64_t v : {m.Nn, m.Ne, m.Nf, m.Nt, ni, (int64_t)c->species.size(), c->step_index}) w.val<int64_t>(v);
    auto dev = [&](const void *src, size_t bytes) -> int {
        if (w.p) QH_HIP(c, hipMemcpy(w.p + w.n, src, bytes, hipMemcpyDeviceToHost));
        w.n += bytes;
        return QH_OK;
    };
    int rc;
    if ((rc = dev(c->e, 8 * m.Ne)) || (rc = dev(c->b, 8 * m.Nf)) || (rc = dev(c->Q, 8 * m.Nn)) ||
        (rc = dev(c->Q_bg, 8 * m.Nn)))
        return rc;
    if (c->wave_hist && ((rc = dev(c->e_prev, 8 * ni)) || (rc = dev(c->g_prev, 8 * m.Ne)))) return rc;
    if (has_d && (rc = dev(c->dbnd, 8 * m.Nn))) return rc;
    for (const Species &s : c->species) {
        w.val<double>(s.qm);
        w.val<int32_t>(s.z);
        w.val<int32_t>(0);
        w.val<int64_t>(s.n);
        w.val<int64_t>(s.next_id);
        const float *f[6] = {s.x, s.y, s.zz, s.vx, s.vy, s.vz};
        for (auto a : f)
            if ((rc = dev(a, 4 * s.n))) return rc;
        if ((rc = dev(s.tet, 4 * s.n)) || (rc = dev(s.id, 4 * s.n))) return rc;
    }
    const uint32_t h = w.p ? fnv1a(w.p, w.n) : 0u;
    w.val<uint32_t>(h);
    return QH_OK;
}
}  // namespace
}  // extern "C++"

int qh_state_save(qh_ctx *c, void *buf, size_t *len) {
    if (!c || !len) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled || !c->have_fields) return qh_fail(c, QH_ESTATE, "mesh, physics and fields first");
    Writer sizer{nullptr};
    int rc = state_write(c, sizer);
    if (rc) return rc;
    if (!buf) {
        *len = sizer.n;
        return QH_OK;
    }
    if (*len < sizer.n) return qh_fail(c, QH_EINVAL, "state buffer smaller than the size qh_state_save(NULL) gives");
    QH_HIP(c, hipStreamSynchronize(c->stream));
    Writer w{static_cast<unsigned char *>(buf)};
    if ((rc = state_write(c, w))) return rc;
    *len = w.n;
    return QH_OK;
}

int qh_state_load(qh_ctx *c, const void *buf, size_t len) {
    if (!c || !buf) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    const HostMesh &m = c->hm;
    const unsigned char *p = static_cast<const unsigned char *>(buf);
    if (len < 8 + 4 + 4 + 7 * 8 + 4 || std::memcmp(p, kStateMagic, 8) != 0)
        return qh_fail(c, QH_EINVAL, "not a state blob");
    uint32_t h;
    std::memcpy(&h, p + len - 4, 4);
    if (h != fnv1a(p, len - 4)) return qh_fail(c, QH_EINVAL, "state blob fails its checksum");
    Reader r{p, len - 4};
    r.take(8);
    const uint32_t version = r.val<uint32_t>(), flags = r.val<uint32_t>();
    int64_t hdr[7];
    for (auto &v : hdr) v = r.val<int64_t>();
    if (version != 1) return qh_fail(c, QH_EINVAL, "state blob of another version");
    if (hdr[0] != m.Nn || hdr[1] != m.Ne || hdr[2] != m.Nf || hdr[3] != m.Nt || hdr[4] != c->A.n ||
        hdr[5] != (int64_t)c->species.size())
        return qh_fail(c, QH_EINVAL, "state blob of another mesh, boundary or species list");
    const int64_t ni = c->A.n;
    const bool wave = flags & 1u, has_d = flags & 2u;
    auto f64 = [&](int64_t k) { return reinterpret_cast<const double *>(r.take(8 * k)); };
    auto i64 = [&](int64_t k) { return reinterpret_cast<const int64_t *>(r.take(8 * k)); };
    const double *e = f64(m.Ne);
    const int64_t *b = i64(m.Nf), *Q = i64(m.Nn), *Qbg = i64(m.Nn);
    const double *ep = wave ? f64(ni) : nullptr;
    const int64_t *gp = wave ? i64(m.Ne) : nullptr;
    const double *d = has_d ? f64(m.Nn) : nullptr;
    struct Sp {
        int64_t n, next;
        const float *f[6];
        const int32_t *tet, *id;
    };
    std::vector<Sp> sp(c->species.size());
    for (size_t k = 0; k < sp.size() && r.ok; ++k) {
        const double qm = r.val<double>();
        const int32_t z = r.val<int32_t>();
        r.val<int32_t>();
        sp[k].n = r.val<int64_t>();
        sp[k].next = r.val<int64_t>();
        if (qm != c->species[k].qm || z != c->species[k].z)
            return qh_fail(c, QH_EINVAL, "species " + std::to_string(k) + " differs from the saved one");
        // counts and ids are int32 on the device: anything else is a corrupted blob (and checked
        // before any size below is formed from it)
        if (sp[k].n < 0 || sp[k].n >= ((int64_t)1 << 31) || sp[k].next < sp[k].n || sp[k].next >= ((int64_t)1 << 31))
            return qh_fail(c, QH_EINVAL, "state blob: species " + std::to_string(k) + " count or next id out of range");
        for (auto &a : sp[k].f) a = reinterpret_cast<const float *>(r.take(4 * sp[k].n));
        sp[k].tet = reinterpret_cast<const int32_t *>(r.take(4 * sp[k].n));
        sp[k].id = reinterpret_cast<const int32_t *>(r.take(4 * sp[k].n));
    }
    if (!r.ok || r.n != len - 4) return qh_fail(c, QH_EINVAL, "state blob has the wrong length");
    for (const Sp &s : sp)
        for (int64_t i = 0; i < s.n; ++i)
            if (s.tet[i] < 0 || s.tet[i] >= m.Nt) return qh_fail(c, QH_EINVAL, "state blob: tet id out of range");
    // everything checked; device storage reserved before anything changes, so a failed
    // allocation leaves the context as it was
    int rc;
    for (size_t k = 0; k < sp.size(); ++k)
        if ((rc = reserve_species(c, c->species[k], sp[k].n, c->species[k].n))) return rc;
    if (has_d && !c->dbnd && (rc = qh_alloc(c, &c->dbnd, m.Nn))) return rc;
    // apply
    std::vector<double> ecopy(e, e + m.Ne);
    std::vector<int64_t> bcopy(b, b + m.Nf);
    if ((rc = set_fields(c, ecopy.data(), bcopy.data()))) return rc;
    for (size_t k = 0; k < sp.size(); ++k) {
        std::vector<float> x(3 * sp[k].n), v(3 * sp[k].n);
        for (int64_t i = 0; i < sp[k].n; ++i)
            for (int dd = 0; dd < 3; ++dd) x[3 * i + dd] = sp[k].f[dd][i], v[3 * i + dd] = sp[k].f[3 + dd][i];
        if ((rc = upload_species(c, (int32_t)k, sp[k].n, x.data(), v.data(), sp[k].tet, sp[k].id, sp[k].next))) return rc;
    }
    QH_HIP(c, hipMemcpy(c->Q, Q, 8 * m.Nn, hipMemcpyHostToDevice));
    QH_HIP(c, hipMemcpy(c->Q_old, Q, 8 * m.Nn, hipMemcpyHostToDevice));
    QH_HIP(c, hipMemcpy(c->Q_bg, Qbg, 8 * m.Nn, hipMemcpyHostToDevice));
    if (wave) {
        QH_HIP(c, hipMemcpy(c->e_prev, ep, 8 * ni, hipMemcpyHostToDevice));
        QH_HIP(c, hipMemcpy(c->g_prev, gp, 8 * m.Ne, hipMemcpyHostToDevice));
    }
    c->wave_hist = wave;
    if (has_d) QH_HIP(c, hipMemcpy(c->dbnd, d, 8 * m.Nn, hipMemcpyHostToDevice));
    c->step_index = hdr[6];
    c->fields_dirty = true;
    return QH_OK;
}

int qh_precond_save(qh_ctx *c, void *buf, size_t *len) {
    if (!c || !len) return QH_EINVAL;
    if (!buf) {
        *len = kBlobSize;
        return QH_OK;
    }
    if (*len < kBlobSize) return qh_fail(c, QH_EINVAL, "blob buffer smaller than the size qh_precond_save(NULL) gives");
    std::vector<float> w(QH_MLP_NPARAM);
    int rc = qh_precond_get_weights(c, w.data(), QH_MLP_NPARAM);
    if (rc) return rc;
    unsigned char *p = static_cast<unsigned char *>(buf);
    const uint32_t n = QH_MLP_NPARAM;
    std::memcpy(p, kBlobMagic, 8);
    std::memcpy(p + 8, &kBlobVersion, 4);
    std::memcpy(p + 12, &n, 4);
    std::memcpy(p + 16, w.data(), 4 * (size_t)n);
    const uint32_t h = fnv1a(p + 16, 4 * (size_t)n);
    std::memcpy(p + 16 + 4 * (size_t)n, &h, 4);
    *len = kBlobSize;
    return QH_OK;
}

int qh_precond_load(qh_ctx *c, const void *buf, size_t len) {
    if (!c || !buf) return QH_EINVAL;
    const unsigned char *p = static_cast<const unsigned char *>(buf);
    uint32_t version = 0, n = 0, h = 0;
    if (len < 16) return qh_fail(c, QH_EINVAL, "preconditioner blob too short");
    std::memcpy(&version, p + 8, 4);
    std::memcpy(&n, p + 12, 4);
    if (std::memcmp(p, kBlobMagic, 8) != 0 || version != kBlobVersion || n != QH_MLP_NPARAM || len < kBlobSize)
        return qh_fail(c, QH_EINVAL, "not a preconditioner blob of this version and size");
    std::memcpy(&h, p + 16 + 4 * (size_t)n, 4);
    if (h != fnv1a(p + 16, 4 * (size_t)n)) return qh_fail(c, QH_EINVAL, "preconditioner blob fails its checksum");
    std::vector<float> w(n);
    std::memcpy(w.data(), p + 16, 4 * (size_t)n);
    return qh_precond_set_weights(c, w.data(), n);
}

int qh_precond_factor(qh_ctx *c, int64_t *nnz, int32_t *rows, int32_t *cols, float *vals) {
    if (!c || !nnz) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    int rc = qh_learned_setup(c);
    if (rc) return rc;
    if ((rc = qh_learned_factor(c))) return rc;
    const LearnedPrec &L = c->lp;
    *nnz = L.nnz;
    if (rows) std::copy(L.h_row.begin(), L.h_row.end(), rows);
    if (cols) std::copy(L.h_col.begin(), L.h_col.end(), cols);
    if (vals) QH_HIP(c, hipMemcpyAsync(vals, L.gval, 4 * L.nnz, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int qh_precond_apply(qh_ctx *c, const double *r, double *z) {
    if (!c || !r || !z) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    int rc = qh_learned_setup(c);
    if (rc) return rc;
    if (!c->lp.factor_valid && (rc = qh_learned_factor(c))) return rc;
    const int32_t n = c->A.n;
    int32_t nmax = std::max(c->A.n, c->K.n);
    if (c->cgx.n < nmax && (rc = qh_cg_alloc(c, c->cgx, nmax))) return rc;
    // r in the standalone solve's residual slot, z in its preconditioned slot; the r.z partials
    // go to its partial buffer (unused here)
    QH_HIP(c, hipMemcpyAsync(c->cgx.r, r, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, launch_prec_apply(c, c->cgx.r, c->cgx.z, c->cgx.partial, nullptr));
    QH_HIP(c, hipMemcpyAsync(z, c->cgx.z, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int qh_precond_loss_grad(qh_ctx *c, const float *probes, double *loss, float *grad) {
    if (!c || !probes || !loss) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    int rc = qh_learned_setup(c);
    if (rc) return rc;
    LearnedPrec &L = c->lp;
    if (!L.V && (rc = qh_alloc(c, &L.V, (int64_t)L.n * 16))) return rc;
    QH_HIP(c, hipMemcpyAsync(L.V, probes, 4 * (int64_t)L.n * 16, hipMemcpyHostToDevice, c->stream));
    if ((rc = qh_learned_loss_grad(c, L.V, grad != nullptr))) return rc;
    QH_HIP(c, hipMemcpyAsync(loss, L.loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (grad) QH_HIP(c, hipMemcpyAsync(grad, L.grad, 4 * QH_MLP_NPARAM, hipMemcpyDeviceToHost, c->stream));
    return sync(c);
}

int qh_pairs_record(qh_ctx *c, int32_t capacity) {
    if (!c || capacity < 0) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    LearnedPrec &L = c->lp;
    QH_HIP(c, hipStreamSynchronize(c->stream));
    qh_release(c, L.pair_b), qh_release(c, L.pair_x), qh_release(c, L.pair_xb);
    L.pair_cap = L.pair_n = 0;
    L.pair_rec = false;
    if (capacity == 0) return QH_OK;
    const int64_t n = c->A.n;
    int rc;
    if ((rc = qh_alloc(c, &L.pair_b, n * capacity)) || (rc = qh_alloc(c, &L.pair_x, n * capacity)) ||
        (rc = qh_alloc(c, &L.pair_xb, capacity)) || (!L.ppart && (rc = qh_alloc(c, &L.ppart, 1024)))) {
        qh_release(c, L.pair_b), qh_release(c, L.pair_x), qh_release(c, L.pair_xb);
        return rc;
    }
    L.pair_cap = capacity;
    L.pair_rec = true;
    return QH_OK;
}

int qh_pairs_add(qh_ctx *c, int32_t n_pairs, const double *rhs, const double *sol) {
    if (!c || n_pairs < 0 || (n_pairs > 0 && (!rhs || !sol))) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    LearnedPrec &L = c->lp;
    if (!L.pair_b) return qh_fail(c, QH_ESTATE, "no pair bank (qh_pairs_record first)");
    if (L.pair_n + n_pairs > L.pair_cap) return qh_fail(c, QH_EINVAL, "pair bank too small");
    const int64_t n = c->A.n;
    int32_t nmax = std::max(c->A.n, c->K.n);
    int rc;
    if (c->cgx.n < nmax && (rc = qh_cg_alloc(c, c->cgx, nmax))) return rc;
    const bool rec = L.pair_rec;
    L.pair_rec = true;
    for (int32_t k = 0; k < n_pairs; ++k) {
        QH_HIP(c, hipMemcpyAsync(c->cgx.r, rhs + k * n, 8 * n, hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(c->cgx.z, sol + k * n, 8 * n, hipMemcpyHostToDevice, c->stream));
        if ((rc = qh_learned_record_pair(c, c->cgx.r, c->cgx.z))) {
            L.pair_rec = rec;
            return rc;
        }
        QH_HIP(c, hipStreamSynchronize(c->stream));
    }
    L.pair_rec = rec;
    return QH_OK;
}

int qh_precond_pair_loss_grad(qh_ctx *c, const int32_t *idx, double *loss, float *grad) {
    if (!c || !idx || !loss) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    LearnedPrec &L = c->lp;
    for (int p = 0; p < QH_PAIR_BATCH; ++p)
        if (idx[p] < 0 || idx[p] >= L.pair_n) return qh_fail(c, QH_EINVAL, "pair index out of the bank");
    int rc = qh_learned_setup(c);
    if (rc) return rc;
    if ((rc = qh_learned_loss_grad(c, nullptr, grad != nullptr, 1.0, idx))) return rc;
    double l[3];
    QH_HIP(c, hipMemcpyAsync(l, L.loss, sizeof(l), hipMemcpyDeviceToHost, c->stream));
    if (grad) QH_HIP(c, hipMemcpyAsync(grad, L.grad, 4 * QH_MLP_NPARAM, hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    *loss = l[2];
    return QH_OK;
}

int qh_pairs_count(const qh_ctx *c, int32_t *n) {
    if (!c || !n) return QH_EINVAL;
    *n = c->lp.pair_n;
    return QH_OK;
}

int qh_precond_train(qh_ctx *c, const qh_train_params_t *P, int32_t n_pairs, const double *rhs, const double *sol,
                     qh_train_stats_t *st) {
    if (!c || !P || P->steps < 0 || n_pairs < 0 || (n_pairs > 0 && !rhs)) return QH_EINVAL;
    if (c->host_only) return qh_fail(c, QH_ESTATE, "host-only context has no device");
    if (!c->assembled) return qh_fail(c, QH_ESTATE, "mesh and physics first");
    int rc = qh_learned_setup(c);
    if (rc) return rc;
    LearnedPrec &L = c->lp;
    const int32_t n = L.n;
    if (!L.V && (rc = qh_alloc(c, &L.V, (int64_t)n * 16))) return rc;
    if (!L.best_w && (rc = qh_alloc(c, &L.best_w, QH_MLP_NPARAM))) return rc;
    if (L.adam_t == 0) {
        QH_HIP(c, hipMemsetAsync(L.adam_m, 0, 4 * QH_MLP_NPARAM, c->stream));
        QH_HIP(c, hipMemsetAsync(L.adam_v, 0, 4 * QH_MLP_NPARAM, c->stream));
    }
    int32_t nmax = std::max(c->A.n, c->K.n);
    if (c->cgx.n < nmax && (rc = qh_cg_alloc(c, c->cgx, nmax))) return rc;
    CgWork w = c->cgx;
    w.n = c->A.n;
    const int n_val = std::min<int32_t>(n_pairs, 2);
    auto validate = [&](bool learned, int *iters) -> int {
        int tot = 0;
        for (int k = 0; k < n_val; ++k) {
            QH_HIP(c, hipMemcpyAsync(w.b, rhs + (int64_t)k * n, 8 * (int64_t)n, hipMemcpyHostToDevice, c->stream));
            QH_HIP(c, hipMemsetAsync(w.x, 0, 8 * (int64_t)n, c->stream));
            if (!learned) QH_HIP(c, launch_diag_inv(c, c->A, w.dinv));
            SolveResult r;
            int rc2 = qh_cg_solve(c, c->A, w, P->val_tol, P->val_max_it, 16, r, nullptr, false, learned);
            if (rc2) return rc2;
            tot += r.converged ? r.iters : 10 * P->val_max_it;
        }
        *iters = tot;
        return QH_OK;
    };
    hipEvent_t e0, e1;
    QH_HIP(c, hipEventCreate(&e0));
    QH_HIP(c, hipEventCreate(&e1));
    QH_HIP(c, hipEventRecord(e0, c->stream));
    qh_train_stats_t S;
    std::memset(&S, 0, sizeof(S));
    QH_HIP(c, launch_diag_inv(c, c->A, w.dinv));
    if (n_val > 0 && (rc = validate(false, &S.val_iters_jacobi))) return rc;
    int best = 1 << 30;
    if (n_val > 0) {
        if ((rc = qh_learned_factor(c)) || (rc = validate(true, &best))) return rc;
        QH_HIP(c, hipMemcpyAsync(L.best_w, L.w, 4 * QH_MLP_NPARAM, hipMemcpyDeviceToDevice, c->stream));
    }
    S.best_step = 0;
    // recorded solver pairs in the objective: a batch drawn without replacement per step
    const bool use_pairs = P->pair_weight > 0.0 && L.pair_n > 0;
    if (P->pair_weight > 0.0 && L.pair_n == 0) return qh_fail(c, QH_ESTATE, "pair weight > 0 but no recorded pairs");
    std::mt19937_64 prng(P->seed ^ 0x5eed5eedull);
    int32_t idx[QH_PAIR_BATCH];
    for (int32_t step = 1; step <= P->steps; ++step) {
        if ((rc = qh_learned_probes(c, L.V, P->seed * 1000003ull + (uint64_t)(L.adam_t + 1)))) return rc;
        if (use_pairs)
            for (int p = 0; p < QH_PAIR_BATCH; ++p) {
                // distinct pairs while the bank holds enough of them
                for (;;) {
                    idx[p] = (int32_t)(prng() % (uint64_t)L.pair_n);
                    bool dup = false;
                    for (int q = 0; q < p && L.pair_n >= QH_PAIR_BATCH; ++q) dup |= idx[q] == idx[p];
                    if (!dup) break;
                }
            }
        if ((rc = qh_learned_loss_grad(c, L.V, true, use_pairs ? P->pair_weight : 0.0, use_pairs ? idx : nullptr)))
            return rc;
        if (step == 1) {
            double lf[3];
            QH_HIP(c, hipMemcpyAsync(lf, L.loss, sizeof(lf), hipMemcpyDeviceToHost, c->stream));
            QH_HIP(c, hipStreamSynchronize(c->stream));
            S.loss_first = lf[0];
            S.pair_loss_first = use_pairs ? lf[2] : 0.0;
        }
        L.adam_t += 1;
        if ((rc = qh_learned_adam(c, P->lr, L.adam_t))) return rc;
        S.steps_done = step;
        if (n_val > 0 && P->validate_every > 0 && (step % P->validate_every == 0 || step == P->steps)) {
            int it = 0;
            if ((rc = qh_learned_factor(c)) || (rc = validate(true, &it))) return rc;
            if (it < best) {
                best = it;
                S.best_step = step;
                QH_HIP(c, hipMemcpyAsync(L.best_w, L.w, 4 * QH_MLP_NPARAM, hipMemcpyDeviceToDevice, c->stream));
            }
        }
    }
    double ll[3];
    QH_HIP(c, hipMemcpyAsync(ll, L.loss, sizeof(ll), hipMemcpyDeviceToHost, c->stream));
    if (n_val > 0) QH_HIP(c, hipMemcpyAsync(L.w, L.best_w, 4 * QH_MLP_NPARAM, hipMemcpyDeviceToDevice, c->stream));
    QH_HIP(c, hipEventRecord(e1, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    (void)hipEventElapsedTime(&S.ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    S.loss_last = ll[0];
    S.pair_loss_last = use_pairs ? ll[2] : 0.0;
    S.val_iters_best = n_val > 0 ? best : 0;
    L.factor_valid = false;
    // energy-norm error of the kept network on the validation pairs, ||x - M b||_A / ||x||_A,
    // with M b from the application kernels and the products with A on the host (FP64)
    S.val_energy_err = 0.0;
    if (n_val > 0 && sol) {
        if ((rc = qh_learned_factor(c))) return rc;
        const HostCsr &H = c->hA;
        const double tau = c->tau_assembled;
        std::vector<double> z(n), vv(n);
        double worst = 0.0;
        for (int k = 0; k < n_val; ++k) {
            QH_HIP(c, hipMemcpyAsync(w.r, rhs + (int64_t)k * n, 8 * (int64_t)n, hipMemcpyHostToDevice, c->stream));
            QH_HIP(c, launch_prec_apply(c, w.r, w.z, w.partial, nullptr));
            QH_HIP(c, hipMemcpyAsync(z.data(), w.z, 8 * (int64_t)n, hipMemcpyDeviceToHost, c->stream));
            QH_HIP(c, hipStreamSynchronize(c->stream));
            const double *x = sol + (int64_t)k * n;
            for (int32_t i = 0; i < n; ++i) vv[i] = x[i] - z[i];
            double vav = 0.0, xax = 0.0;
            for (int32_t i = 0; i < n; ++i) {
                double av = 0.0, ax = 0.0;
                for (int32_t q = H.ptr[i]; q < H.ptr[i + 1]; ++q) {
                    const double a = H.val[q] + tau * H.val2[q];
                    av += a * vv[H.col[q]];
                    ax += a * x[H.col[q]];
                }
                vav += vv[i] * av;
                xax += x[i] * ax;
            }
            worst = std::max(worst, xax > 0 ? std::sqrt(vav / xax) : 0.0);
        }
        S.val_energy_err = worst;
    }
    if (st) *st = S;
    return QH_OK;
}

int qh_matrix_info(const qh_ctx *c, int32_t which, int64_t *nrow, int64_t *ncol, int64_t *nnz) {
    if (!c || !nrow || !ncol || !nnz) return QH_EINVAL;
    if (!c->assembled) return QH_ESTATE;
    const HostCsr *h = which <= 2 ? &c->hA : which == 3 ? &c->hCMb : which == 4 ? &c->hGtM : which == 5 ? &c->hK : nullptr;
    if (!h) return QH_EINVAL;
    *nrow = h->nrow;
    *ncol = h->ncol;
    *nnz = (int64_t)h->col.size();
    return QH_OK;
}

int qh_matrix_download(const qh_ctx *c, int32_t which, int32_t *ptr, int32_t *col, double *val) {
    if (!c) return QH_EINVAL;
    if (!c->assembled) return QH_ESTATE;
    const HostCsr *h = which <= 2 ? &c->hA : which == 3 ? &c->hCMb : which == 4 ? &c->hGtM : which == 5 ? &c->hK : nullptr;
    if (!h || which < 0) return QH_EINVAL;
    if (ptr) std::copy(h->ptr.begin(), h->ptr.end(), ptr);
    if (col) std::copy(h->col.begin(), h->col.end(), col);
    if (val) {
        double tau = 0.25 * c->phys.dt * c->phys.dt;
        for (size_t j = 0; j < h->col.size(); ++j)
            val[j] = which == 0 ? h->val[j] + tau * h->val2[j] : which == 2 ? h->val2[j] : h->val[j];
    }
    return QH_OK;
}

// Per-kernel timing with HIP events on the context stream (for roofline figures).
int qh_timing_enable(qh_ctx *c, int32_t on) {
    if (!c) return QH_EINVAL;
    qh_tflush(c);
    c->timing = on != 0;
    for (int k = 0; k < 16; ++k) {
        c->t_ms[k] = 0;
        c->t_cnt[k] = 0;
    }
    return QH_OK;
}

int qh_timing_read(const qh_ctx *c, int32_t n, double *ms_total, int64_t *launches) {
    if (!c || n < 0 || n > 16) return QH_EINVAL;
    for (int k = 0; k < n; ++k) {
        if (ms_total) ms_total[k] = c->t_ms[k];
        if (launches) launches[k] = c->t_cnt[k];
    }
    return QH_OK;
}

}  // extern "C"
