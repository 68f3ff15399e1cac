// Host-side mesh complex K = {N, E, F, T} and FP64 assembly of the Hodge and mixed
// matrices (Sec. II.C). Runs once per mesh; everything the time loop needs is uploaded.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "qh_internal.h"

namespace {

const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int LF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

inline void cross(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// local edge index of the pair (i, j), i < j
inline int local_edge(int i, int j) {
    static const int tab[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
    return tab[i][j];
}

}  // namespace

std::string qh_build_mesh(HostMesh &m, int64_t Nn, const double *xyz, int64_t Nt,
                          const int32_t *tet_nodes) {
    if (Nn <= 0 || Nt <= 0 || !xyz || !tet_nodes) return "empty mesh or null pointer";
    if (Nn >= (int64_t)1 << 31 || 6 * Nt >= (int64_t)1 << 31) return "mesh too large for int32 ids";
    const bool neumann = m.neumann;  // the boundary condition is chosen before the mesh
    m = HostMesh();
    m.neumann = neumann;
    m.Nn = Nn;
    m.Nt = Nt;
    m.xyz.assign(xyz, xyz + 3 * Nn);
    m.tn.resize(4 * Nt);
    for (int64_t t = 0; t < Nt; ++t) {
        int32_t v[4] = {tet_nodes[4 * t], tet_nodes[4 * t + 1], tet_nodes[4 * t + 2], tet_nodes[4 * t + 3]};
        for (int i = 0; i < 4; ++i)
            if (v[i] < 0 || v[i] >= Nn) return "tet " + std::to_string(t) + ": vertex id out of range";
        std::sort(v, v + 4);
        for (int i = 0; i < 3; ++i)
            if (v[i] == v[i + 1]) return "tet " + std::to_string(t) + ": repeated vertex";
        std::copy(v, v + 4, &m.tn[4 * t]);
    }

    // edges: unique sorted pairs, key a * Nn + b
    std::vector<uint64_t> ek(6 * Nt);
    for (int64_t t = 0; t < Nt; ++t)
        for (int k = 0; k < 6; ++k)
            ek[6 * t + k] = (uint64_t)m.tn[4 * t + LE[k][0]] * (uint64_t)Nn + (uint64_t)m.tn[4 * t + LE[k][1]];
    std::vector<uint64_t> eu(ek);
    std::sort(eu.begin(), eu.end());
    eu.erase(std::unique(eu.begin(), eu.end()), eu.end());
    m.Ne = (int64_t)eu.size();
    m.edges.resize(2 * m.Ne);
    for (int64_t e = 0; e < m.Ne; ++e) {
        m.edges[2 * e] = (int32_t)(eu[e] / Nn);
        m.edges[2 * e + 1] = (int32_t)(eu[e] % Nn);
    }
    m.te.resize(6 * Nt);
    for (int64_t i = 0; i < 6 * Nt; ++i)
        m.te[i] = (int32_t)(std::lower_bound(eu.begin(), eu.end(), ek[i]) - eu.begin());
    auto edge_id = [&](int32_t a, int32_t b) -> int32_t {
        uint64_t k = (uint64_t)a * (uint64_t)Nn + (uint64_t)b;
        return (int32_t)(std::lower_bound(eu.begin(), eu.end(), k) - eu.begin());
    };

    // faces: unique sorted triples, 128-bit key
    using u128 = unsigned __int128;
    std::vector<u128> fk(4 * Nt);
    for (int64_t t = 0; t < Nt; ++t)
        for (int k = 0; k < 4; ++k) {
            const int32_t *v = &m.tn[4 * t];
            fk[4 * t + k] = ((u128)v[LF[k][0]] * (u128)Nn + (u128)v[LF[k][1]]) * (u128)Nn + (u128)v[LF[k][2]];
        }
    std::vector<u128> fu(fk);
    std::sort(fu.begin(), fu.end());
    fu.erase(std::unique(fu.begin(), fu.end()), fu.end());
    m.Nf = (int64_t)fu.size();
    m.faces.resize(3 * m.Nf);
    m.face_edges.resize(3 * m.Nf);
    for (int64_t f = 0; f < m.Nf; ++f) {
        u128 k = fu[f];
        int32_t c = (int32_t)(k % (u128)Nn);
        k /= (u128)Nn;
        int32_t b = (int32_t)(k % (u128)Nn);
        int32_t a = (int32_t)(k / (u128)Nn);
        m.faces[3 * f] = a;
        m.faces[3 * f + 1] = b;
        m.faces[3 * f + 2] = c;
        m.face_edges[3 * f] = edge_id(a, b);
        m.face_edges[3 * f + 1] = edge_id(a, c);
        m.face_edges[3 * f + 2] = edge_id(b, c);
    }
    m.tf.resize(4 * Nt);
    for (int64_t i = 0; i < 4 * Nt; ++i)
        m.tf[i] = (int32_t)(std::lower_bound(fu.begin(), fu.end(), fk[i]) - fu.begin());

    // neighbours through faces
    std::vector<int32_t> ft(2 * m.Nf, -1);
    for (int64_t t = 0; t < Nt; ++t)
        for (int k = 0; k < 4; ++k) {
            int32_t f = m.tf[4 * t + k];
            if (ft[2 * f] < 0) ft[2 * f] = (int32_t)t;
            else if (ft[2 * f + 1] < 0) ft[2 * f + 1] = (int32_t)t;
            else return "non-manifold mesh: face shared by more than two tets";
        }
    m.nbr.resize(4 * Nt);
    for (int64_t t = 0; t < Nt; ++t)
        for (int k = 0; k < 4; ++k) {
            int32_t f = m.tf[4 * t + k];
            m.nbr[4 * t + k] = ft[2 * f] == t ? ft[2 * f + 1] : ft[2 * f];
        }

    // walls
    m.wall_face.assign(m.Nf, 0);
    m.wall_edge.assign(m.Ne, 0);
    m.wall_node.assign(Nn, 0);
    for (int64_t f = 0; f < m.Nf; ++f)
        if (ft[2 * f + 1] < 0) {
            m.wall_face[f] = 1;
            for (int i = 0; i < 3; ++i) {
                m.wall_node[m.faces[3 * f + i]] = 1;
                m.wall_edge[m.face_edges[3 * f + i]] = 1;
            }
        }
    m.int_edge_of.assign(m.Ne, -1);
    m.int_node_of.assign(Nn, -1);
    // unknowns: everything but the walls (PEC), or everything (natural boundary)
    for (int64_t e = 0; e < m.Ne; ++e)
        if (m.neumann || !m.wall_edge[e]) {
            m.int_edge_of[e] = (int32_t)m.int_edges.size();
            m.int_edges.push_back((int32_t)e);
        }
    for (int64_t n = 0; n < Nn; ++n)
        if (m.neumann || !m.wall_node[n]) {
            m.int_node_of[n] = (int32_t)m.int_nodes.size();
            m.int_nodes.push_back((int32_t)n);
        }

    // geometry: grad lambda_i from the inverse Jacobian (rows = grad lambda_1..3)
    m.grad.resize(12 * Nt);
    m.vol.resize(Nt);
    m.cen.resize(3 * Nt);
    m.tsign.resize(Nt);
    for (int64_t t = 0; t < Nt; ++t) {
        const double *p[4];
        for (int i = 0; i < 4; ++i) p[i] = &m.xyz[3 * (int64_t)m.tn[4 * t + i]];
        double e1[3], e2[3], e3[3], c23[3], c31[3], c12[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = p[1][d] - p[0][d];
            e2[d] = p[2][d] - p[0][d];
            e3[d] = p[3][d] - p[0][d];
        }
        cross(e2, e3, c23);
        cross(e3, e1, c31);
        cross(e1, e2, c12);
        double det = dot(e1, c23);
        double scale = std::max({dot(e1, e1), dot(e2, e2), dot(e3, e3)});
        if (!(std::fabs(det) > 1e-12 * scale * std::sqrt(scale)))
            return "tet " + std::to_string(t) + ": degenerate";
        double *g = &m.grad[12 * t];
        for (int d = 0; d < 3; ++d) {
            g[3 + d] = c23[d] / det;
            g[6 + d] = c31[d] / det;
            g[9 + d] = c12[d] / det;
            g[d] = -(g[3 + d] + g[6 + d] + g[9 + d]);
            m.cen[3 * t + d] = 0.25 * (p[0][d] + p[1][d] + p[2][d] + p[3][d]);
        }
        m.vol[t] = std::fabs(det) / 6.0;
        m.tsign[t] = det > 0 ? 1 : -1;
    }

    // incidence lists
    auto build_lists = [](int64_t nrows, const std::vector<int32_t> &rowof, int per, std::vector<int32_t> &ptr,
                          std::vector<int32_t> &lst, int64_t Nt) {
        ptr.assign(nrows + 1, 0);
        for (int64_t i = 0; i < (int64_t)rowof.size(); ++i) ptr[rowof[i] + 1]++;
        for (int64_t r = 0; r < nrows; ++r) ptr[r + 1] += ptr[r];
        lst.resize(rowof.size());
        std::vector<int32_t> cur(ptr.begin(), ptr.end() - 1);
        for (int64_t i = 0; i < (int64_t)rowof.size(); ++i) {
            int64_t t = i / per, k = i % per;
            lst[cur[rowof[i]]++] = (int32_t)(t * 8 + k);
        }
        (void)Nt;
    };
    build_lists(m.Ne, m.te, 6, m.e2t_ptr, m.e2t, Nt);
    build_lists(Nn, m.tn, 4, m.n2t_ptr, m.n2t, Nt);
    m.n2e_ptr.assign(Nn + 1, 0);
    for (int64_t e = 0; e < m.Ne; ++e) {
        m.n2e_ptr[m.edges[2 * e] + 1]++;
        m.n2e_ptr[m.edges[2 * e + 1] + 1]++;
    }
    for (int64_t n = 0; n < Nn; ++n) m.n2e_ptr[n + 1] += m.n2e_ptr[n];
    m.n2e.resize(2 * m.Ne);
    {
        std::vector<int32_t> cur(m.n2e_ptr.begin(), m.n2e_ptr.end() - 1);
        for (int64_t e = 0; e < m.Ne; ++e) {
            m.n2e[cur[m.edges[2 * e]]++] = -(int32_t)(e + 1);
            m.n2e[cur[m.edges[2 * e + 1]]++] = (int32_t)(e + 1);
        }
    }
    return "";
}

namespace {

// [*eps] element block on local edges p, q: eps int W1_p . W1_q, with
// int lambda_i lambda_j = |T| (1 + delta_ij) / 20.
inline double meps_local(const double *g, double vol, double eps, int p, int q) {
    int a = LE[p][0], b = LE[p][1], c = LE[q][0], d = LE[q][1];
    auto GG = [&](int i, int j) { return dot(g + 3 * i, g + 3 * j); };
    auto LL = [](int i, int j) { return (i == j ? 2.0 : 1.0) / 20.0; };
    return eps * vol *
           (LL(a, c) * GG(b, d) - LL(a, d) * GG(b, c) - LL(b, c) * GG(a, d) + LL(b, d) * GG(a, c));
}

// curl W1_ab = 2 grad(lambda_a) x grad(lambda_b)
inline void curl_w1(const double *g, int p, double *out) {
    double c[3];
    cross(g + 3 * LE[p][0], g + 3 * LE[p][1], c);
    for (int d = 0; d < 3; ++d) out[d] = 2.0 * c[d];
}

// int_T W2_f for local face k: W2_abc = sum_i lambda_i v_i, int lambda_i = |T|/4
inline void int_w2(const double *g, double vol, int k, double *out) {
    int a = LF[k][0], b = LF[k][1], c = LF[k][2];
    double x1[3], x2[3], x3[3];
    cross(g + 3 * b, g + 3 * c, x1);
    cross(g + 3 * c, g + 3 * a, x2);
    cross(g + 3 * a, g + 3 * b, x3);
    for (int d = 0; d < 3; ++d) out[d] = 0.5 * vol * (x1[d] + x2[d] + x3[d]);
}

// Assemble one CSR whose row r collects contributions from a list of (tet, local row)
// incidences; emit(t, local_row, cols[], vals[], vals2[]) yields up to 6 entries.
template <class Emit>
void assemble_rows(int64_t nrow, const std::vector<int32_t> &rows_global,
                   const std::vector<int32_t> &inc_ptr, const std::vector<int32_t> &inc,
                   bool two, HostCsr &out, Emit emit) {
    out.nrow = nrow;
    out.ptr.assign(nrow + 1, 0);
    std::vector<std::vector<int32_t>> cols(nrow);
    std::vector<std::vector<double>> v1(nrow), v2(nrow);
    for (int64_t r = 0; r < nrow; ++r) {
        int32_t gidx = rows_global[r];
        auto &cl = cols[r];
        auto &a1 = v1[r];
        auto &a2 = v2[r];
        for (int32_t j = inc_ptr[gidx]; j < inc_ptr[gidx + 1]; ++j) {
            int32_t t = inc[j] / 8, k = inc[j] % 8;
            int32_t cc[8];
            double vv[8], ww[8];
            int cnt = emit(t, k, cc, vv, ww);
            for (int i = 0; i < cnt; ++i) {
                if (cc[i] < 0) continue;
                auto it = std::find(cl.begin(), cl.end(), cc[i]);
                if (it == cl.end()) {
                    cl.push_back(cc[i]);
                    a1.push_back(vv[i]);
                    a2.push_back(two ? ww[i] : 0.0);
                } else {
                    size_t pos = it - cl.begin();
                    a1[pos] += vv[i];
                    if (two) a2[pos] += ww[i];
                }
            }
        }
        out.ptr[r + 1] = out.ptr[r] + (int32_t)cl.size();
    }
    out.col.resize(out.ptr[nrow]);
    out.val.resize(out.ptr[nrow]);
    if (two) out.val2.resize(out.ptr[nrow]);
    for (int64_t r = 0; r < nrow; ++r) {
        auto &cl = cols[r];
        std::vector<int32_t> ord(cl.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return cl[x] < cl[y]; });
        for (size_t i = 0; i < ord.size(); ++i) {
            out.col[out.ptr[r] + i] = cl[ord[i]];
            out.val[out.ptr[r] + i] = v1[r][ord[i]];
            if (two) out.val2[out.ptr[r] + i] = v2[r][ord[i]];
        }
    }
}

}  // namespace

// Largest element eigenvalue of [*mu^-1]-curl-curl against [*eps] with eps = mu = 1. S_T = |T|
// C^T C with C the 3 x 6 matrix of the constant curls of W1 on the tet, so the nonzero
// eigenvalues of M_T^-1 S_T are those of the 3 x 3 matrix |T| C M_T^-1 C^T: a Cholesky solve with
// M_T and the largest root of a symmetric 3 x 3 characteristic polynomial (trigonometric form).
// The assembled pair's largest eigenvalue is at most the largest element one (both element
// matrices are positive semi-definite, M_T definite), and restricting to the interior edges
// only lowers it.
double qh_cfl_lambda_geo(const HostMesh &m) {
    double lmax = 0.0;
    for (int64_t t = 0; t < m.Nt; ++t) {
        const double *g = &m.grad[12 * t];
        double Mt[6][6], L[6][6] = {}, Ct[6][3];
        for (int p = 0; p < 6; ++p) {
            curl_w1(g, p, Ct[p]);
            for (int q = 0; q < 6; ++q) Mt[p][q] = meps_local(g, m.vol[t], 1.0, p, q);
        }
        for (int i = 0; i < 6; ++i)  // Cholesky M_T = L L^T
            for (int j = 0; j <= i; ++j) {
                double s = Mt[i][j];
                for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
                L[i][j] = i == j ? std::sqrt(std::max(s, 1e-300)) : s / L[j][j];
            }
        double X[6][3];  // X = M_T^-1 C^T
        for (int c = 0; c < 3; ++c) {
            double y[6];
            for (int i = 0; i < 6; ++i) {
                double s = Ct[i][c];
                for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
                y[i] = s / L[i][i];
            }
            for (int i = 5; i >= 0; --i) {
                double s = y[i];
                for (int k = i + 1; k < 6; ++k) s -= L[k][i] * X[k][c];
                X[i][c] = s / L[i][i];
            }
        }
        double B[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int i = 0; i < 6; ++i) s += Ct[i][a] * X[i][b];
                B[a][b] = m.vol[t] * s;
            }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < a; ++b) B[a][b] = B[b][a] = 0.5 * (B[a][b] + B[b][a]);
        const double p1 = B[0][1] * B[0][1] + B[0][2] * B[0][2] + B[1][2] * B[1][2];
        const double q = (B[0][0] + B[1][1] + B[2][2]) / 3.0;
        const double p2 = (B[0][0] - q) * (B[0][0] - q) + (B[1][1] - q) * (B[1][1] - q) + (B[2][2] - q) * (B[2][2] - q) + 2.0 * p1;
        double lam = q;
        if (p2 > 0.0) {
            const double p = std::sqrt(p2 / 6.0);
            double D[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) D[a][b] = (B[a][b] - (a == b ? q : 0.0)) / p;
            const double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
                               D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                               D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
            const double r = std::min(1.0, std::max(-1.0, 0.5 * det));
            lam = q + 2.0 * p * std::cos(std::acos(r) / 3.0);
        }
        lmax = std::max(lmax, lam);
    }
    return lmax;
}

void qh_assemble(const HostMesh &m, double eps0, double mu0, HostCsr &A, HostCsr &CMb, HostCsr &GtM,
                 HostCsr &K) {
    const double *G = m.grad.data();
    // A pattern: val = [*eps], val2 = S = mu^-1 int curl W1_p . curl W1_q
    assemble_rows((int64_t)m.int_edges.size(), m.int_edges, m.e2t_ptr, m.e2t, true, A,
                  [&](int32_t t, int p, int32_t *cc, double *vv, double *ww) {
                      const double *g = G + 12 * (int64_t)t;
                      double cp[3], cq[3];
                      curl_w1(g, p, cp);
                      for (int q = 0; q < 6; ++q) {
                          cc[q] = m.int_edge_of[m.te[6 * (int64_t)t + q]];
                          vv[q] = meps_local(g, m.vol[t], eps0, p, q);
                          curl_w1(g, q, cq);
                          ww[q] = m.vol[t] / mu0 * dot(cp, cq);
                      }
                      return 6;
                  });
    A.ncol = A.nrow;
    // C^T [*mu^-1]: mu^-1 int curl W1_e . W2_f  (interior edges x all faces)
    assemble_rows((int64_t)m.int_edges.size(), m.int_edges, m.e2t_ptr, m.e2t, false, CMb,
                  [&](int32_t t, int p, int32_t *cc, double *vv, double *) {
                      const double *g = G + 12 * (int64_t)t;
                      double cp[3], w[3];
                      curl_w1(g, p, cp);
                      for (int k = 0; k < 4; ++k) {
                          cc[k] = m.tf[4 * (int64_t)t + k];
                          int_w2(g, m.vol[t], k, w);
                          vv[k] = dot(cp, w) / mu0;
                      }
                      return 4;
                  });
    CMb.ncol = m.Nf;
    // G^T [*eps]: eps int grad(lambda_n) . W1_e = eps |T|/4 grad(l_n).(grad(l_b) - grad(l_a))
    assemble_rows((int64_t)m.int_nodes.size(), m.int_nodes, m.n2t_ptr, m.n2t, false, GtM,
                  [&](int32_t t, int i, int32_t *cc, double *vv, double *) {
                      const double *g = G + 12 * (int64_t)t;
                      for (int q = 0; q < 6; ++q) {
                          int a = LE[q][0], b = LE[q][1];
                          cc[q] = m.int_edge_of[m.te[6 * (int64_t)t + q]];
                          vv[q] = eps0 * m.vol[t] * 0.25 * (dot(g + 3 * i, g + 3 * b) - dot(g + 3 * i, g + 3 * a));
                      }
                      return 6;
                  });
    GtM.ncol = (int64_t)m.int_edges.size();
    // K = eps sum |T| grad(l_i) . grad(l_j) (interior nodes)
    assemble_rows((int64_t)m.int_nodes.size(), m.int_nodes, m.n2t_ptr, m.n2t, false, K,
                  [&](int32_t t, int i, int32_t *cc, double *vv, double *) {
                      const double *g = G + 12 * (int64_t)t;
                      for (int j = 0; j < 4; ++j) {
                          cc[j] = m.int_node_of[m.tn[4 * (int64_t)t + j]];
                          vv[j] = eps0 * m.vol[t] * dot(g + 3 * i, g + 3 * j);
                      }
                      return 4;
                  });
    K.ncol = K.nrow;
    (void)local_edge;
}
