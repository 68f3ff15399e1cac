/* FP64 oracle for the particle half of one PIC cycle.
 *
 * TEST INFRASTRUCTURE ONLY: the product library never links or calls this file.
 *
 * Follows the paper's point-particle model (Sec. II.A: rho = q sum delta(r - r_p),
 * J = q sum v_p delta(r - r_p), Lorentz force q(E + v x B)), with E and B read from
 * the Whitney expansions E = sum e_i W1_i, B = sum b_i W2_i (Sec. II.C), and the
 * time-integrated current as the path integral of W1 along each particle's path
 * (Sec. IV.B.1, the definition of G^n and rho^n = -[grad]^T G^n).
 *
 * Plain and serial per particle; threads only split the particle loop and keep
 * private integer accumulators, which are summed at the end (integer sums do not
 * depend on order, so the result equals the serial one bit for bit).
 *
 * Readings taken where the paper is silent:
 *   - push: non-relativistic Boris, v at half steps (the paper uses a 4th-order Adams
 *     method whose details are in another paper);
 *   - path: the straight line x^n -> x^n + dt v^{n+1/2}, broken at faces and walls;
 *   - walls: specular reflection of the remaining displacement and of v, or (absorbing
 *     walls) the particle stops at the wall point and leaves the domain: its path up to
 *     the wall is deposited, its charge is not (it leaves through the wall);
 *   - exit face: smallest exit parameter, ties to the lowest local index; the face
 *     just entered is never an exit candidate in the tet it leads into;
 *   - fixed point: Lambda_i = round-half-even(lambda_i * 2^F), clamped to [0, 2^F];
 *     the largest coordinate (first one on ties) takes 2^F minus the others; at a
 *     face point the coordinate of the vertex opposite the face is forced to 0 and
 *     the vector is carried into the next tet by global vertex id;
 *   - per straight piece inside a tet, edge a->b gets z(L_a^0 L_b^1 - L_a^1 L_b^0),
 *     which is 2^{2F} times the line integral of W1_ab between the quantised end
 *     points; each node gets z 2^F L_n at the particle's final position.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t Nn, Ne, Nf, Nt;
    const int64_t *tet_nodes; /* Nt*4, ascending */
    const int64_t *tet_edges; /* Nt*6, local edge order 01 02 03 12 13 23 */
    const int64_t *tet_faces; /* Nt*4, face k opposite local vertex k */
    const int64_t *tet_nbr;   /* Nt*4, -1 = wall */
    const double *minv;       /* Nt*16, lambda_i(r) = m[4i] + m[4i+1..3] . r */
} orc_mesh;

static const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
static const int LF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void lam_of(const orc_mesh *m, int64_t t, const double *r, double *lam) {
    const double *M = m->minv + 16 * t;
    for (int i = 0; i < 4; ++i)
        lam[i] = M[4 * i] + M[4 * i + 1] * r[0] + M[4 * i + 2] * r[1] + M[4 * i + 3] * r[2];
}

static const double *grad_of(const orc_mesh *m, int64_t t, int i) { return m->minv + 16 * t + 4 * i + 1; }

/* E(r) = sum_e e_e (lambda_a grad lambda_b - lambda_b grad lambda_a) */
static void gather_E(const orc_mesh *m, const double *e, int64_t t, const double *r, double *E) {
    double lam[4];
    lam_of(m, t, r, lam);
    E[0] = E[1] = E[2] = 0.0;
    for (int k = 0; k < 6; ++k) {
        int a = LE[k][0], b = LE[k][1];
        double c = e[m->tet_edges[6 * t + k]];
        const double *ga = grad_of(m, t, a), *gb = grad_of(m, t, b);
        for (int d = 0; d < 3; ++d) E[d] += c * (lam[a] * gb[d] - lam[b] * ga[d]);
    }
}

/* B(r) = sum_f b_f 2(la gb x gc + lb gc x ga + lc ga x gb) */
static void gather_B(const orc_mesh *m, const double *b, int64_t t, const double *r, double *B) {
    double lam[4], x1[3], x2[3], x3[3];
    lam_of(m, t, r, lam);
    B[0] = B[1] = B[2] = 0.0;
    for (int k = 0; k < 4; ++k) {
        int a = LF[k][0], bb = LF[k][1], c = LF[k][2];
        double coef = b[m->tet_faces[4 * t + k]];
        cross3(grad_of(m, t, bb), grad_of(m, t, c), x1);
        cross3(grad_of(m, t, c), grad_of(m, t, a), x2);
        cross3(grad_of(m, t, a), grad_of(m, t, bb), x3);
        for (int d = 0; d < 3; ++d)
            B[d] += coef * 2.0 * (lam[a] * x1[d] + lam[bb] * x2[d] + lam[c] * x3[d]);
    }
}

/* Boris (1970): half electric kick, magnetic rotation, half electric kick. */
static void boris(double *v, const double *E, const double *B, double qm, double dt) {
    double h = 0.5 * qm * dt, vm[3], t[3], s[3], vp[3], c[3];
    for (int d = 0; d < 3; ++d) { vm[d] = v[d] + h * E[d]; t[d] = h * B[d]; }
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int d = 0; d < 3; ++d) s[d] = 2.0 * t[d] / (1.0 + tt);
    cross3(vm, t, c);
    for (int d = 0; d < 3; ++d) vp[d] = vm[d] + c[d];
    cross3(vp, s, c);
    for (int d = 0; d < 3; ++d) v[d] = vm[d] + c[d] + h * E[d];
}

static void quantize(const double *lam, int forced, int F, int64_t *L) {
    const int64_t S = (int64_t)1 << F;
    for (int i = 0; i < 4; ++i) {
        if (i == forced) { L[i] = 0; continue; }
        double q = nearbyint(lam[i] * (double)S); /* default rounding: half to even */
        if (q < 0.0) q = 0.0;
        if (q > (double)S) q = (double)S;
        L[i] = (int64_t)q;
    }
    int im = 0;
    for (int i = 1; i < 4; ++i)
        if (L[i] > L[im]) im = i;
    int64_t rest = 0;
    for (int i = 0; i < 4; ++i)
        if (i != im) rest += L[i];
    L[im] = S - rest;
}

typedef struct {
    int64_t *g, *Q;
    int64_t lost, crossings, wall_hits;
    /* optional serial segment dump */
    int64_t cap, count;
    int64_t *seg_tet, *seg_l0, *seg_l1, *seg_pid;
} acc_t;

static void deposit_segment(const orc_mesh *m, acc_t *A, int64_t t, const int64_t *L0,
                            const int64_t *L1, int64_t z, int64_t pid) {
    for (int k = 0; k < 6; ++k) {
        int a = LE[k][0], b = LE[k][1];
        A->g[m->tet_edges[6 * t + k]] += z * (L0[a] * L1[b] - L1[a] * L0[b]);
    }
    if (A->cap > 0 && A->count < A->cap) {
        int64_t s = A->count++;
        A->seg_tet[s] = t;
        A->seg_pid[s] = pid;
        for (int i = 0; i < 4; ++i) { A->seg_l0[4 * s + i] = L0[i]; A->seg_l1[4 * s + i] = L1[i]; }
    }
}

static void one_particle(const orc_mesh *m, const double *e, const double *b, double *x,
                         double *v, int64_t *tet, double qm, double dt, int64_t z, int F,
                         int max_seg, int absorb, acc_t *A, int64_t pid, int32_t *lost_flag) {
    int64_t t = *tet;
    double E[3], B[3], lam[4], lq[4], p[3], q[3], rem[3];
    gather_E(m, e, t, x, E);
    gather_B(m, b, t, x, B);
    boris(v, E, B, qm, dt);
    for (int d = 0; d < 3; ++d) { p[d] = x[d]; rem[d] = dt * v[d]; }

    int64_t Lprev[4], Lc[4];
    lam_of(m, t, p, lam);
    quantize(lam, -1, F, Lprev);
    int entry = -1, nseg = 0;
    *lost_flag = 0;
    for (;;) {
        for (int d = 0; d < 3; ++d) q[d] = p[d] + rem[d];
        lam_of(m, t, p, lam);
        lam_of(m, t, q, lq);
        int k = -1;
        double smin = 2.0;
        for (int i = 0; i < 4; ++i) {
            if (i == entry || !(lq[i] < 0.0)) continue;
            double s = lam[i] <= 0.0 ? 0.0 : lam[i] / (lam[i] - lq[i]);
            if (s < smin) { smin = s; k = i; }
        }
        if (k < 0) { for (int d = 0; d < 3; ++d) p[d] = q[d]; break; }
        if (nseg >= max_seg - 1) { *lost_flag = 1; A->lost++; break; }
        double pc[3];
        for (int d = 0; d < 3; ++d) pc[d] = p[d] + smin * rem[d];
        lam_of(m, t, pc, lam);
        quantize(lam, k, F, Lc);
        deposit_segment(m, A, t, Lprev, Lc, z, pid);
        ++nseg;
        for (int d = 0; d < 3; ++d) { rem[d] *= (1.0 - smin); p[d] = pc[d]; }
        int64_t nb = m->tet_nbr[4 * t + k];
        if (nb >= 0) {
            /* carry Lambda by global vertex id; the vertex new to nb gets 0 */
            int64_t Ln[4];
            int new_local = -1;
            for (int j = 0; j < 4; ++j) {
                int64_t gid = m->tet_nodes[4 * nb + j];
                Ln[j] = 0;
                int found = 0;
                for (int i = 0; i < 4; ++i)
                    if (m->tet_nodes[4 * t + i] == gid) { Ln[j] = Lc[i]; found = 1; }
                if (!found) new_local = j;
            }
            memcpy(Lprev, Ln, sizeof Ln);
            entry = new_local;
            t = nb;
            A->crossings++;
        } else if (absorb) {
            for (int d = 0; d < 3; ++d) x[d] = p[d];
            *tet = t;
            *lost_flag = 2;
            A->wall_hits++;
            return;
        } else {
            /* specular reflection about the wall plane (normal along grad lambda_k) */
            const double *n = grad_of(m, t, k);
            double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
            double rn = (rem[0] * n[0] + rem[1] * n[1] + rem[2] * n[2]) / nn;
            double vn = (v[0] * n[0] + v[1] * n[1] + v[2] * n[2]) / nn;
            for (int d = 0; d < 3; ++d) { rem[d] -= 2.0 * rn * n[d]; v[d] -= 2.0 * vn * n[d]; }
            memcpy(Lprev, Lc, sizeof Lc);
            entry = k;
            A->wall_hits++;
        }
    }
    int64_t Lend[4];
    lam_of(m, t, p, lam);
    quantize(lam, -1, F, Lend);
    deposit_segment(m, A, t, Lprev, Lend, z, pid);
    const int64_t S = (int64_t)1 << F;
    for (int i = 0; i < 4; ++i) A->Q[m->tet_nodes[4 * t + i]] += z * S * Lend[i];
    for (int d = 0; d < 3; ++d) x[d] = p[d];
    *tet = t;
}

/* One push + walk + deposit for np particles.
 * x, v: 3*np (in/out), tet: np (in/out). g (Ne) and Q (Nn) are ADDED to.
 * lost_flags: 1 = hit the piece cap, 2 = absorbed at a wall (absorb != 0).
 * seg_cap > 0 runs serially and records the straight pieces in particle order.
 * Returns the number of particles that hit the piece cap. */
int64_t orc_push(const orc_mesh *m, const double *e, const double *b, int64_t np, double *x,
                 double *v, int64_t *tet, double qm, double dt, int64_t z, int F, int max_seg, int absorb,
                 int64_t *g, int64_t *Q, int32_t *lost_flags, int64_t *stats /* crossings, wall hits */,
                 int64_t seg_cap, int64_t *seg_count, int64_t *seg_tet, int64_t *seg_l0,
                 int64_t *seg_l1, int64_t *seg_pid, int nthreads) {
    int64_t lost = 0, cross = 0, walls = 0;
    if (seg_cap > 0) nthreads = 1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(+ : lost, cross, walls)
#endif
    {
        acc_t A;
        memset(&A, 0, sizeof A);
        A.g = (int64_t *)calloc((size_t)m->Ne, sizeof(int64_t));
        A.Q = (int64_t *)calloc((size_t)m->Nn, sizeof(int64_t));
        A.cap = seg_cap;
        A.seg_tet = seg_tet; A.seg_l0 = seg_l0; A.seg_l1 = seg_l1; A.seg_pid = seg_pid;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t i = 0; i < np; ++i)
            one_particle(m, e, b, x + 3 * i, v + 3 * i, tet + i, qm, dt, z, F, max_seg, absorb, &A, i,
                         lost_flags + i);
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            for (int64_t j = 0; j < m->Ne; ++j) g[j] += A.g[j];
            for (int64_t j = 0; j < m->Nn; ++j) Q[j] += A.Q[j];
            if (seg_cap > 0 && seg_count) *seg_count = A.count;
        }
        lost += A.lost; cross += A.crossings; walls += A.wall_hits;
        free(A.g);
        free(A.Q);
    }
    if (stats) { stats[0] = cross; stats[1] = walls; }
    return lost;
}

/* Integer deposit from an explicit list of straight pieces and of charge points.
 * Piece s: tet seg_tet[s], end points l0[4s..], l1[4s..] (local vertex order), charge
 * number seg_z[s]. Point p: tet pt_tet[p], coordinates pt_l[4p..], charge number pt_z[p].
 * g (Ne) and Q (Nn) are ADDED to. */
void orc_deposit_list(const orc_mesh *m, int64_t n_seg, const int64_t *seg_tet, const int64_t *l0,
                      const int64_t *l1, const int64_t *seg_z, int64_t n_pt, const int64_t *pt_tet,
                      const int64_t *pt_l, const int64_t *pt_z, int F, int64_t *g, int64_t *Q) {
    for (int64_t s = 0; s < n_seg; ++s) {
        int64_t t = seg_tet[s];
        for (int k = 0; k < 6; ++k) {
            int a = LE[k][0], b = LE[k][1];
            g[m->tet_edges[6 * t + k]] +=
                seg_z[s] * (l0[4 * s + a] * l1[4 * s + b] - l1[4 * s + a] * l0[4 * s + b]);
        }
    }
    const int64_t S = (int64_t)1 << F;
    for (int64_t p = 0; p < n_pt; ++p)
        for (int i = 0; i < 4; ++i) Q[m->tet_nodes[4 * pt_tet[p] + i]] += pt_z[p] * S * pt_l[4 * p + i];
}

/* Quantised barycentric coordinates of points (exported for tests). */
void orc_quantize_points(const orc_mesh *m, int64_t n, const double *x, const int64_t *tet, int F,
                         int64_t *L) {
    double lam[4];
    for (int64_t i = 0; i < n; ++i) {
        lam_of(m, tet[i], x + 3 * i, lam);
        quantize(lam, -1, F, L + 4 * i);
    }
}

/* E and B at points (exported for tests). */
void orc_gather(const orc_mesh *m, const double *e, const double *b, int64_t n, const double *x,
                const int64_t *tet, double *E, double *B) {
    for (int64_t i = 0; i < n; ++i) {
        gather_E(m, e, tet[i], x + 3 * i, E + 3 * i);
        gather_B(m, b, tet[i], x + 3 * i, B + 3 * i);
    }
}
