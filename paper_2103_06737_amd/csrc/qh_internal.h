// Internal declarations shared by the libqh translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qh.h"

constexpr int QH_FBITS = 20;                  // fixed-point bits of barycentric coordinates
constexpr int QH_SCALE = 1 << QH_FBITS;
constexpr int QH_MAX_PIECES = 64;             // straight pieces per particle per step
constexpr int QH_COUNTER_SLOTS = 256;         // spread of the per-block event counters
// Counters past the 4 * QH_COUNTER_SLOTS per-block slots (crossings, wall hits, lost, posted
// pieces): the step's continuity and D b violations, cleared every step, then the totals of a
// whole qh_pic_step call (cleared when the call starts): headroom overflows, lost particles,
// continuity and D b violations.
enum { QH_CNT_CONT = 0, QH_CNT_DIVB = 1, QH_CNT_STEP_END = 3, QH_CNT_HEADROOM_CALL = 3, QH_CNT_LOST_CALL = 4,
       QH_CNT_CONT_CALL = 5, QH_CNT_DIVB_CALL = 6, QH_CNT_ALL = 8 };
constexpr int QH_CHUNK = 512;                 // particles per block of the particle kernels
constexpr int kMailTets = 128;                // tets per deposit mailbox
constexpr int kMailCap = 1024;                // records per mailbox
constexpr int kMailWords = 5;                 // int32 words per record: both points packed (4), tet | end << 31 (1)

// ---------------------------------------------------------------------------------------
// Host-side mesh complex and FP64 assembly (qh_mesh.hip)
struct HostCsr {
    int64_t nrow = 0, ncol = 0;
    std::vector<int32_t> ptr, col;
    std::vector<double> val, val2;  // val2: second value array on the same pattern
};

struct HostMesh {
    int64_t Nn = 0, Ne = 0, Nf = 0, Nt = 0;
    bool neumann = false;                       // every edge and node is an unknown (no PEC walls)
    std::vector<double> xyz;                    // 3*Nn
    std::vector<int32_t> tn;                    // 4*Nt, ascending
    std::vector<int32_t> te;                    // 6*Nt
    std::vector<int32_t> tf;                    // 4*Nt
    std::vector<int32_t> nbr;                   // 4*Nt
    std::vector<int8_t> tsign;                  // Nt, orientation of the sorted tet
    std::vector<int32_t> edges;                 // 2*Ne
    std::vector<int32_t> faces;                 // 3*Nf
    std::vector<int32_t> face_edges;            // 3*Nf: [ab, ac, bc]
    std::vector<uint8_t> wall_edge, wall_node, wall_face;
    std::vector<int32_t> int_edge_of, int_node_of;  // global -> interior index or -1
    std::vector<int32_t> int_edges, int_nodes;      // interior index -> global
    std::vector<double> grad;                   // 12*Nt: grad lambda_0..3
    std::vector<double> vol;                    // Nt
    std::vector<double> cen;                    // 3*Nt
    // incidence lists
    std::vector<int32_t> e2t_ptr, e2t;          // edge -> (tet*8 + local edge)
    std::vector<int32_t> n2t_ptr, n2t;          // node -> (tet*4 + local vertex)
    std::vector<int32_t> n2e_ptr, n2e;          // node -> signed edge (+(e+1) head, -(e+1) tail)
};

// Build topology + geometry. Returns empty string or an error message.
std::string qh_build_mesh(HostMesh &m, int64_t n_nodes, const double *xyz, int64_t n_tets,
                          const int32_t *tet_nodes);
// Assemble: A pattern with val=[*eps], val2=S (interior edges); CMb = C^T [*mu^-1]
// (interior edges x all faces); GtM = G^T [*eps] (interior nodes x interior edges);
// K = G^T [*eps] G (interior nodes).
// Upper bound of lambda_max([*eps]^-1 S) for eps = mu = 1 (element eigenvalue bound).
double qh_cfl_lambda_geo(const HostMesh &m);
void qh_assemble(const HostMesh &m, double eps0, double mu0, HostCsr &A, HostCsr &CMb,
                 HostCsr &GtM, HostCsr &K);

// ---------------------------------------------------------------------------------------
// Device containers
// Column indices of a tiled matrix as the tiled products read them. A tile whose columns lie in
// at most four windows [w_k, w_k + 2^14) keeps each as 16 bits: the window number in the top two
// bits, the offset from its start in the low fourteen (tbase[tile] = {w_0, w_1, w_2, w_3}); a
// row couples a few index clusters (on a box mesh: the layers below, at and above it), each
// narrow. Any other tile reads the 32-bit columns (tbase[tile].x = -1). tbase == nullptr: 32-bit
// columns throughout.
struct TileCols {
    const int32_t *col;
    const uint16_t *col16;
    const int4 *tbase;
    // optional, BF16 values only: value bits << 16 | 16-bit column per entry, one load each in
    // the compact tiles (the value and column arrays still serve the others)
    const uint32_t *pk = nullptr;
    // every tile compact and non-empty: the packed words alone describe the matrix
    bool all_pk = false;
};

struct DevCsr {
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t *ptr = nullptr, *col = nullptr;
    double *val = nullptr;
    double *val2 = nullptr;
    float *val32 = nullptr; // FP32 copy of val for the mixed-precision solve (allocated on first use)
    double val32_tau = -1.0; // the context's tau when val32 was taken (A's values follow dt)
    int2 *tiles = nullptr;  // row tiles of the tiled product (qh_spmv.h)
    int32_t ntiles = 0;
    uint16_t *col16 = nullptr;  // per-tile 16-bit columns (TileCols)
    int4 *tbase = nullptr;
    int64_t nnz_c16 = 0;        // entries in tiles with 16-bit columns
    TileCols cols() const { return TileCols{col, col16, tbase}; }
};

struct Species {
    double qm = 0.0;
    int32_t z = 0;
    int64_t n = 0, cap = 0;
    int64_t next_id = 0;       // id of the next particle uploaded or injected
    float *x = nullptr, *y = nullptr, *zz = nullptr, *vx = nullptr, *vy = nullptr, *vz = nullptr;
    int32_t *tet = nullptr, *id = nullptr;
    // sort scratch (same layout)
    float *sx = nullptr, *sy = nullptr, *sz = nullptr, *svx = nullptr, *svy = nullptr, *svz = nullptr;
    int32_t *stet = nullptr, *sid = nullptr;
    int32_t *own = nullptr;    // owned tet range per particle block (see qh_particles.hip)
    uint16_t *ovf = nullptr;   // per particle block: overflow list of the walk queue
};

// Krylov workspace for one system.
struct CgWork {
    int32_t n = 0;
    double *x = nullptr, *r = nullptr, *z = nullptr, *q = nullptr, *p0 = nullptr, *p1 = nullptr;
    double *dinv = nullptr, *b = nullptr;
    double *partial = nullptr;  // reduction partials
    double *scal = nullptr;     // device scalars (see qh_solver.hip)
    unsigned int *counter = nullptr;
    int32_t *flags = nullptr;   // [0] done, [1] iterations
    // iterations of the last converged solve (Jacobi, learned), FP64 and mixed precision, and
    // for the mixed one its iterations per 1e-4 of residual reduction (0: unknown)
    int32_t last_iters[2] = {0, 0};
    int32_t last_mixed[2] = {0, 0};
    int32_t last_segment[2] = {0, 0};
    // mixed-precision solve: FP32 inner iterate, residual, preconditioned residual, directions,
    // inverse diagonal (allocated on first use, n32 entries)
    float *x32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr, *dinv32 = nullptr;
    int32_t n32 = 0;
};

// Learned preconditioner state (qh_learned.hip)
struct LearnedPrec {
    bool built = false, have_weights = false, factor_valid = false;
    double tau = -1.0;
    int32_t n = 0;
    int64_t nnz = 0;                         // entries of G (lower triangle of A's pattern)
    std::vector<int32_t> h_row, h_col;
    int32_t *gptr = nullptr, *gcol = nullptr, *grow = nullptr;   // G, row-major
    int32_t *tptr = nullptr, *tcol = nullptr, *tsrc = nullptr;   // G^T rows; tsrc: entry of G
    int2 *gtiles = nullptr, *ttiles = nullptr;                   // row tiles of G and G^T
    int32_t ngtiles = 0, nttiles = 0;
    uint16_t *gcol16 = nullptr, *tcol16 = nullptr;               // their compact columns (TileCols)
    int4 *gtbase = nullptr, *ttbase = nullptr;
    int64_t nnz_c16 = 0;                                         // entries of G and G^T in such tiles
    bool g_all_pk = false, t_all_pk = false;                     // every tile compact and non-empty
    unsigned short *feats = nullptr;         // nnz x 16 BF16 features
    float *gscale = nullptr;                 // 1/sqrt(A_jj) (1/sqrt(A_ii) on the diagonal)
    float *gval = nullptr, *tval = nullptr, *o = nullptr, *d_o = nullptr;
    uint16_t *gval_h = nullptr, *tval_h = nullptr;  // BF16 copies of G and G^T for the application
    uint32_t *gpk = nullptr, *tpk = nullptr;         // the same packed with their 16-bit columns
    double *y = nullptr;
    float *y32 = nullptr;  // the application's intermediate G r on FP32 vectors (allocated on first use)
    float *w = nullptr, *best_w = nullptr, *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;
    float *gpart = nullptr, *W = nullptr, *AW = nullptr, *V = nullptr;
    double *tpart = nullptr, *lpart = nullptr, *loss = nullptr, *gpart2 = nullptr;
    int32_t adam_t = 0;
    // (rhs, solution) pairs of the edge system recorded from field steps, FP32, pair-major
    // [k][n], with x.b of each (= ||x||_A^2 for A x = b), and the training's pair products
    float *pair_b = nullptr, *pair_x = nullptr;
    double *pair_xb = nullptr;
    int32_t pair_cap = 0, pair_n = 0;
    bool pair_rec = false;
    float *PB = nullptr, *PX = nullptr, *PY = nullptr, *PV = nullptr, *PAV = nullptr, *PGAV = nullptr;
    double *ppart = nullptr, *pw = nullptr;
};

struct qh_ctx {
    int device = 0;
    int32_t bc = QH_BC_PEC;  // field boundary condition (qh_set_boundary, before the mesh)
    int32_t walls = QH_WALLS_REFLECT;  // what particles do at the walls (qh_set_walls)
    uint8_t *wall_node_d = nullptr;    // geometric wall nodes (Nn)
    bool host_only = false;  // device < 0: host mesh and assembly only (no GPU calls)
    hipStream_t stream = nullptr;
    std::string err;
    bool have_mesh = false, have_phys = false, have_fields = false;

    HostMesh hm;
    HostCsr hA, hCMb, hGtM, hK;
    qh_phys_t phys{};

    // device mesh records
    float4 *geo = nullptr;       // 3*Nt: (g1, cx) (g2, cy) (g3, cz), FP32
    int4 *tnodes = nullptr;      // Nt
    int32_t *tedges = nullptr;   // 8*Nt (6 used)
    int4 *tnbr = nullptr;        // Nt
    int32_t *tfaces = nullptr;   // 4*Nt
    int8_t *tsign = nullptr;     // Nt
    float4 *frec = nullptr;      // 3*Nt: (alpha, beta_x) (beta_y, beta_z, B_x, B_y) (B_z, -, -, -)
    int32_t *face_edges = nullptr;  // 3*Nf
    int32_t *int_edges = nullptr;   // interior -> global edge
    int32_t *int_nodes = nullptr;   // interior -> global node
    int32_t *int_node_of = nullptr; // global node -> interior or -1
    int32_t *edge_nodes = nullptr;  // 2*Ne
    int32_t *n2e_ptr = nullptr, *n2e = nullptr;
    int32_t *e2t_ptr = nullptr, *e2t = nullptr;  // edge -> tet*8 + local edge
    int32_t *n2t_ptr = nullptr, *n2t = nullptr;  // node -> tet*8 + local vertex
    int64_t *acc_tet = nullptr;                  // 10*Nt per-tet deposit sums, plane-major [10][Nt]
    unsigned int *mail_cnt = nullptr;            // per mailbox (run of kMailTets tets): records posted
    int32_t *mail = nullptr;                     // mailboxes: ceil(Nt / kMailTets) x kMailCap x kMailWords int32

    DevCsr A, CMb, GtM, K;  // A: val = [*eps] + tau S, val2 = [*eps]
    double *A_S = nullptr;  // S values on the pattern of A
    double *A_rhs = nullptr;  // [*eps] - tau S on the pattern of A (right-hand side)
    double tau_assembled = -1.0;
    int32_t last_refinements = 0;  // the last step's reliable updates (mixed-precision edge solve)
    bool assembled = false;

    // fields and deposits
    double *e = nullptr;                    // Ne (wall entries 0)
    double *e_old = nullptr;                // interior edges: e^n during a field update
    double *e_prev = nullptr;               // interior edges: e^{n-1} for the wave-equation update
    int64_t *g_prev = nullptr;              // Ne: the previous step's current (wave-equation update)
    bool wave_hist = false;                 // e_prev, g_prev hold the previous step's values
    // plane wave through the natural boundary (qh_set_plane_wave)
    bool pw_on = false;
    double pw_amp = 0.0, pw_f0 = 0.0, pw_sig = 0.0, pw_t0 = 0.0, pw_c = 0.0;  // amp = E0 / eta
    int32_t pw_nb = 0, pw_nn = 0, pw_nu = 0;  // boundary edges, boundary nodes, distinct point x
    int32_t *pw_ptr = nullptr, *pw_edge = nullptr;   // per boundary edge: its rule points, its unknown index
    double *pw_coef = nullptr;              // per point: weight x W1 . (n x y-hat)
    int32_t *pw_xi = nullptr;               // per point: index of its x among the distinct ones
    double *pw_xs = nullptr, *pw_tab = nullptr;      // distinct x; s' there at t^{n-1}, t^n, t^{n+1}
    double *pw_hsum = nullptr;              // per boundary edge: dt/2 (h^n + h^{n+1}) of this step
    int32_t *pw_nptr = nullptr, *pw_nlist = nullptr; // per boundary node: boundary edge index << 1 | (1: tail)
    int32_t *pw_node = nullptr;             // boundary node ids
    double *dbnd = nullptr;                 // Nn: boundary flux accumulated into the Gauss-law target
    double *e_star = nullptr;               // interior edges: edge-solve solution of the last step
    int64_t *b = nullptr;                   // Nf
    int64_t *g = nullptr;                   // Ne
    int64_t *Q = nullptr, *Q_old = nullptr, *Q_bg = nullptr;  // Nn
    int64_t *divb0 = nullptr;               // Nt
    int64_t *u_int = nullptr;               // Ne (Faraday increments)
    double *rhs_e = nullptr, *rho = nullptr;  // interior edges, interior nodes

    CgWork cge, cgn;            // cge.x holds e on the interior edges between steps
    CgWork cgx;                 // standalone solves (qh_field_solve)
    double *scratch_d = nullptr;  // small device scalars (gauss thresholds etc.)
    double *dec_e = nullptr;      // interior edge values of E_s (qh_fields_decompose)
    double cfl_lambda = -1.0;     // qh_cfl_lambda_geo of the mesh (computed on first request)
    double *xyz_d = nullptr;      // 3*Nn FP64 node coordinates (uploaded on the first energy request)
    double *energy_d = nullptr;   // energy partial sums, then the two totals
    // point location: a uniform grid of buckets over the bounding box, a seed tet per bucket
    int32_t *loc_seed = nullptr;
    float loc_lo[3] = {0, 0, 0}, loc_inv[3] = {0, 0, 0};
    int32_t loc_n[3] = {0, 0, 0};
    unsigned long long *counters = nullptr;  // 4*QH_COUNTER_SLOTS + QH_CNT_ALL (see QH_CNT_*)
    int32_t *hist = nullptr, *cursor = nullptr, *scan_tmp = nullptr;
    int32_t *perm = nullptr;   // the sort's source index per destination slot (perm_cap entries)
    int64_t perm_cap = 0;

    std::vector<Species> species;

    // segment capture
    int64_t cap_segments = 0;
    bool capture_next = false;
    unsigned long long *seg_count = nullptr;
    int32_t *seg_buf = nullptr;  // cap * 12 ints: pid species seq tet lam0[4] lam1[4]

    LearnedPrec lp;
    int last_fallbacks = 0;
    int64_t step_index = 0;
    bool fields_dirty = true;
    std::vector<void *> allocations;

    // optional per-kernel timing with HIP events on the context stream
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    struct Pending { int slot; int kernel; };
    std::vector<Pending> pending;
    double t_ms[16] = {0};
    int64_t t_cnt[16] = {0};
};

// kernel ids of the timing table
enum {
    QK_FIELD_PREP = 0, QK_PARTICLE, QK_SORT, QK_EDGE_RHS, QK_CG_SPMV, QK_CG_UPDATE, QK_CG_INIT,
    QK_GAUSS, QK_FARADAY, QK_TRUE_RES, QK_NODE_SPMV, QK_NODE_UPDATE, QK_PREC, QK_BOUNDARY, QK_NKERNELS
};
int qh_tbeg(qh_ctx *c);
void qh_tend(qh_ctx *c, int slot, int kernel);
void qh_tflush(qh_ctx *c);

// error helpers
int qh_fail(qh_ctx *c, int code, const std::string &msg);
#define QH_HIP(c, call)                                                                   \
    do {                                                                                  \
        hipError_t _e = (call);                                                           \
        if (_e != hipSuccess)                                                             \
            return qh_fail((c), QH_EHIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <class T>
int qh_alloc(qh_ctx *c, T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) return qh_fail(c, QH_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c->allocations.push_back((void *)*p);
    return QH_OK;
}

// Frees a buffer from qh_alloc before qh_destroy (the caller has synchronised its stream).
template <class T>
void qh_release(qh_ctx *c, T *&p) {
    if (!p) return;
    for (auto it = c->allocations.begin(); it != c->allocations.end(); ++it)
        if (*it == (void *)p) {
            c->allocations.erase(it);
            (void)hipFree((void *)p);
            break;
        }
    p = nullptr;
}

// ---------------------------------------------------------------------------------------
// Kernel launchers
// qh_particles.hip
void launch_field_prep(qh_ctx *c);
hipError_t launch_particle_step(qh_ctx *c, Species &s, int sidx, bool capture);
hipError_t launch_charge_deposit(qh_ctx *c, Species &s, int64_t first = 0);
hipError_t launch_own_extend(qh_ctx *c, Species &s, int32_t b0, int32_t b1);
hipError_t launch_probe(qh_ctx *c, int64_t n, const double *xyz, const int32_t *tet, double *E, double *B);
hipError_t launch_locate(qh_ctx *c, int64_t n, const float *x, const float *y, const float *z, int32_t *tet);
int qh_sort_species(qh_ctx *c, Species &s);
int64_t qh_species_blocks(int64_t n);
hipError_t launch_deposit_lists(qh_ctx *c, int64_t n_seg, const int32_t *seg_tet,
                                const int32_t *l0, const int32_t *l1, const int32_t *sz,
                                int64_t n_pt, const int32_t *pt_tet, const int32_t *pl,
                                const int32_t *pz, int64_t *g, int64_t *Q);
hipError_t launch_verify(qh_ctx *c, bool check_divb);
hipError_t launch_divb(qh_ctx *c, int64_t *out);
// Field energy (qh_diag.hip): qh_energy_parts(c) partial sums in part, out[0] electric, out[1] magnetic
int32_t qh_energy_parts(const qh_ctx *c);
hipError_t launch_field_energy(qh_ctx *c, double *part, double *out);
hipError_t launch_divb_check(qh_ctx *c, const int64_t *b, unsigned long long *bad);
hipError_t launch_fields_in(qh_ctx *c, const double *e_in, double *x);

// qh_static.hip: the deposit from explicit lists in a file-scope device array (no allocation)
size_t qh_static_scratch_bytes();
int qh_static_scratch_init(qh_ctx *c);
size_t qh_static_deposit_bytes(int64_t ne, int64_t nn, int64_t n_seg, int64_t n_pt);
int qh_static_deposit(qh_ctx *c, int64_t n_seg, const int32_t *seg_tet, const int32_t *lam0, const int32_t *lam1,
                      const int32_t *seg_z, int64_t n_pt, const int32_t *pt_tet, const int32_t *pt_lam,
                      const int32_t *pt_z, int64_t *g_out, int64_t *q_out);

// qh_solver.hip
struct SolveResult {
    int iters = 0;
    double res = 0.0;       // recomputed ||b - A x|| / ||b||
    bool converged = false; // the recurrence met the target and so did the recomputed residual
    bool true_ok = false;   // the recomputed residual meets the target
    int flag = 0;           // why the iteration stopped: 0 iteration cap, 1 target met, 2 stall rule
                            // (learned preconditioner), 3 non-finite values
    int restarts = 0;       // restarts from the iterate after the recomputed residual missed the target
    int refinements = 0;    // mixed precision: reliable updates (FP64 residuals after the start)
};
int qh_cg_alloc(qh_ctx *c, CgWork &w, int32_t n);
// Jacobi PCG on matrix M, rhs in w.b, initial guess in w.x; thr2 target on ||r||^2 set on device.
int qh_cg_solve(qh_ctx *c, const DevCsr &M, CgWork &w, double tol, int max_it, int check_every,
                SolveResult &out, const double *abs_thr2_dev, bool node_system = false, bool learned = false);
// The edge system in mixed precision: FP32 PCG with FP64 reliable updates (Jacobi or the
// learned preconditioner), stopping on the FP64 residual ||b - A x|| <= tol ||b||.
int qh_cg_solve_mixed(qh_ctx *c, DevCsr &M, CgWork &w, double tol, int max_it, int check_every,
                      SolveResult &out, bool learned);
// FP32 buffers of a CgWork for n unknowns (kept when large enough)
int qh_cg_alloc32(qh_ctx *c, CgWork &w, int32_t n);

// qh_learned.hip
int qh_learned_setup(qh_ctx *c);
int qh_learned_factor(qh_ctx *c);
unsigned qh_prec_grid(qh_ctx *c);
hipError_t launch_prec_apply(qh_ctx *c, const double *r, double *z, double *part, const int32_t *done);
// the same on FP32 vectors (the mixed-precision solve's inner iterations)
hipError_t launch_prec_apply32(qh_ctx *c, const float *r, float *z, double *part, const int32_t *done);
int qh_learned_loss_grad(qh_ctx *c, const float *V_dev, bool want_grad, double pair_weight = 0.0,
                         const int32_t *pair_idx = nullptr);
// records the edge system's (rhs, solution) into the next slot of the pair bank
int qh_learned_record_pair(qh_ctx *c, const double *rhs, const double *sol);
constexpr int QH_PAIR_BATCH = 16;  // pairs per training step
int qh_learned_adam(qh_ctx *c, float lr, int32_t t);
int qh_learned_probes(qh_ctx *c, float *V_dev, uint64_t seed);
hipError_t launch_diag_inv(qh_ctx *c, const DevCsr &M, double *dinv);
hipError_t launch_assemble_A(qh_ctx *c, double tau);
hipError_t launch_edge_rhs(qh_ctx *c);
hipError_t launch_wave_rhs(qh_ctx *c);
hipError_t launch_plane_wave(qh_ctx *c, bool wave);
hipError_t launch_gauss_rhs(qh_ctx *c, double *thr2_dev, double tol_n);
hipError_t launch_gauss_apply(qh_ctx *c);
hipError_t launch_div_e(qh_ctx *c, double *out3, double tol_n);
hipError_t launch_grad_add(qh_ctx *c, const double *delta, double *e_int);
hipError_t launch_faraday(qh_ctx *c);
hipError_t launch_true_residual(qh_ctx *c, const DevCsr &M, const double *x, const double *b,
                                double *out2 /* [0] ||b-Ax||^2 [1] ||b||^2 */);
hipError_t launch_gauss_check(qh_ctx *c, double *out3);
