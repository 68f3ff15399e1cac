/* qh.h - C ABI of libqh: one charge-conserving FEM-PIC cycle on a tetrahedral mesh with
 * the implicit quasi-Helmholtz field update, on one AMD Instinct MI355X (gfx950).
 *
 * Method: O'Connor, Crawford, Ramachandran, Luginsland, Shanker, "Quasi-Helmholtz
 * Decomposition, Gauss' Laws and Charge Conservation for Finite Element Particle-in-Cell",
 * arXiv 2103.06737. Section references below are to that paper.
 *
 * Conventions shared by every call
 *  - Status: every int-returning call returns QH_OK (0) or a negative QH_E* code; the
 *    message of the last failure is qh_last_error(ctx). Nothing throws across the ABI.
 *  - Ownership: host arrays passed in are borrowed for the duration of the call and
 *    copied; output arrays are caller-allocated with the sizes from qh_mesh_info. All
 *    device state belongs to the context and is freed by qh_destroy.
 *  - Ordering: all device work is queued on the context's HIP stream; a call returns
 *    after its results are in the caller's host buffers. A context is not thread-safe.
 *  - Mesh complex (Sec. II.C): each tet lists its 4 vertices; the library sorts them
 *    ascending. Edges [a,b] (a<b) and faces [a,b,c] (a<b<c) are numbered in lexicographic
 *    order of their vertex tuples. Edge a->b has G = -1 at a, +1 at b; face [a,b,c] has
 *    boundary [b,c] - [a,c] + [a,b]. Local edge order inside a tet: 01 02 03 12 13 23;
 *    local face k is opposite local vertex k.
 *  - Walls: every boundary face is a perfect electric conductor (n x E = 0, Sec. II.A,
 *    eq. bceq with Psi_D = 0) and a specularly reflecting particle wall. Wall edges keep
 *    e = 0, wall nodes are grounded, wall-face fluxes never change.
 *  - Fixed point: deposits are int64 in units of u_q (coulombs): a particle of charge
 *    number z at barycentric coordinates lambda adds z * 2^20 * Lambda_n to node n, with
 *    Lambda_n = lambda_n quantised to 2^-20; a straight piece adds
 *    z * (L_a^0 L_b^1 - L_a^1 L_b^0) to edge a->b (2^40 times the line integral of W1 along
 *    the piece, Sec. IV.B.1). Face fluxes b are int64 in units of u_b (webers).
 */
#ifndef QH_H
#define QH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QH_OK 0
#define QH_EINVAL (-1)    /* bad argument (null pointer, size, index out of range) */
#define QH_ENOMEM (-2)    /* device or host allocation failed */
#define QH_EHIP (-3)      /* a HIP runtime call failed */
#define QH_ENOTCONV (-4)  /* a Krylov solve hit its iteration cap; stats are still filled */
#define QH_EOVERFLOW (-5) /* fixed-point headroom exceeded: a step's int64 current on an edge or
                              charge on a node beyond 2^60 (the steps are still taken) */
#define QH_ELOST (-6)     /* a particle hit the 64-piece walk cap; it is kept, flagged */
#define QH_ESTATE (-7)    /* call out of order (e.g. a step before a mesh is uploaded) */
#define QH_EVERIFY (-8)   /* verify = 1 found a broken invariant: discrete continuity G^T g = Q^{n+1} - Q^n
                             (Sec. IV.B.1) at some node, or D b changed in some tet (Sec. IV.A); the
                             steps are still taken */

#define QH_FIELDS_FROZEN 0 /* particles only: E, B stay as uploaded */
#define QH_FIELDS_SOLVE 1  /* full cycle: implicit field update after each push */
/* full cycle with the edge update of the wave equation (eq. wave_cont, [*eps] e'' + S e = -J'),
 * Newmark beta = 1/4, gamma = 1/2: ([*eps] + tau S) e^{n+1} = [*eps](2e^n - e^{n-1})
 * - tau S (2e^n + e^{n-1}) - u_q (g^{n+1/2} - g^{n-1/2}); the same matrix, preconditioners,
 * Gauss-law correction and integer Faraday update as QH_FIELDS_SOLVE. It needs e^{n-1} and the
 * previous step's current: a step in this mode after any other step (or after fields,
 * particles or physics are set) takes the QH_FIELDS_SOLVE update and records them. */
#define QH_FIELDS_WAVE 2

#define QH_PC_JACOBI 0  /* diagonal preconditioner, conjugate gradients */
#define QH_PC_LEARNED 1 /* learned edge-local preconditioner M = G^T G, conjugate gradients, Jacobi fallback */

#define QH_SYS_EDGE 0 /* ([*eps] + dt^2/4 S) on interior edges */
#define QH_SYS_NODE 1 /* G^T [*eps] G on interior nodes (discrete Laplacian) */

typedef struct qh_ctx qh_ctx;

typedef struct {
    int64_t n_nodes, n_edges, n_faces, n_tets;
    int64_t n_int_nodes, n_int_edges; /* unknowns of the node and edge systems */
    int64_t nnz_edge, nnz_node;       /* nonzeros of the two system matrices */
    int64_t nnz_edge_c16;             /* nonzeros of the edge matrix whose column index the products
                                         read as 16 bits (one of four windows of 2^14 columns per
                                         row tile, and the offset in it; the rest: 32-bit); 0 until
                                         the matrices are assembled on the device */
    int64_t nnz_factor, nnz_factor_c16; /* entries of the learned factor G (lower triangle of the
                                         edge pattern) and of G and G^T together read with 16-bit
                                         columns; 0 until the learned preconditioner is built */
    double dt_cfl; /* explicit (leap-frog) stability bound 2 / sqrt(lambda), lambda the largest
                      element eigenvalue of S_T against [*eps]_T: at most the true explicit limit
                      2 / sqrt(lambda_max([*eps]^-1 S)) (the assembled eigenvalue never exceeds the
                      element ones), with the context's eps0, mu0 (vacuum before qh_set_physics);
                      computed on the first call (one pass over the tets on the host) */
} qh_mesh_info_t;

typedef struct {
    double eps0; /* permittivity (F/m) */
    double mu0;  /* permeability (H/m) */
    double dt;   /* time step (s) */
    double u_q;  /* coulombs per integer deposit unit (e.g. e * weight * 2^-40) */
    double u_b;  /* webers per integer face-flux unit */
} qh_phys_t;

typedef struct {
    int32_t field_mode;  /* QH_FIELDS_FROZEN, QH_FIELDS_SOLVE or QH_FIELDS_WAVE */
    int32_t sort_every;  /* counting-sort particles by tet every k steps (0 = never) */
    int32_t precond;     /* QH_PC_JACOBI or QH_PC_LEARNED */
    int32_t gauss;       /* 1: solve the discrete Gauss law each step (the method); 0: skip */
    double tol_edge;     /* relative residual of the edge solve (e.g. 1e-8) */
    double tol_node;     /* Gauss-law residual target, relative to ||rho|| + || |G^T[*eps]| |e| || */
    int32_t max_it_edge, max_it_node;
    int32_t check_every; /* iterations between host reads of the convergence flag; the first read
                            of a solve comes after as many iterations as the previous solve of
                            the same system and preconditioner took (QH_SOLVER_MIXED: a read and
                            reliable update each time the previous solve had reduced its residual
                            by another 1e-4, the last at its iteration count) */
    int32_t verify;      /* 1: check continuity and D b on the device every step */
    int32_t solver;      /* edge solve: QH_SOLVER_FP64 (0), or QH_SOLVER_MIXED (1): PCG in FP32 (FP32
                            copy of A's values and FP32 vectors, FP64 products and dot products, the
                            same preconditioner) with reliable updates in FP64 (x accumulated and
                            b - A x recomputed in FP64 between batches, replacing the FP32
                            residual), stopping on the same FP64 residual tol_edge */
} qh_step_params_t;

#define QH_SOLVER_FP64 0
#define QH_SOLVER_MIXED 1

typedef struct {
    int32_t edge_iters, node_iters; /* Krylov iterations of this step */
    double edge_res, node_res;      /* final relative residuals, recomputed in FP64 */
    double gauss_res;               /* ||rho - G^T[*eps] e|| / (||rho|| + || |G^T[*eps]| |e| ||) */
    int64_t crossings, wall_hits, lost;
    int64_t continuity_bad;         /* nodes where G^T g != Q^{n+1} - Q^n (verify = 1) */
    int64_t divb_bad;               /* tets where D b changed (verify = 1) */
    int32_t fallbacks;              /* learned -> Jacobi restarts */
    float ms_particles, ms_fields;  /* device time of the two halves (HIP events) */
    int64_t foreign;                /* deposits into tets outside a block's range (mailbox records) */
    double gauss_res_rho;           /* ||rho - G^T[*eps] e|| / ||rho|| (0 when rho = 0): the same residual
                                       against the charge alone, for comparison with gauss_res */
    int32_t edge_refinements;       /* QH_SOLVER_MIXED: reliable updates of the edge solve (FP64
                                       residuals recomputed after the start); 0 otherwise */
} qh_step_stats_t;

typedef struct {
    int32_t iters;
    double res;  /* final ||b - A x|| / ||b||, recomputed with a fresh FP64 product */
    int32_t fallback;
    float ms;
} qh_solve_stats_t;

/* Context ------------------------------------------------------------------------------ */
/* device: HIP device ordinal; stream: a hipStream_t (NULL = the null stream).
 * device < 0 makes a host-only context: mesh build, assembly, qh_mesh_info,
 * qh_mesh_topology and qh_matrix_* work; every call that needs the GPU returns QH_ESTATE. */
int qh_create(qh_ctx **out, int device, void *stream);
void qh_destroy(qh_ctx *ctx);
const char *qh_last_error(const qh_ctx *ctx);

#define QH_WALLS_REFLECT 0 /* particles reflect specularly at the walls */
#define QH_WALLS_ABSORB 1  /* a particle reaching a wall stops there and leaves the domain */
#define QH_BC_PEC 0     /* walls are perfect conductors: wall edges carry no E, wall nodes are grounded */
#define QH_BC_NEUMANN 1 /* natural boundary: every edge and node is an unknown; the Gauss-law solve
                           is singular (constants) and its potential is fixed only up to the
                           zero-mean constraint of eq. zero_mean_constraint, which e does not see */

/* Field boundary condition of the context (Sec. II.C, eq. zero_mean_constraint): QH_BC_PEC
 * (default) or QH_BC_NEUMANN. Call before qh_mesh_upload (QH_ESTATE afterwards). Particles
 * reflect specularly at the walls in both cases. */
int qh_set_boundary(qh_ctx *ctx, int32_t mode);

/* Plane wave entering through the natural boundary (the Neumann test of Sec. VI.A.2): E along
 * -z, travelling along +x, E_inc = -z E0 s'(t - x/c), H_inc = y (E0/eta) s'(t - x/c), with
 * s(u) = exp(-(u - t0)^2 / (2 sig^2)) cos(2 pi f0 (u - t0)), sig = 1/(2 pi bandwidth) (the
 * derivative of a modulated Gaussian). Each field update adds the boundary term of Ampere's law,
 * h_i(t) = integral over the boundary of W1_i . (n x H_inc) dS (Dunavant's degree-4 rule per
 * face), averaged over the step as the update's rule requires, and the Gauss-law target gains
 * the normal flux this brings in (G^T of the same term, accumulated). t = steps taken by the
 * context x dt. Needs QH_BC_NEUMANN, a mesh and physics; E0 = 0 switches it off. The accumulated
 * flux survives a later call (the field still holds it) and is cleared by qh_fields_upload. A
 * call replaces the previous wave's tables (device memory of the size of the boundary). */
int qh_set_plane_wave(qh_ctx *ctx, double E0, double f0, double bandwidth, double t0);

/* Mesh (Sec. II.C): builds K = {N, E, F, T}, incidence, geometry, the Hodge matrices
 * [*eps] (W1 mass), [*mu^-1] (W2 mass), S = C^T [*mu^-1] C and G^T [*eps] G on the host in
 * FP64 and uploads them. xyz: 3*n_nodes doubles (x0 y0 z0 x1 ...); tet_nodes: 4*n_tets
 * vertex ids. Errors: QH_EINVAL for ids out of range, degenerate tets, non-manifold faces. */
int qh_mesh_upload(qh_ctx *ctx, int64_t n_nodes, const double *xyz, int64_t n_tets,
                   const int32_t *tet_nodes);
int qh_mesh_info(const qh_ctx *ctx, qh_mesh_info_t *out);
/* Topology as built (any pointer may be NULL): edges 2*Ne, faces 3*Nf, tet_nodes 4*Nt
 * (sorted), tet_edges 6*Nt, tet_faces 4*Nt, tet_nbr 4*Nt (-1 = wall), wall_edge Ne,
 * wall_node Nn (1 = on a wall). */
int qh_mesh_topology(const qh_ctx *ctx, int32_t *edges, int32_t *faces, int32_t *tet_nodes,
                     int32_t *tet_edges, int32_t *tet_faces, int32_t *tet_nbr,
                     uint8_t *wall_edge, uint8_t *wall_node);

/* Physical constants, time step and fixed-point units. Re-assembles the edge system
 * A = [*eps] + dt^2/4 S when dt changes. */
int qh_set_physics(qh_ctx *ctx, const qh_phys_t *phys);

/* Fields (Sec. II.C: E = sum e_i W1_i, B = sum b_i W2_i). e: Ne doubles (volts; wall
 * entries are forced to 0); b: Nf int64 in units of u_b. D b must be 0 in every tet
 * (QH_EINVAL otherwise): B then is constant inside each tet. */
int qh_fields_upload(qh_ctx *ctx, const double *e, const int64_t *b);
int qh_fields_download(const qh_ctx *ctx, double *e, int64_t *b);
/* Device-pointer variants (for instance torch tensors' data_ptr()): the same arrays in device
 * memory, copied on the context's stream and ordered with its other work (no host sync, except
 * the upload's D b check, which reads one count back). The caller keeps ownership and keeps the
 * buffers alive until the stream has passed the copy. qh_fields_upload_dev: QH_EINVAL if D b != 0
 * (the fields are then unchanged); on PEC walls e is taken as 0. The buffers must come from the
 * HIP runtime this library uses: a process that also loads PyTorch's own runtime should import
 * torch before loading this library, so that both resolve to torch's. */
int qh_fields_upload_dev(qh_ctx *ctx, const double *e_dev, const int64_t *b_dev);
int qh_fields_download_dev(qh_ctx *ctx, double *e_dev, int64_t *b_dev);
/* Synthetic initial fields from caller-drawn standard normals (white_e, white_a: Ne each):
 * e = l_e sigma_e w_e on interior edges; a = line integral of (0, bz x, 0) plus
 * sigma_b l_e^2 / (2 sqrt 3) w'_e, rounded to units of u_b; b = C a. */
int qh_fields_init_synthetic(qh_ctx *ctx, const double *white_e, const double *white_a,
                             double sigma_e, double bz, double sigma_b);

/* Particles (Sec. II.A, point charges moved by the Lorentz force). A species has one
 * charge-to-mass ratio q_over_m (C/kg) and an integer charge number z (deposit sign and
 * multiple of u_q). */
int qh_species_add(qh_ctx *ctx, double q_over_m, int32_t charge_number, int32_t *species_id);
/* x, v: 3n floats (x0 y0 z0 ...); tet: n tet ids holding each point, or NULL to locate them
 * on the device (qh_locate; QH_EINVAL naming the first point outside the mesh, and the species
 * is then left empty). Replaces the species' particles and recomputes the node charge Q of all
 * species. */
int qh_particles_upload(qh_ctx *ctx, int32_t species, int64_t n, const float *x,
                        const float *v, const int32_t *tet);
/* Ordered by particle id (ascending; ids are the upload order, then the injection order).
 * Any pointer may be NULL. Sizes follow qh_particles_count. */
int qh_particles_download(const qh_ctx *ctx, int32_t species, float *x, float *v, int32_t *tet);
/* Number of particles the species holds now (after injections and absorptions). */
int qh_particles_count(const qh_ctx *ctx, int32_t species, int64_t *n);
/* The ids of the species' particles, ascending (the order of qh_particles_download). */
int qh_particles_ids(const qh_ctx *ctx, int32_t species, int32_t *ids);

/* What particles do at the walls: QH_WALLS_REFLECT (default; specular reflection about the
 * wall plane, exact sign flips on walls normal to an axis) or QH_WALLS_ABSORB (the beam test of Sec. VI.B: a particle reaching a
 * wall stops at the wall point; its current up to there is deposited, its charge is not, since
 * it leaves through the conductor, and it is removed at the end of the step). With absorbing
 * walls continuity holds at every node off the walls, which is what the step's verification
 * then checks, and every step ends with a sort of each species (a device-to-host copy of the
 * particle count, so the step synchronises its stream). */
int qh_set_walls(qh_ctx *ctx, int32_t mode);

/* Appends n particles to a species (x, v: 3n floats; tet: the tet holding each point), with
 * ids continuing from the last one given. Their W0 charge is added to the present node charge,
 * so the next step's continuity G^T g = Q^{n+1} - Q^n holds bit for bit. Injected at a wall
 * (the beam test of Sec. VI.B injects through the z = 0 face) the charge lies on wall nodes,
 * which a PEC field solve does not see: the charge enters through the wall. The species'
 * storage grows as needed (device memory is reallocated; injected particles are sorted into
 * place at the next sort). QH_EINVAL for a tet id out of range. */
int qh_particles_inject(qh_ctx *ctx, int32_t species, int64_t n, const float *x, const float *v,
                        const int32_t *tet);  /* tet NULL: located on the device, as for upload */

/* Tet holding each of n points (xyz: 3n doubles, host), found on the device: from a seed tet
 * of a uniform bucket grid over the bounding box, the straight segment from its centroid to the
 * point is walked face by face in the FP32 barycentrics the push uses, so the tet is the one
 * the push sees (a point on a face may get either neighbour; a point on a wall up to rounding,
 * its barycentric for the wall face above -1e-5, the tet behind it). tet[i] = -1 for a point
 * outside the mesh, or when the segment leaves a non-convex mesh. QH_EINVAL for a non-finite
 * point. */
int qh_locate(qh_ctx *ctx, int64_t n, const double *xyz, int32_t *tet);

/* E (V/m) and B (T) at n points (xyz: 3n doubles, tet: the tet holding each point) from the
 * present e and b, evaluated as the push gathers them (E = sum e_i W1_i linear in the tet,
 * B = sum b_i W2_i constant in it; Sec. II.C), in FP32. Host arrays; E, B: 3n doubles (either
 * may be NULL). A diagnostic: it allocates device memory per call. */
int qh_probe_fields(qh_ctx *ctx, int64_t n, const double *xyz, const int32_t *tet, double *E, double *B);
/* Static background charge for Gauss's law: mode 0 none, mode 1 the negative of the
 * present particle charge (neutral start); rho = u_q (Q_bg - Q) on interior nodes. */
int qh_charge_background(qh_ctx *ctx, int32_t mode);

/* n_steps PIC cycles (Sec. IV): field prep, per particle gather (E from W1, B from W2),
 * Boris push, tet walk with wall reflection, integer deposit of the path integral of W1
 * and of the W0 charge; then, if field_mode is QH_FIELDS_SOLVE, the implicit update of
 * Sec. IV.B (trapezoidal edge solve, discrete Gauss law for the non-solenoidal part,
 * integer Faraday update of b); QH_FIELDS_WAVE replaces the edge solve's right-hand side by
 * that of the wave equation (see its definition). stats: n_steps entries or NULL. The status
 * covers every step of the call whether or not stats are given, the most serious failure first:
 * QH_EVERIFY if verification found a broken invariant, QH_ENOTCONV if a solve hit its cap (the
 * step is still taken), QH_ELOST if a particle hit the walk cap, QH_EOVERFLOW if a step's edge
 * current or node charge came within 2^3 of the int64 range. */
int qh_pic_step(qh_ctx *ctx, const qh_step_params_t *params, int32_t n_steps,
                qh_step_stats_t *stats);
/* Deposits of the last step: g (Ne) path-integrated current, Q (Nn) node charge,
 * both int64 in units of u_q. Either may be NULL. */
int qh_deposits_download(const qh_ctx *ctx, int64_t *g, int64_t *Q);
int qh_deposits_download_dev(qh_ctx *ctx, int64_t *g_dev, int64_t *q_dev);  /* device pointers, as above */
/* Right-hand side of the last step's edge system (n_int_edges) and its solution e* as solved
 * to tol_edge, before the Gauss-law correction. Either may be NULL. These are the (rhs,
 * solution) pairs of the plain solver used to validate the learned preconditioner. */
int qh_edge_system_download(const qh_ctx *ctx, double *rhs, double *sol);
/* Record every straight piece of the next qh_pic_step (first step only) into a device
 * buffer of capacity cap (0 = off); read back with qh_segments_download. */
int qh_capture_segments(qh_ctx *ctx, int64_t cap);
/* n_out: pieces recorded (may exceed cap: then only cap were kept). Arrays of cap:
 * pid (particle index in upload order), species, seq (piece index along the path),
 * tet, lam0, lam1 (4 int32 each). */
int qh_segments_download(const qh_ctx *ctx, int64_t *n_out, int32_t *pid, int32_t *species,
                         int32_t *seq, int32_t *tet, int32_t *lam0, int32_t *lam1);

/* Integer deposit from explicit lists (Sec. IV.B.1, the time-integrated current G^n and
 * the charge rho^n = -[grad]^T G^n): piece s in tet seg_tet[s] from local coordinates
 * lam0[4s..4s+3] to lam1[4s..] (each summing to 2^20) with charge number seg_z[s]; point
 * p in tet pt_tet[p] with coordinates pt_lam[4p..] and charge number pt_z[p]. Writes g
 * (Ne) and Q (Nn), int64 in units of u_q. Deterministic (integer sums). */
int qh_deposit(qh_ctx *ctx, int64_t n_seg, const int32_t *seg_tet, const int32_t *lam0,
               const int32_t *lam1, const int32_t *seg_z, int64_t n_pt, const int32_t *pt_tet,
               const int32_t *pt_lam, const int32_t *pt_z, int64_t *g_out, int64_t *q_out);

/* qh_deposit without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same arguments and
 * results, bit for bit. The staged lists and the edge and node sums live in one file-scope
 * device array of 64 MiB per GPU (held until the process ends; its address is looked up when a
 * context is created on the device). A call needs 8 bytes per edge and node of the mesh, 40 per
 * piece and 24 per point; beyond 64 MiB it returns QH_EINVAL and does nothing. Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (several contexts or threads, or
 * streams not ordered with each other) race and must be serialised by the caller. Synchronises
 * the context stream. */
int qh_deposit_noalloc(qh_ctx *ctx, int64_t n_seg, const int32_t *seg_tet, const int32_t *lam0,
                       const int32_t *lam1, const int32_t *seg_z, int64_t n_pt, const int32_t *pt_tet,
                       const int32_t *pt_lam, const int32_t *pt_z, int64_t *g_out, int64_t *q_out);

/* Quasi-Helmholtz split of the present electric field (Sec. III, the projector P^Sigma_e; eq.
 * zero_mean_constraint under natural walls): rho_bar = G^T [*eps] e (the discrete divergence,
 * which the Gauss-law correction holds equal to the charge), E_ns = K^{-1} rho_bar (node
 * coefficients of the potential part, grad of sum E_ns,j W0_j), E_s = e - G E_ns (the
 * solenoidal remainder, G^T [*eps] E_s = 0 to the solve's tolerance). The node solve stops at
 * the backward error tol, as the Gauss-law correction does. Outputs (host, caller-allocated,
 * any may be NULL): e_ns and rho_bar n_nodes values (zero on PEC wall nodes; under natural walls
 * E_ns has zero W0-weighted mean), e_s n_edges values (zero on PEC wall edges). B is solenoidal
 * by construction (D b = 0 in integers): B_s = b, B_ns = 0. QH_ENOTCONV if the solve stopped at
 * max_it (outputs filled). */
int qh_fields_decompose(qh_ctx *ctx, double tol, int32_t max_it, double *e_ns, double *e_s, double *rho_bar,
                        qh_solve_stats_t *stats);

/* Energy of the present fields (Sec. VI.A.1: the source-free trapezoidal update leaves it
 * unchanged), in joules: *w_e = 1/2 e^T [*eps] e over the edge unknowns, *w_m =
 * 1/2 b^T [*mu^-1] b with b in webers (b_int u_b). D b = 0 makes the Whitney 2-form field
 * constant in each tet, so w_m = sum_T |B_T|^2 |T| / (2 mu0), evaluated with FP64 geometry.
 * Both sums are FP64 with a fixed reduction order (the same bits on every call). The first call
 * uploads the FP64 node coordinates (24 bytes per node) and keeps them with the context.
 * Synchronises the context stream. QH_ESTATE without mesh, physics and fields or on a host-only
 * context; QH_EINVAL for NULL outputs. */
int qh_fields_energy(qh_ctx *ctx, double *w_e, double *w_m);

/* Solve system (QH_SYS_EDGE or QH_SYS_NODE) A x = rhs on its interior unknowns
 * (n_int_edges or n_int_nodes values), to ||rhs - A x|| <= tol ||rhs|| in FP64: FP64 PCG with
 * FP64 dot products (solver = QH_SOLVER_FP64), or FP32 PCG with FP64 reliable updates
 * (QH_SOLVER_MIXED). x holds the initial guess on entry. A learned or mixed solve that does not
 * converge is restarted as FP64 Jacobi-PCG (stats->fallback = 1). */
int qh_field_solve(qh_ctx *ctx, int32_t system, const double *rhs, double *x, double tol,
                   int32_t max_it, int32_t precond, int32_t solver, qh_solve_stats_t *stats);

/* Learned preconditioner for the edge system (used with precond = QH_PC_LEARNED).
 * M = G^T G with G sparse lower triangular on the pattern of A; a network 16 -> 64 -> 64 -> 1
 * (ReLU) maps 16 dimensionless local features of each entry (i, j), j <= i, to o_ij and
 * G_ij = o_ij / sqrt(A_jj), G_ii = softplus(o_ii + s0) / sqrt(A_ii), softplus(s0) = 1 (a zero
 * network is Jacobi). Inference runs on MFMA in BF16 with FP32 accumulation. Weights: FP32,
 * QH_MLP_NPARAM values: W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3 (out x in, row
 * major). Not from the paper, which leaves the linear solver open. */
#define QH_MLP_NPARAM 5313
int qh_precond_set_weights(qh_ctx *ctx, const float *w, int64_t n);
int qh_precond_get_weights(qh_ctx *ctx, float *w, int64_t n);
/* The network as a self-describing byte blob (magic "QHPRECND", version 1, parameter count, the
 * FP32 weights, an FNV-1a checksum of them), to keep a trained preconditioner across runs and
 * meshes. save: buf NULL sets *len to the size needed; a smaller *len is QH_EINVAL. load:
 * QH_EINVAL for a blob that is short, of another version or size, or fails its checksum (the
 * present weights are then kept). */
int qh_precond_save(qh_ctx *ctx, void *buf, size_t *len);

/* Checkpoint of a run (host blob, magic "QHSTATE1", FNV-1a checksum): e, b, the node charge Q
 * and background Q_bg, the wave update's history (e^{n-1} and the previous step's current),
 * the plane wave's accumulated boundary flux, the step count, and every species' particles with
 * their ids and next id. Not in it: the mesh, physics, boundary and wall modes, plane-wave
 * parameters and species definitions (set them up as before loading; load checks mesh sizes
 * and each species' q/m and charge number), the learned preconditioner (qh_precond_save). The
 * integer deposits make a resumed run bit-identical to an uninterrupted one. save: buf NULL sets
 * *len to the size needed. load: QH_EINVAL for a blob that is corrupted or does not fit the
 * context (nothing is changed then). */
int qh_state_save(qh_ctx *ctx, void *buf, size_t *len);
int qh_state_load(qh_ctx *ctx, const void *buf, size_t len);
int qh_precond_load(qh_ctx *ctx, const void *buf, size_t len);
/* Entries of G: rows/cols (interior-edge indices, row-major lower triangle of A's pattern) and
 * FP32 values for the current weights. Pass rows = cols = vals = NULL to query *nnz. */
int qh_precond_factor(qh_ctx *ctx, int64_t *nnz, int32_t *rows, int32_t *cols, float *vals);
/* The preconditioner's application z = G^T (G r) as the learned solve applies it (the same
 * kernels: BF16 copies of G and G^T, FP64 products and sums), for the current weights. r, z:
 * n_int_edges doubles (host). QH_ESTATE before mesh and physics. */
int qh_precond_apply(qh_ctx *ctx, const double *r, double *z);
/* Training objective L = log(tr(G A G^T)/n) - (2/n) sum_i log G_ii (log of the Kaporin
 * condition number of G A G^T up to a constant), trace estimated with the 16 probe vectors
 * probes[i*16 + p] (node-major, n_int_edges x 16); and, if grad != NULL, dL/dweights
 * (QH_MLP_NPARAM floats, computed by the MFMA backward kernel). */
int qh_precond_loss_grad(qh_ctx *ctx, const float *probes, double *loss, float *grad);
typedef struct {
    int32_t steps;          /* Adam steps, 16 Rademacher probes each */
    float lr;
    uint64_t seed;          /* probe and pair-batch generator seed */
    int32_t validate_every; /* PCG on the first (up to 2) pairs every k steps; best weights kept */
    double val_tol;         /* validation solve tolerance (e.g. 1e-8) */
    int32_t val_max_it;
    double pair_weight;     /* lambda: the objective is L + lambda L_E, L_E the energy-norm loss on a
                               batch of 16 recorded solver pairs per step (qh_pairs_record); 0: L only */
} qh_train_params_t;
typedef struct {
    int32_t steps_done;
    double loss_first, loss_last;
    int32_t val_iters_jacobi, val_iters_best, best_step; /* summed over the validation pairs */
    float ms;
    double pair_loss_first, pair_loss_last; /* L_E of the first and last step's batch (0 without pairs) */
    double val_energy_err;  /* max over the validation pairs of ||x - M b||_A / ||x||_A, kept weights */
} qh_train_stats_t;
/* Solver pairs for training: every following field step of qh_pic_step (QH_FIELDS_SOLVE or
 * QH_FIELDS_WAVE) stores its edge system's right-hand side and solution e* (as solved, before the
 * Gauss-law correction) in FP32 into a device bank of `capacity` pairs (8 bytes per interior edge
 * and pair), until it is full. A call replaces the bank (capacity 0 frees it). With the plain
 * (Jacobi) solver these are the pairs "the plain solver generates". */
int qh_pairs_record(qh_ctx *ctx, int32_t capacity);
int qh_pairs_count(const qh_ctx *ctx, int32_t *n);
/* Appends n_pairs host pairs (rhs, sol: n_pairs x n_int_edges, pair-major) to the bank (after
 * qh_pairs_record; QH_EINVAL past its capacity). */
int qh_pairs_add(qh_ctx *ctx, int32_t n_pairs, const double *rhs, const double *sol);
/* The energy-norm loss L_E on 16 bank pairs (idx: 16 indices) and, if grad != NULL, dL_E/dweights
 * (QH_MLP_NPARAM floats) from the same kernels training uses. */
int qh_precond_pair_loss_grad(qh_ctx *ctx, const int32_t *idx, double *loss, float *grad);
/* Train on the GPU: Adam on L (the log Kaporin number above, 16 Rademacher probes per step) plus
 * pair_weight times the energy-norm loss L_E = mean ||x - G^T G b||_A^2 / ||x||_A^2 over a batch
 * of 16 pairs drawn from the recorded bank (QH_ESTATE if pair_weight > 0 and the bank is empty).
 * rhs, sol: n_pairs x n_int_edges (pair-major) held-out right-hand sides and solutions of the
 * edge system from the plain solver: the first (up to 2) validate each candidate (PCG iterations
 * to val_tol) and select the weights kept, and give the kept network's energy-norm error. */
int qh_precond_train(qh_ctx *ctx, const qh_train_params_t *params, int32_t n_pairs,
                     const double *rhs, const double *sol, qh_train_stats_t *stats);

/* Assembled FP64 matrices as CSR (0-based, sorted columns), host copies. which:
 * 0 A = [*eps] + dt^2/4 S, 1 [*eps], 2 S = C^T [*mu^-1] C (all interior edges x interior
 * edges), 3 C^T [*mu^-1] (interior edges x all faces), 4 G^T [*eps] (interior nodes x
 * interior edges), 5 K = G^T [*eps] G (interior nodes). ptr: nrow+1, col/val: nnz. */
int qh_matrix_info(const qh_ctx *ctx, int32_t which, int64_t *nrow, int64_t *ncol, int64_t *nnz);
int qh_matrix_download(const qh_ctx *ctx, int32_t which, int32_t *ptr, int32_t *col, double *val);

/* Per-kernel device time, measured with HIP events recorded around each launch on the
 * context stream while enabled (enabling resets the table). Index k of the table:
 * 0 field prep, 1 particle step, 2 sort, 3 edge right-hand side, 4 edge-system CG product
 * (fused direction update + SpMV + dot), 5 edge-system CG vector update, 6 CG init,
 * 7 Gauss-law set-up and correction, 8 Faraday update, 9 residual check, 10 node-system CG
 * product, 11 node-system CG vector update, 12 learned preconditioner application, 13 plane-wave
 * boundary source (edge term and boundary flux).
 * ms_total[k]: summed ms; launches[k]: count. */
int qh_timing_enable(qh_ctx *ctx, int32_t on);
int qh_timing_read(const qh_ctx *ctx, int32_t n, double *ms_total, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* QH_H */
