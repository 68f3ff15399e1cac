// Particle half of the PIC cycle on gfx950: per-tet field records, the fused
// gather -> Boris -> tet walk -> integer deposit kernel, and the counting sort by tet.
//
// Gather (Sec. II.C): E = sum e_i W1_i is affine inside a tet, E(r) = alpha + beta x (r - c)
// with alpha = E(c) = sum e_ab (grad l_b - grad l_a)/4 and beta = sum e_ab grad l_a x grad l_b;
// B = sum b_f W2_f is constant inside a tet whenever D b = 0 there (the integer Faraday update
// keeps D b = 0 exactly), B = sum b_f W2_f(c) with W2_abc(c) = (grad l_b - grad l_a) x
// (grad l_c - grad l_a) / 2. Both are computed once per tet per step (field_prep) and read by
// every particle of the tet.
//
// Deposit (Sec. IV.B.1): the time-integrated current of a particle is the path integral of W1
// along its path. For a straight piece inside a tet, int W1_ab . dl = l_a(r0) l_b(r1) -
// l_a(r1) l_b(r0); with coordinates quantised to 2^-20 (summing to exactly 2^20, carried across
// faces by vertex id) the piece adds z (L_a^0 L_b^1 - L_a^1 L_b^0) to edge a->b and the end
// point adds z 2^20 L_n to node n. G^T g then telescopes to Q^{n+1} - Q^n in int64: discrete
// continuity holds bit for bit and the sums are independent of order.
#include <type_traits>

#include "qh_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kPpt = 2;                  // consecutive particles per thread
constexpr int kChunk = kBlock * kPpt;    // particles per block
static_assert(kChunk == QH_CHUNK, "particle chunk size");
constexpr int kWin = 128;                // owned tets whose sums a block keeps in LDS

__device__ __forceinline__ void lam4(const float4 A, const float4 B, const float4 C, float x,
                                     float y, float z, float l[4]) {
    float dx = x - A.w, dy = y - B.w, dz = z - C.w;
    l[1] = __fmaf_rn(A.x, dx, __fmaf_rn(A.y, dy, __fmaf_rn(A.z, dz, 0.25f)));
    l[2] = __fmaf_rn(B.x, dx, __fmaf_rn(B.y, dy, __fmaf_rn(B.z, dz, 0.25f)));
    l[3] = __fmaf_rn(C.x, dx, __fmaf_rn(C.y, dy, __fmaf_rn(C.z, dz, 0.25f)));
    l[0] = __fsub_rn(__fsub_rn(__fsub_rn(1.0f, l[1]), l[2]), l[3]);
}

// Fixed point: round half to even, clamp to [0, 2^F], the largest coordinate (first on
// ties) absorbs the remainder so the four sum to 2^F. forced >= 0 pins that one to 0.
__device__ __forceinline__ void quantize(const float l[4], int forced, int L[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float q = rintf(l[i] * (float)QH_SCALE);
        q = fminf(fmaxf(q, 0.0f), (float)QH_SCALE);
        L[i] = (i == forced) ? 0 : (int)q;
    }
    int im = 0;
#pragma unroll
    for (int i = 1; i < 4; ++i)
        if (L[i] > L[im]) im = i;
    int rest = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (i != im) rest += L[i];
    L[im] = QH_SCALE - rest;
}

__device__ __forceinline__ void atomic_add_i64(int64_t *p, int64_t v) {
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

__device__ __forceinline__ void atomic_add_lds(long long *p, long long v) {
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

struct StepArgs {
    const float4 *geo;
    const float4 *frec;
    const int4 *tnodes;
    const int32_t *tedges;
    const int4 *tnbr;
    float *x, *y, *z, *vx, *vy, *vz;
    int32_t *tet;
    const int32_t *pid;
    const int32_t *own;     // own[b] .. own[b+1]: tets owned by block b (from the last sort)
    unsigned int *mail_cnt; // records posted to each mailbox (tets [kMailTets m, kMailTets (m+1))) this launch
    int32_t *mail;          // per mailbox: kMailCap packed point pairs (uint4), then kMailCap heads (tet | end << 31)
    int64_t n;
    int32_t nt;
    float hqm;              // q/m * dt / 2
    float dt;
    int32_t zq;             // charge number
    int32_t absorb;         // walls absorb (1) or reflect (0)
    int32_t zeroed;         // acc_tet was cleared before the launch: write the window sums only
    int64_t *g, *Q;         // deposits that find no mailbox slot (atomics)
    int64_t *acc_tet;       // per-tet sums, plane-major: acc_tet[k * nt + t], k = 6 edges, 4 nodes
    uint16_t *ovf;          // per block: chunk indices of queued particles past the LDS queue
    unsigned long long *counters;
    // capture
    int32_t species;
    int64_t cap;
    unsigned long long *seg_count;
    int32_t *seg_buf;
};

}  // namespace

// ------------------------------------------------------------------------------------------
// Field records: (alpha.xyz, beta.x) (beta.y, beta.z, B.x, B.y) (B.z, 0, 0, 0)
__global__ void __launch_bounds__(256) k_field_prep(const float4 *__restrict__ geo,
                                                    const int32_t *__restrict__ tedges,
                                                    const int32_t *__restrict__ tfaces,
                                                    const double *__restrict__ e,
                                                    const int64_t *__restrict__ b, double u_b,
                                                    int32_t nt, float4 *__restrict__ frec) {
    int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    float4 A = geo[3 * t], B = geo[3 * t + 1], C = geo[3 * t + 2];
    double g[4][3];
    g[1][0] = A.x; g[1][1] = A.y; g[1][2] = A.z;
    g[2][0] = B.x; g[2][1] = B.y; g[2][2] = B.z;
    g[3][0] = C.x; g[3][1] = C.y; g[3][2] = C.z;
    for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    const int LF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    double al[3] = {0, 0, 0}, be[3] = {0, 0, 0}, Bf[3] = {0, 0, 0};
    for (int k = 0; k < 6; ++k) {
        double c = e[tedges[8 * t + k]];
        const double *ga = g[LE[k][0]], *gb = g[LE[k][1]];
        double cx = ga[1] * gb[2] - ga[2] * gb[1];
        double cy = ga[2] * gb[0] - ga[0] * gb[2];
        double cz = ga[0] * gb[1] - ga[1] * gb[0];
        al[0] += 0.25 * c * (gb[0] - ga[0]);
        al[1] += 0.25 * c * (gb[1] - ga[1]);
        al[2] += 0.25 * c * (gb[2] - ga[2]);
        be[0] += c * cx; be[1] += c * cy; be[2] += c * cz;
    }
    for (int k = 0; k < 4; ++k) {
        double c = (double)b[tfaces[4 * t + k]] * u_b;
        const double *ga = g[LF[k][0]], *gb = g[LF[k][1]], *gc = g[LF[k][2]];
        double u[3] = {gb[0] - ga[0], gb[1] - ga[1], gb[2] - ga[2]};
        double w[3] = {gc[0] - ga[0], gc[1] - ga[1], gc[2] - ga[2]};
        Bf[0] += 0.5 * c * (u[1] * w[2] - u[2] * w[1]);
        Bf[1] += 0.5 * c * (u[2] * w[0] - u[0] * w[2]);
        Bf[2] += 0.5 * c * (u[0] * w[1] - u[1] * w[0]);
    }
    frec[3 * t] = make_float4((float)al[0], (float)al[1], (float)al[2], (float)be[0]);
    frec[3 * t + 1] = make_float4((float)be[1], (float)be[2], (float)Bf[0], (float)Bf[1]);
    frec[3 * t + 2] = make_float4((float)Bf[2], 0.f, 0.f, 0.f);
}

void launch_field_prep(qh_ctx *c) {
    int32_t nt = (int32_t)c->hm.Nt;
    hipLaunchKernelGGL(k_field_prep, dim3((nt + 255) / 256), dim3(256), 0, c->stream, c->geo,
                       c->tedges, c->tfaces, c->e, c->b, c->phys.u_b, nt, c->frec);
}

// ------------------------------------------------------------------------------------------
// Deposit routing.
//
// A block owns the tets [own[b], own[b+1]) that its chunk of particles held at the last sort;
// the first kWin of them (its window) are summed in LDS per unit charge (edges sum
// L_a^0 L_b^1 - L_a^1 L_b^0, nodes sum the L_n of end points; the charge number and 2^20 scale
// them when they leave LDS). A piece in a tet outside the window (a particle that moved since
// the sort, a walk piece past the range) is posted as one compact record into the mailbox of
// that tet's run of kMailTets tets; a slot costs one 32-bit atomic (per wave and mailbox on the
// fast path, per piece in the walk) instead of ten 64-bit atomics per piece. k_mail_apply adds
// each mailbox into acc_tet, and the gather kernels add acc_tet into edges and nodes. Only records that find no mailbox slot use int64
// atomics on edges and nodes. Integer sums do not depend on order, so the result is the same
// bits on every path.

// A mailbox record holds a piece's two points in 16 bytes: the four quantised coordinates of a
// point sum to exactly 2^20, so three of them (21 bits each, values 0 .. 2^20) fix the fourth.
static_assert(QH_FBITS <= 20, "a quantised coordinate must fit 21 bits");
__device__ __forceinline__ uint4 pack_points(const int P0[4], const int P1[4]) {
    const unsigned long long a = (unsigned long long)P0[1] | (unsigned long long)P0[2] << 21 |
                                 (unsigned long long)P0[3] << 42;
    const unsigned long long b = (unsigned long long)P1[1] | (unsigned long long)P1[2] << 21 |
                                 (unsigned long long)P1[3] << 42;
    return make_uint4((unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32));
}

__device__ __forceinline__ void unpack_point(unsigned lo, unsigned hi, int P[4]) {
    const unsigned long long w = (unsigned long long)hi << 32 | lo;
    P[1] = (int)(w & 0x1fffff);
    P[2] = (int)((w >> 21) & 0x1fffff);
    P[3] = (int)((w >> 42) & 0x1fffff);
    P[0] = QH_SCALE - P[1] - P[2] - P[3];
}

// Unit-charge values of one straight piece P0 -> P1 (6 edges; 4 nodes when P1 is the end).
__device__ __forceinline__ void piece_values(const int P0[4], const int P1[4], bool end, long long v[10]) {
    const int LE0[6] = {0, 0, 0, 1, 1, 2};
    const int LE1[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int j = 0; j < 6; ++j)
        v[j] = (long long)P0[LE0[j]] * P1[LE1[j]] - (long long)P1[LE0[j]] * P0[LE1[j]];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[6 + r] = end ? P1[r] : 0;
}

template <int WIN>
__device__ __forceinline__ void put_lds(long long *acc, int slot, const long long *v) {
#pragma unroll
    for (int k = 0; k < 10; ++k) atomic_add_lds(&acc[k * WIN + slot], v[k]);
}

// A piece in a tet outside the window: one record into the tet's mailbox, or, when the
// mailbox is full, int64 atomics on edges and nodes. GROUP: slots are reserved with one atomic
// per distinct mailbox among the active lanes (the lanes' tets cluster in a few mailboxes, as in
// the fast path); otherwise one atomic per lane (walk pieces scatter over the neighbours in all
// directions, and a serial loop over their mailboxes costs more than it saves).
template <bool GROUP>
__device__ __forceinline__ void post_piece(const StepArgs &a, int tt, const int P0[4], const int P1[4], bool end) {
    const int o = tt / kMailTets;
    unsigned int slot = 0xffffffffu;
    if (GROUP) {
        const int lane = __lane_id();
        unsigned long long pending = __ballot(1);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int lo = __shfl(o, leader);
            const unsigned long long same = __ballot(o == lo);
            unsigned int first = 0;
            if (lane == leader) first = atomicAdd(&a.mail_cnt[lo], (unsigned int)__popcll(same));
            first = (unsigned int)__shfl((int)first, leader);
            if (o == lo) slot = first + (unsigned int)__popcll(same & ((1ull << lane) - 1ull));
            pending &= ~same;
        }
    } else {
        slot = atomicAdd(&a.mail_cnt[o], 1u);
    }
    if (slot < (unsigned)kMailCap) {
        int32_t *box = a.mail + (int64_t)o * kMailCap * kMailWords;
        reinterpret_cast<uint4 *>(box)[slot] = pack_points(P0, P1);
        box[4 * kMailCap + slot] = tt | (end ? (int32_t)0x80000000u : 0);
        return;
    }
    long long v[10];
    piece_values(P0, P1, end, v);
    const int32_t *te = a.tedges + 8 * (int64_t)tt;
    const int4 tn = a.tnodes[tt];
    const int nv[4] = {tn.x, tn.y, tn.z, tn.w};
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if (v[k]) atomic_add_i64(a.g + te[k], a.zq * v[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (v[6 + k]) atomic_add_i64(a.Q + nv[k], (long long)a.zq * QH_SCALE * v[6 + k]);
}

__device__ __forceinline__ void record_piece(const StepArgs &a, int32_t pid, int seq, int tt, const int L0[4],
                                             const int L1[4]) {
    unsigned long long s = atomicAdd(a.seg_count, 1ull);
    if ((int64_t)s < a.cap) {
        int32_t *o = a.seg_buf + 12 * s;
        o[0] = pid; o[1] = a.species; o[2] = seq; o[3] = tt;
        for (int r = 0; r < 4; ++r) { o[4 + r] = L0[r]; o[8 + r] = L1[r]; }
    }
}

// ------------------------------------------------------------------------------------------
// Walk of one particle from (px, py, pz) in tet t along dt v^{n+1/2}, face by face (exit
// face = smallest crossing parameter, the entry face excluded; at most QH_MAX_PIECES
// pieces), reflecting specularly at the walls, or, with absorbing walls, stopping at
// the wall point (gone: the charge leaves through the wall, so no end point is deposited).
// deposit(tet, L_start, L_end, end) takes each straight piece; on return the state holds the
// end point, its tet and the (possibly reflected) velocity.
template <bool CAPTURE, typename Dep>
__device__ __forceinline__ void walk_one(const StepArgs &a, float &px, float &py, float &pz, float &vx, float &vy,
                                         float &vz, int &t, int32_t pid, Dep &&deposit, unsigned int &n_cross,
                                         unsigned int &n_wall, unsigned int &n_lost, bool &gone) {
    int seq = 0;
    float4 A = a.geo[3 * t], B = a.geo[3 * t + 1], C = a.geo[3 * t + 2];
    int4 nb4 = a.tnbr[t], on = a.tnodes[t];  // loaded with the geometry: one round trip per tet
    float rx = a.dt * vx, ry = a.dt * vy, rz = a.dt * vz;
    float l[4];
    int Lp[4], Lc[4];
    lam4(A, B, C, px, py, pz, l);
    quantize(l, -1, Lp);
    int entry = -1, pieces = 0;
    for (;;) {
        float gl[4];
        gl[1] = A.x * rx + A.y * ry + A.z * rz;
        gl[2] = B.x * rx + B.y * ry + B.z * rz;
        gl[3] = C.x * rx + C.y * ry + C.z * rz;
        gl[0] = -(gl[1] + gl[2] + gl[3]);
        lam4(A, B, C, px, py, pz, l);
        int k = -1;
        float smin = 2.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r == entry) continue;
            float le = l[r] + gl[r];
            // a face is crossed only when the path moves out through it: a point rounded to just
            // outside a face (at a crossing or a wall corner) that moves back in does not leave
            // (it would bounce between two walls, reflected outward, until the piece cap)
            if (!(le < 0.0f) || !(gl[r] < 0.0f)) continue;
            float s = l[r] <= 0.0f ? 0.0f : l[r] / (l[r] - le);
            if (s < smin) { smin = s; k = r; }
        }
        if (k < 0) { px += rx; py += ry; pz += rz; break; }
        if (pieces >= QH_MAX_PIECES - 1) { ++n_lost; break; }
        float cx = __fmaf_rn(smin, rx, px), cy = __fmaf_rn(smin, ry, py), cz = __fmaf_rn(smin, rz, pz);
        lam4(A, B, C, cx, cy, cz, l);
        quantize(l, k, Lc);
        deposit(t, Lp, Lc, false);
        if (CAPTURE) record_piece(a, pid, seq, t, Lp, Lc);
        ++seq;
        ++pieces;
        float rem = 1.0f - smin;
        rx *= rem; ry *= rem; rz *= rem;
        px = cx; py = cy; pz = cz;
        int nb = k == 0 ? nb4.x : k == 1 ? nb4.y : k == 2 ? nb4.z : nb4.w;
        if (nb >= 0) {
            const int4 nn = a.tnodes[nb];
            A = a.geo[3 * nb]; B = a.geo[3 * nb + 1]; C = a.geo[3 * nb + 2];
            const int4 nbn = a.tnbr[nb];
            int ov[4] = {on.x, on.y, on.z, on.w}, nv[4] = {nn.x, nn.y, nn.z, nn.w};
            int fresh = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int val = 0, found = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (ov[r] == nv[j]) { val = Lc[r]; found = 1; }
                Lp[j] = val;
                if (!found) fresh = j;
            }
            entry = fresh;
            t = nb;
            nb4 = nbn;
            on = nn;
            ++n_cross;
        } else if (a.absorb) {
            gone = true;
            ++n_wall;
            return;
        } else {
            // specular reflection: the wall normal is grad l_k. A normal along an axis (two zero
            // components, as on box walls) flips that component exactly; any other mirrors the
            // displacement and the velocity about the wall plane
            float nx, ny, nz;
            if (k == 0) { nx = -(A.x + B.x + C.x); ny = -(A.y + B.y + C.y); nz = -(A.z + B.z + C.z); }
            else if (k == 1) { nx = A.x; ny = A.y; nz = A.z; }
            else if (k == 2) { nx = B.x; ny = B.y; nz = B.z; }
            else { nx = C.x; ny = C.y; nz = C.z; }
            const int zeros = (nx == 0.0f) + (ny == 0.0f) + (nz == 0.0f);
            if (zeros == 2) {
                // selects, not branches: keeps the components in registers
                const bool fx = nx != 0.0f, fy = ny != 0.0f, fz = nz != 0.0f;
                rx = fx ? -rx : rx; vx = fx ? -vx : vx;
                ry = fy ? -ry : ry; vy = fy ? -vy : vy;
                rz = fz ? -rz : rz; vz = fz ? -vz : vz;
            } else {
                const float inv = 1.0f / (nx * nx + ny * ny + nz * nz);
                const float rn = 2.0f * (rx * nx + ry * ny + rz * nz) * inv;
                const float vn = 2.0f * (vx * nx + vy * ny + vz * nz) * inv;
                rx -= rn * nx; ry -= rn * ny; rz -= rn * nz;
                vx -= vn * nx; vy -= vn * ny; vz -= vn * nz;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) Lp[r] = Lc[r];
            entry = k;
            ++n_wall;
        }
    }
    int Le[4];
    lam4(A, B, C, px, py, pz, l);
    quantize(l, -1, Le);
    deposit(t, Lp, Le, true);
    if (CAPTURE) record_piece(a, pid, seq, t, Lp, Le);
}

// ------------------------------------------------------------------------------------------
// Fused particle step. A block takes kChunk consecutive particles (sorted by tet at the last
// sort), kPpt consecutive ones per thread.
// Phase A (all waves): gather, Boris; a particle whose straight path stays in its tet gets its
// new position and the deposit of the piece (LDS window or post) and is written back from
// registers; a particle whose path leaves the tet is queued in LDS with its start state (past
// kQueue queued particles: its new velocity to memory and its index to an overflow list).
// Phase B (wave 0 only; the other waves exit): the queued particles are walked one per lane and
// written back; then the window sums go to acc_tet as plain stores (zeros for owned tets past the
// window) and the event counters to memory. Waves 1-3 do not wait for the walks.
constexpr int kQueue = 128;
template <bool CAPTURE>
__global__ void __launch_bounds__(kBlock) k_particle_step(StepArgs a) {
    __shared__ long long acc[10 * kWin];  // plane-major: acc[k * kWin + slot]
    __shared__ float4 qrec[2 * kQueue];   // queued particle: (x, y, z, vx) (vy, vz, tet, chunk index) as bits
    __shared__ unsigned int s_cnt[5];     // queued particles, -, -, -, posted pieces of phase A
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    const int T0 = a.own[blockIdx.x], T1 = a.own[blockIdx.x + 1];
    const int W = min(T1 - T0, kWin);
    for (int j = threadIdx.x; j < 10 * kWin; j += kBlock) acc[j] = 0;
    if (threadIdx.x < 5) s_cnt[threadIdx.x] = 0;
    // owned tets past the window get no LDS sums: the whole block zeroes them now (the mailbox
    // kernel that follows adds their posted pieces), unless the host cleared every sum
    if (!a.zeroed)
        for (int j = W + threadIdx.x; j < T1 - T0; j += kBlock)
#pragma unroll
            for (int k = 0; k < 10; ++k) a.acc_tet[(int64_t)k * a.nt + T0 + j] = 0;
    __syncthreads();
    unsigned int n_cross = 0, n_wall = 0, n_lost = 0, n_foreign = 0;
    auto deposit_to = [&](auto group, int tt, const int P0[4], const int P1[4], bool end) {
        const int slot = tt - T0;
        if ((unsigned)slot < (unsigned)W) {
            long long v[10];
            piece_values(P0, P1, end, v);
            put_lds<kWin>(acc, slot, v);
        } else {
            ++n_foreign;
            post_piece<decltype(group)::value>(a, tt, P0, P1, end);
        }
    };
    // fast path: grouped mailbox reservations; walk: one per lane
    auto deposit = [&](int tt, const int P0[4], const int P1[4], bool end) {
        deposit_to(std::true_type{}, tt, P0, P1, end);
    };
    auto deposit_walk = [&](int tt, const int P0[4], const int P1[4], bool end) {
        deposit_to(std::false_type{}, tt, P0, P1, end);
    };

    // ---- phase A
    const int64_t i0 = base + (int64_t)threadIdx.x * kPpt;
    const bool full = base + kChunk <= a.n;
    float2 X, Y, Z, VX, VY, VZ;
    int2 TT;
    if (full) {
        const int64_t v = i0 / 2;
        X = ((const float2 *)a.x)[v]; Y = ((const float2 *)a.y)[v]; Z = ((const float2 *)a.z)[v];
        VX = ((const float2 *)a.vx)[v]; VY = ((const float2 *)a.vy)[v]; VZ = ((const float2 *)a.vz)[v];
        TT = ((const int2 *)a.tet)[v];
    }
    bool queued[kPpt];
#pragma unroll
    for (int q = 0; q < kPpt; ++q) {
        queued[q] = false;
        const int64_t i = i0 + q;
        if (!full && i >= a.n) break;
        float px, py, pz, vx, vy, vz;
        int t;
        if (full) {
            px = q == 0 ? X.x : X.y;
            py = q == 0 ? Y.x : Y.y;
            pz = q == 0 ? Z.x : Z.y;
            vx = q == 0 ? VX.x : VX.y;
            vy = q == 0 ? VY.x : VY.y;
            vz = q == 0 ? VZ.x : VZ.y;
            t = q == 0 ? TT.x : TT.y;
        } else {
            px = a.x[i]; py = a.y[i]; pz = a.z[i];
            vx = a.vx[i]; vy = a.vy[i]; vz = a.vz[i];
            t = a.tet[i];
        }
        // gather at x^n: E = alpha + beta x (r - c), B constant
        const float4 A = a.geo[3 * t], B = a.geo[3 * t + 1], C = a.geo[3 * t + 2];
        const float4 F0 = a.frec[3 * t], F1 = a.frec[3 * t + 1], F2 = a.frec[3 * t + 2];
        float dx = px - A.w, dy = py - B.w, dz = pz - C.w;
        float Ex = F0.x + (F1.x * dz - F1.y * dy);
        float Ey = F0.y + (F1.y * dx - F0.w * dz);
        float Ez = F0.z + (F0.w * dy - F1.x * dx);
        // Boris
        const float h = a.hqm;
        float mx = vx + h * Ex, my = vy + h * Ey, mz = vz + h * Ez;
        float tx = h * F1.z, ty = h * F1.w, tz = h * F2.x;
        float s2 = 2.0f / (1.0f + tx * tx + ty * ty + tz * tz);
        float sx = s2 * tx, sy = s2 * ty, sz = s2 * tz;
        float qx = mx + (my * tz - mz * ty);
        float qy = my + (mz * tx - mx * tz);
        float qz = mz + (mx * ty - my * tx);
        vx = mx + (qy * sz - qz * sy) + h * Ex;
        vy = my + (qz * sx - qx * sz) + h * Ey;
        vz = mz + (qx * sy - qy * sx) + h * Ez;
        const float rx = a.dt * vx, ry = a.dt * vy, rz = a.dt * vz;
        // does the straight path leave the tet? (same test as the walk's first step)
        float l[4], gl[4];
        lam4(A, B, C, px, py, pz, l);
        gl[1] = A.x * rx + A.y * ry + A.z * rz;
        gl[2] = B.x * rx + B.y * ry + B.z * rz;
        gl[3] = C.x * rx + C.y * ry + C.z * rz;
        gl[0] = -(gl[1] + gl[2] + gl[3]);
        const bool leaves = (l[0] + gl[0] < 0.0f) | (l[1] + gl[1] < 0.0f) | (l[2] + gl[2] < 0.0f) |
                            (l[3] + gl[3] < 0.0f);
        if (!leaves) {
            int L0[4], L1[4];
            quantize(l, -1, L0);
            px += rx; py += ry; pz += rz;
            lam4(A, B, C, px, py, pz, l);
            quantize(l, -1, L1);
            deposit(t, L0, L1, true);
            if (CAPTURE) record_piece(a, a.pid[i], 0, t, L0, L1);
        } else {
            const unsigned int k = atomicAdd(&s_cnt[0], 1u);
            queued[q] = true;
            if (k < (unsigned)kQueue) {
                qrec[2 * k] = make_float4(px, py, pz, vx);
                qrec[2 * k + 1] = make_float4(vy, vz, __int_as_float(t), __int_as_float(threadIdx.x * kPpt + q));
            } else {
                // past the LDS queue: the new velocity goes to memory (position and tet there are
                // still the start state) and the chunk index to this block's overflow list
                a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
                a.ovf[base + (k - kQueue)] = (uint16_t)(threadIdx.x * kPpt + q);
            }
        }
        if (full) {
            if (q == 0) {
                X.x = px; Y.x = py; Z.x = pz; VX.x = vx; VY.x = vy; VZ.x = vz; TT.x = t;
            } else {
                X.y = px; Y.y = py; Z.y = pz; VX.y = vx; VY.y = vy; VZ.y = vz; TT.y = t;
            }
        } else if (!queued[q]) {
            a.x[i] = px; a.y[i] = py; a.z[i] = pz;
            a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
            a.tet[i] = t;
        }
    }
    // write-back of the finished particles; a queued one is written by its walker
    if (full) {
        const int64_t v = i0 / 2;
        if (!queued[0] && !queued[1]) {
            ((float2 *)a.x)[v] = X; ((float2 *)a.y)[v] = Y; ((float2 *)a.z)[v] = Z;
            ((float2 *)a.vx)[v] = VX; ((float2 *)a.vy)[v] = VY; ((float2 *)a.vz)[v] = VZ;
            ((int2 *)a.tet)[v] = TT;
        } else if (!queued[0]) {
            a.x[i0] = X.x; a.y[i0] = Y.x; a.z[i0] = Z.x; a.vx[i0] = VX.x; a.vy[i0] = VY.x; a.vz[i0] = VZ.x;
            a.tet[i0] = TT.x;
        } else if (!queued[1]) {
            a.x[i0 + 1] = X.y; a.y[i0 + 1] = Y.y; a.z[i0 + 1] = Z.y; a.vx[i0 + 1] = VX.y; a.vy[i0 + 1] = VY.y;
            a.vz[i0 + 1] = VZ.y; a.tet[i0 + 1] = TT.y;
        }
    }
    // posted pieces of phase A
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n_foreign += __shfl_xor(n_foreign, off, 64);
    const int lane = threadIdx.x & 63;
    if (lane == 0 && n_foreign) atomicAdd(&s_cnt[4], n_foreign);
    __syncthreads();
    if (threadIdx.x >= 64) return;  // phase B and the write-out are wave 0's

    // ---- phase B: the queued particles, one per lane of wave 0
    n_foreign = 0;
    const int nall = (int)s_cnt[0], nq = min(nall, kQueue);
    for (int qi = lane; qi < nall; qi += 64) {
        int64_t i;
        float px, py, pz, vx, vy, vz;
        int t;
        if (qi < nq) {
            const float4 q0 = qrec[2 * qi], q1 = qrec[2 * qi + 1];
            i = base + __float_as_int(q1.w);
            px = q0.x; py = q0.y; pz = q0.z; vx = q0.w; vy = q1.x; vz = q1.y;
            t = __float_as_int(q1.z);
        } else {
            i = base + a.ovf[base + (qi - kQueue)];
            px = a.x[i]; py = a.y[i]; pz = a.z[i];
            vx = a.vx[i]; vy = a.vy[i]; vz = a.vz[i];
            t = a.tet[i];
        }
        const int32_t pid = CAPTURE ? a.pid[i] : 0;
        bool gone = false;
        walk_one<CAPTURE>(a, px, py, pz, vx, vy, vz, t, pid, deposit_walk, n_cross, n_wall, n_lost, gone);
        a.x[i] = px; a.y[i] = py; a.z[i] = pz;
        a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
        a.tet[i] = gone ? -1 : t;  // dropped by the sort that follows the step
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        n_cross += __shfl_xor(n_cross, off, 64);
        n_wall += __shfl_xor(n_wall, off, 64);
        n_lost += __shfl_xor(n_lost, off, 64);
        n_foreign += __shfl_xor(n_foreign, off, 64);
    }
    // owned tets: the window sums (the tets beyond were zeroed at the start); this wave's own
    // LDS additions are ordered before these reads
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        int64_t *dst = a.acc_tet + (int64_t)k * a.nt + T0;
        const long long scale = k < 6 ? (long long)a.zq : (long long)a.zq * QH_SCALE;
        for (int j = lane; j < W; j += 64) dst[j] = scale * acc[k * kWin + j];
    }
    // event counters: crossings, wall hits, lost, posted pieces
    if (lane < 4) {
        const unsigned int v = lane == 0 ? n_cross : lane == 1 ? n_wall : lane == 2 ? n_lost : n_foreign + s_cnt[4];
        if (v) atomicAdd(&a.counters[(blockIdx.x & (QH_COUNTER_SLOTS - 1)) * 4 + lane], (unsigned long long)v);
        // lost particles also into the total of the whole step call, which no step clears
        if (lane == 2 && v) atomicAdd(&a.counters[4 * QH_COUNTER_SLOTS + QH_CNT_LOST_CALL], (unsigned long long)v);
    }
}

// Owned per-tet sums into edges and nodes: deterministic gathers over the incidence lists,
// 8 lanes per edge or node. Blocks are dealt to the 8 XCDs round-robin by the hardware; the
// block index is remapped so each XCD takes one contiguous range (its L2 then holds the
// neighbouring tets' sums the range needs, instead of every L2 fetching all of them).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nblocks) {
    const unsigned per = (nblocks + 7) / 8;
    const unsigned x = b & 7, k = b >> 3;
    const unsigned lb = x * per + k;
    return lb < nblocks ? lb : 0xffffffffu;
}

// Fixed-point headroom: a step's current on one edge or charge on one node beyond 2^60 (eight
// times below the int64 range; a piece is at most 64 * 2^40) is counted as an overflow risk.
constexpr long long kHeadroom = 1ll << 60;

template <int OFF, int LPI>
__global__ void __launch_bounds__(256) k_gather(int64_t nitems, const int32_t *__restrict__ ptr,
                                                const int32_t *__restrict__ lst,
                                                const int64_t *__restrict__ acc_tet, int64_t nt,
                                                int64_t *__restrict__ out,
                                                unsigned nblocks_grid, unsigned long long *headroom) {
    // LPI lanes per item; the grid is padded to a multiple of 8 blocks so the remap is a
    // bijection onto [0, grid)
    const unsigned lb = xcd_block(blockIdx.x, nblocks_grid);
    const int sub = threadIdx.x & (LPI - 1);
    const int64_t item = (int64_t)lb * (256 / LPI) + (threadIdx.x / LPI);
    int64_t s = 0;
    if (lb != 0xffffffffu && item < nitems) {
        for (int32_t j = ptr[item] + sub; j < ptr[item + 1]; j += LPI) {
            int32_t v = lst[j];
            s += acc_tet[(int64_t)(OFF + (v & 7)) * nt + (v >> 3)];
        }
    }
#pragma unroll
    for (int off = LPI / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LPI);
    if (sub == 0 && lb != 0xffffffffu && item < nitems) {
        const int64_t t = out[item] + s;
        out[item] = t;
        if (t > kHeadroom || t < -kHeadroom) atomicAdd(headroom, 1ull);
    }
}

// Mailbox m (tets [kMailTets m, kMailTets (m+1))) into acc_tet: each record's 10 values (as
// in the particle kernel) summed in LDS by tet, then added to the (already written) per-tet
// sums. One block per mailbox, so every tet has a single writer.
__global__ void __launch_bounds__(256) k_mail_apply(const unsigned int *__restrict__ mail_cnt,
                                                    const int32_t *__restrict__ mail, int32_t zq, int64_t nt,
                                                    int64_t *__restrict__ acc_tet) {
    const int o = blockIdx.x;
    const unsigned int cnt = min(mail_cnt[o], (unsigned)kMailCap);
    if (cnt == 0) return;
    __shared__ long long acc[10 * kMailTets];
    const int T0 = o * kMailTets;
    const int W = (int)min((int64_t)kMailTets, nt - T0);
    for (int j = threadIdx.x; j < 10 * kMailTets; j += 256) acc[j] = 0;
    __syncthreads();
    const int LE0[6] = {0, 0, 0, 1, 1, 2};
    const int LE1[6] = {1, 2, 3, 2, 3, 3};
    const int32_t *box = mail + (int64_t)o * kMailCap * kMailWords;
    for (unsigned int r = threadIdx.x; r < cnt; r += 256) {
        const uint4 pk = reinterpret_cast<const uint4 *>(box)[r];
        const int head = box[4 * kMailCap + r];
        const int tt = head & 0x7fffffff;
        const bool end = head < 0;
        int P0[4], P1[4];
        unpack_point(pk.x, pk.y, P0);
        unpack_point(pk.z, pk.w, P1);
        long long v[10];
#pragma unroll
        for (int j = 0; j < 6; ++j)
            v[j] = zq * ((long long)P0[LE0[j]] * P1[LE1[j]] - (long long)P1[LE0[j]] * P0[LE1[j]]);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[6 + j] = end ? (long long)zq * QH_SCALE * P1[j] : 0;
        const int slot = tt - T0;  // in [0, W): records are posted to the mailbox of their tet
#pragma unroll
        for (int k = 0; k < 10; ++k)
            if (v[k]) atomic_add_lds(&acc[k * kMailTets + slot], v[k]);
    }
    __syncthreads();
    // all loads of a thread issued before its stores
    constexpr int kPer = 10 * kMailTets / 256;
    long long vv[kPer], old[kPer];
    int64_t at[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = threadIdx.x + 256 * u;
        const int k = j / kMailTets, sl = j - k * kMailTets;
        vv[u] = sl < W ? acc[j] : 0;
        at[u] = (int64_t)k * nt + T0 + sl;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) old[u] = vv[u] ? acc_tet[at[u]] : 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u)
        if (vv[u]) acc_tet[at[u]] = old[u] + vv[u];
}

// owned tet ranges after a sort: own[b] = tet of the block's first particle, own[0] = 0,
// own[nblocks] = nt
__global__ void k_own(const int32_t *__restrict__ tet, int64_t n, int32_t nblocks, int32_t nt,
                      int32_t *__restrict__ own) {
    int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nblocks) return;
    own[b] = b == 0 ? 0 : b == nblocks ? nt : tet[(int64_t)b * kChunk];
}

hipError_t launch_particle_step(qh_ctx *c, Species &s, int sidx, bool capture) {
    if (s.n == 0) return hipSuccess;
    StepArgs a;
    a.geo = c->geo; a.frec = c->frec; a.tnodes = c->tnodes; a.tedges = c->tedges; a.tnbr = c->tnbr;
    a.x = s.x; a.y = s.y; a.z = s.zz; a.vx = s.vx; a.vy = s.vy; a.vz = s.vz;
    a.tet = s.tet; a.pid = s.id; a.own = s.own; a.n = s.n; a.nt = (int32_t)c->hm.Nt;
    a.mail_cnt = c->mail_cnt; a.mail = c->mail; a.ovf = s.ovf;
    a.hqm = (float)(0.5 * s.qm * c->phys.dt);
    a.dt = (float)c->phys.dt;
    a.zq = s.z;
    a.absorb = c->walls == QH_WALLS_ABSORB ? 1 : 0;
    a.g = c->g; a.Q = c->Q; a.acc_tet = c->acc_tet; a.counters = c->counters;
    a.species = sidx; a.cap = c->cap_segments; a.seg_count = c->seg_count; a.seg_buf = c->seg_buf;
    dim3 grid((unsigned)((s.n + kChunk - 1) / kChunk));
    const unsigned nmail = (unsigned)((c->hm.Nt + kMailTets - 1) / kMailTets);
    hipError_t e = hipMemsetAsync(c->mail_cnt, 0, sizeof(unsigned int) * nmail, c->stream);
    if (e != hipSuccess) return e;
    // few particles on a large mesh (the blocks' windows cannot cover it): one fill clears the
    // per-tet sums instead of each block zeroing a long owned range
    a.zeroed = (int64_t)grid.x * kWin < c->hm.Nt ? 1 : 0;
    if (a.zeroed && (e = hipMemsetAsync(c->acc_tet, 0, sizeof(int64_t) * 10 * c->hm.Nt, c->stream)) != hipSuccess)
        return e;
    if (capture) hipLaunchKernelGGL(k_particle_step<true>, grid, dim3(kBlock), 0, c->stream, a);
    else hipLaunchKernelGGL(k_particle_step<false>, grid, dim3(kBlock), 0, c->stream, a);
    const HostMesh &m = c->hm;
    hipLaunchKernelGGL(k_mail_apply, dim3(nmail), dim3(256), 0, c->stream, c->mail_cnt, c->mail, s.z, m.Nt, c->acc_tet);
    constexpr int kLpiE = 2, kLpiN = 8;  // lanes per edge / per node (edges border 4-6 tets, nodes ~24)
    const unsigned ge = (unsigned)(((m.Ne + 256 / kLpiE - 1) / (256 / kLpiE) + 7) / 8 * 8);
    const unsigned gn = (unsigned)(((m.Nn + 256 / kLpiN - 1) / (256 / kLpiN) + 7) / 8 * 8);
    unsigned long long *headroom = c->counters + 4 * QH_COUNTER_SLOTS + QH_CNT_HEADROOM_CALL;
    hipLaunchKernelGGL((k_gather<0, kLpiE>), dim3(ge), dim3(256), 0, c->stream, m.Ne, c->e2t_ptr, c->e2t, c->acc_tet,
                       m.Nt, c->g, ge, headroom);
    hipLaunchKernelGGL((k_gather<6, kLpiN>), dim3(gn), dim3(256), 0, c->stream, m.Nn, c->n2t_ptr, c->n2t, c->acc_tet,
                       m.Nt, c->Q, gn, headroom);
    return hipGetLastError();
}

int64_t qh_species_blocks(int64_t n) { return (n + kChunk - 1) / kChunk; }

// ------------------------------------------------------------------------------------------
// W0 charge of the present positions (after an upload).
__global__ void __launch_bounds__(256) k_charge(const float4 *__restrict__ geo, const int4 *__restrict__ tnodes,
                                                const float *__restrict__ x, const float *__restrict__ y,
                                                const float *__restrict__ z, const int32_t *__restrict__ tet,
                                                int64_t n, int32_t zq, int64_t *__restrict__ Q) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int t = tet[i];
    float l[4];
    int L[4];
    lam4(geo[3 * t], geo[3 * t + 1], geo[3 * t + 2], x[i], y[i], z[i], l);
    quantize(l, -1, L);
    int4 tn = tnodes[t];
    int nv[4] = {tn.x, tn.y, tn.z, tn.w};
    for (int q = 0; q < 4; ++q) atomic_add_i64(Q + nv[q], (long long)zq * QH_SCALE * L[q]);
}

// W0 charge of particles [first, n) of a species, added to Q.
hipError_t launch_charge_deposit(qh_ctx *c, Species &s, int64_t first) {
    const int64_t n = s.n - first;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_charge, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->geo,
                       c->tnodes, s.x + first, s.y + first, s.zz + first, s.tet + first, n, s.z, c->Q);
    return hipGetLastError();
}

// Ownership after particles are appended without a sort: own[0] = 0, the blocks past the old
// last one own no tets (own[b] = nt for b in (b0, b1]); the old last block keeps [own, nt).
__global__ void k_own_extend(int32_t *__restrict__ own, int32_t b0, int32_t b1, int32_t nt) {
    const int32_t b = b0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b > b1) return;
    own[b] = b == 0 ? 0 : (b == b0 ? own[b] : nt);
}

hipError_t launch_own_extend(qh_ctx *c, Species &s, int32_t b0, int32_t b1) {
    hipLaunchKernelGGL(k_own_extend, dim3((unsigned)((b1 - b0 + 1 + 255) / 256)), dim3(256), 0, c->stream, s.own, b0,
                       b1, (int32_t)c->hm.Nt);
    return hipGetLastError();
}

// E and B at points from the per-tet records the push reads (FP32): E = alpha + beta x (r - c),
// B constant in the tet.
__global__ void k_probe(const float4 *__restrict__ geo, const float4 *__restrict__ frec, int64_t n,
                        const double *__restrict__ xyz, const int32_t *__restrict__ tet, double *__restrict__ E,
                        double *__restrict__ B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = tet[i];
    const float4 A = geo[3 * t], Bg = geo[3 * t + 1], C = geo[3 * t + 2];
    const float4 F0 = frec[3 * t], F1 = frec[3 * t + 1], F2 = frec[3 * t + 2];
    const float dx = (float)xyz[3 * i] - A.w, dy = (float)xyz[3 * i + 1] - Bg.w, dz = (float)xyz[3 * i + 2] - C.w;
    E[3 * i] = F0.x + (F1.x * dz - F1.y * dy);
    E[3 * i + 1] = F0.y + (F1.y * dx - F0.w * dz);
    E[3 * i + 2] = F0.z + (F0.w * dy - F1.x * dx);
    B[3 * i] = F1.z;
    B[3 * i + 1] = F1.w;
    B[3 * i + 2] = F2.x;
}

// Point location: from the seed tet of the point's bucket, the straight segment from that tet's
// centroid to the point is walked face by face in the push's FP32 barycentrics, so the tet found
// is the one the push sees. A point on a wall up to rounding (its barycentric for the wall face
// above -kOnWall) belongs to the tet behind it. -1 when the segment leaves the mesh through a
// wall (the point is outside, or the domain is not convex along the segment) or crosses more
// than kLocateSteps tets.
constexpr int kLocateSteps = 4096;
constexpr float kOnWall = 1e-5f;
__global__ void __launch_bounds__(256) k_locate(int64_t n, const float *__restrict__ x, const float *__restrict__ y,
                                                const float *__restrict__ z, const float4 *__restrict__ geo,
                                                const int4 *__restrict__ tnbr, const int4 *__restrict__ tnodes,
                                                const int32_t *__restrict__ seed, float lx, float ly, float lz,
                                                float ix, float iy, float iz, int nx, int ny, int nz,
                                                int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float qx = x[i], qy = y[i], qz = z[i];
    const int bx = min(max((int)((qx - lx) * ix), 0), nx - 1);
    const int by = min(max((int)((qy - ly) * iy), 0), ny - 1);
    const int bz = min(max((int)((qz - lz) * iz), 0), nz - 1);
    int t = seed[(bz * ny + by) * nx + bx];
    float4 A = geo[3 * t], B = geo[3 * t + 1], C = geo[3 * t + 2];
    int4 on = tnodes[t], nb4 = tnbr[t];
    float px = A.w, py = B.w, pz = C.w;  // the centroid (barycentrics 1/4)
    float rx = qx - px, ry = qy - py, rz = qz - pz;
    int entry = -1;
    for (int step = 0; step < kLocateSteps; ++step) {
        float l[4], gl[4];
        lam4(A, B, C, px, py, pz, l);
        gl[1] = A.x * rx + A.y * ry + A.z * rz;
        gl[2] = B.x * rx + B.y * ry + B.z * rz;
        gl[3] = C.x * rx + C.y * ry + C.z * rz;
        gl[0] = -(gl[1] + gl[2] + gl[3]);
        int k = -1;
        float smin = 2.0f, lek = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r == entry) continue;
            const float le = l[r] + gl[r];
            if (!(le < 0.0f)) continue;
            const float s = l[r] <= 0.0f ? 0.0f : l[r] / (l[r] - le);
            if (s < smin) { smin = s; k = r; lek = le; }
        }
        if (k < 0) {
            out[i] = t;
            return;
        }
        px = __fmaf_rn(smin, rx, px); py = __fmaf_rn(smin, ry, py); pz = __fmaf_rn(smin, rz, pz);
        const float rem = 1.0f - smin;
        rx *= rem; ry *= rem; rz *= rem;
        const int nb = k == 0 ? nb4.x : k == 1 ? nb4.y : k == 2 ? nb4.z : nb4.w;
        if (nb < 0) {
            out[i] = lek > -kOnWall ? t : -1;
            return;
        }
        const int4 nn = tnodes[nb];
        const int ov[4] = {on.x, on.y, on.z, on.w}, nv[4] = {nn.x, nn.y, nn.z, nn.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            bool found = false;
#pragma unroll
            for (int r = 0; r < 4; ++r) found |= ov[r] == nv[j];
            if (!found) entry = j;
        }
        t = nb;
        A = geo[3 * nb]; B = geo[3 * nb + 1]; C = geo[3 * nb + 2];
        on = nn;
        nb4 = tnbr[nb];
    }
    out[i] = -1;
}

hipError_t launch_locate(qh_ctx *c, int64_t n, const float *x, const float *y, const float *z, int32_t *tet) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_locate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, x, y, z, c->geo,
                       c->tnbr, c->tnodes, c->loc_seed, c->loc_lo[0], c->loc_lo[1], c->loc_lo[2], c->loc_inv[0],
                       c->loc_inv[1], c->loc_inv[2], c->loc_n[0], c->loc_n[1], c->loc_n[2], tet);
    return hipGetLastError();
}

hipError_t launch_probe(qh_ctx *c, int64_t n, const double *xyz, const int32_t *tet, double *E, double *B) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->geo, c->frec, n, xyz,
                       tet, E, B);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Integer deposit from explicit lists.
__global__ void k_deposit_segments(const int32_t *__restrict__ tedges, int64_t n,
                                   const int32_t *__restrict__ st, const int32_t *__restrict__ l0,
                                   const int32_t *__restrict__ l1, const int32_t *__restrict__ sz,
                                   int64_t *__restrict__ g) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int LE0[6] = {0, 0, 0, 1, 1, 2};
    const int LE1[6] = {1, 2, 3, 2, 3, 3};
    int t = st[s];
    for (int k = 0; k < 6; ++k) {
        long long v = (long long)l0[4 * s + LE0[k]] * l1[4 * s + LE1[k]] -
                      (long long)l1[4 * s + LE0[k]] * l0[4 * s + LE1[k]];
        v *= sz[s];
        if (v) atomic_add_i64(g + tedges[8 * (int64_t)t + k], v);
    }
}

__global__ void k_deposit_points(const int4 *__restrict__ tnodes, int64_t n, const int32_t *__restrict__ pt,
                                 const int32_t *__restrict__ pl, const int32_t *__restrict__ pz,
                                 int64_t *__restrict__ Q) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int4 tn = tnodes[pt[p]];
    int nv[4] = {tn.x, tn.y, tn.z, tn.w};
    for (int q = 0; q < 4; ++q) atomic_add_i64(Q + nv[q], (long long)pz[p] * QH_SCALE * pl[4 * p + q]);
}

hipError_t launch_deposit_lists(qh_ctx *c, int64_t n_seg, const int32_t *seg_tet, const int32_t *l0,
                                const int32_t *l1, const int32_t *sz, int64_t n_pt, const int32_t *pt_tet,
                                const int32_t *pl, const int32_t *pz, int64_t *g, int64_t *Q) {
    if (n_seg > 0)
        hipLaunchKernelGGL(k_deposit_segments, dim3((unsigned)((n_seg + 255) / 256)), dim3(256), 0, c->stream,
                           c->tedges, n_seg, seg_tet, l0, l1, sz, g);
    if (n_pt > 0)
        hipLaunchKernelGGL(k_deposit_points, dim3((unsigned)((n_pt + 255) / 256)), dim3(256), 0, c->stream,
                           c->tnodes, n_pt, pt_tet, pl, pz, Q);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Invariants: continuity (G^T g == Q - Q_old at every node; with absorbing walls at every node
// off the walls, since the charge of absorbed particles leaves through them) and D b == D b0
// in every tet.
__global__ void k_continuity(const int32_t *__restrict__ ptr, const int32_t *__restrict__ lst,
                             const int64_t *__restrict__ g, const int64_t *__restrict__ Q,
                             const int64_t *__restrict__ Qo, const uint8_t *__restrict__ skip, int64_t nn,
                             unsigned long long *bad, unsigned long long *bad_total) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn || (skip && skip[n])) return;
    int64_t s = 0;
    for (int j = ptr[n]; j < ptr[n + 1]; ++j) {
        int32_t v = lst[j];
        s += v > 0 ? g[v - 1] : -g[-v - 1];
    }
    if (s != Q[n] - Qo[n]) {
        atomicAdd(bad, 1ull);
        atomicAdd(bad_total, 1ull);
    }
}

__global__ void k_divb(const int32_t *__restrict__ tfaces, const int8_t *__restrict__ tsign,
                       const int64_t *__restrict__ b, int32_t nt, int64_t *__restrict__ out,
                       const int64_t *__restrict__ ref, unsigned long long *bad, unsigned long long *bad_total) {
    int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int64_t s = (int64_t)tsign[t] * (b[tfaces[4 * t]] - b[tfaces[4 * t + 1]] + b[tfaces[4 * t + 2]] - b[tfaces[4 * t + 3]]);
    if (out) out[t] = s;
    if (ref && s != ref[t]) {
        atomicAdd(bad, 1ull);
        if (bad_total) atomicAdd(bad_total, 1ull);
    }
}

hipError_t launch_verify(qh_ctx *c, bool check_divb) {
    int64_t nn = c->hm.Nn;
    hipLaunchKernelGGL(k_continuity, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c->stream, c->n2e_ptr,
                       c->n2e, c->g, c->Q, c->Q_old, c->walls == QH_WALLS_ABSORB ? c->wall_node_d : nullptr, nn,
                       c->counters + 4 * QH_COUNTER_SLOTS + QH_CNT_CONT, c->counters + 4 * QH_COUNTER_SLOTS + QH_CNT_CONT_CALL);
    if (check_divb) {
        int32_t nt = (int32_t)c->hm.Nt;
        hipLaunchKernelGGL(k_divb, dim3((nt + 255) / 256), dim3(256), 0, c->stream, c->tfaces, c->tsign, c->b, nt,
                           (int64_t *)nullptr, c->divb0, c->counters + 4 * QH_COUNTER_SLOTS + QH_CNT_DIVB,
                           c->counters + 4 * QH_COUNTER_SLOTS + QH_CNT_DIVB_CALL);
    }
    return hipGetLastError();
}

// Tets where D b != 0 for a caller's device flux vector, counted into *bad.
hipError_t launch_divb_check(qh_ctx *c, const int64_t *b, unsigned long long *bad) {
    int32_t nt = (int32_t)c->hm.Nt;
    hipLaunchKernelGGL(k_divb, dim3((nt + 255) / 256), dim3(256), 0, c->stream, c->tfaces, c->tsign, b, nt,
                       (int64_t *)nullptr, (const int64_t *)c->divb0, bad, (unsigned long long *)nullptr);
    return hipGetLastError();
}

// e_out <- e_in on the interior edges, 0 elsewhere (PEC walls); x[i] <- e_in[int_edges[i]]
__global__ void k_fields_in(int32_t n_int, const int32_t *__restrict__ int_edges, const double *__restrict__ e_in,
                            double *__restrict__ e_out, double *__restrict__ x) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    const int32_t g = int_edges[i];
    const double v = e_in[g];
    e_out[g] = v;
    if (x) x[i] = v;
}

hipError_t launch_fields_in(qh_ctx *c, const double *e_in, double *x) {
    const int32_t n = (int32_t)c->hm.int_edges.size();
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fields_in, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->int_edges, e_in, c->e, x);
    return hipGetLastError();
}

hipError_t launch_divb(qh_ctx *c, int64_t *out) {
    int32_t nt = (int32_t)c->hm.Nt;
    hipLaunchKernelGGL(k_divb, dim3((nt + 255) / 256), dim3(256), 0, c->stream, c->tfaces, c->tsign, c->b, nt,
                       out, (const int64_t *)nullptr, (unsigned long long *)nullptr, (unsigned long long *)nullptr);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Counting sort of one species by tet: histogram, exclusive scan, scatter.
// Particles are nearly sorted by tet between sorts, so a wave sees a few runs of equal tets:
// the first lane of each run (its head) adds the run's length, one atomic per run.
__device__ __forceinline__ void wave_runs(int t, bool valid, int &head, int &len, int &rank) {
    const int lane = __lane_id();
    const int prev = __shfl_up(t, 1, 64);
    const bool is_head = valid && (lane == 0 || prev != t);
    const unsigned long long heads = __ballot(is_head);
    const unsigned long long valid_m = __ballot(valid);
    // my run's head: the highest head at or below this lane
    const unsigned long long below = heads & ((2ull << lane) - 1ull);  // lanes 0..lane
    head = 63 - __clzll((long long)below);
    // run end: the next head above this lane, else the end of the valid lanes
    const unsigned long long above = heads & ~((2ull << lane) - 1ull);
    const int vend = 64 - __clzll((long long)valid_m);
    const int next = above ? __ffsll((unsigned long long)above) - 1 : vend;
    len = next - head;
    rank = lane - head;
}

// Bucket of a particle: its tet, or nt for one that left through an absorbing wall (tet -1).
__device__ __forceinline__ int sort_key(int t, int32_t nt) { return t < 0 ? nt : t; }

__global__ void k_hist(const int32_t *__restrict__ tet, int64_t n, int32_t nt, int32_t *__restrict__ hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    const int t = valid ? sort_key(tet[i], nt) : -1;
    int head, len, rank;
    wave_runs(t, valid, head, len, rank);
    if (valid && rank == 0) atomicAdd(&hist[t], len);
}

// scan over chunks of 1024: per-chunk sums
__global__ void __launch_bounds__(1024) k_scan_sums(const int32_t *__restrict__ in, int32_t n,
                                                    int32_t *__restrict__ sums) {
    __shared__ int32_t sh[1024];
    int32_t i = blockIdx.x * 1024 + threadIdx.x;
    sh[threadIdx.x] = i < n ? in[i] : 0;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = sh[0];
}

// exclusive scan of the chunk sums in one block (serial over groups of 1024)
__global__ void __launch_bounds__(1024) k_scan_top(int32_t *__restrict__ sums, int32_t m) {
    __shared__ int32_t sh[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < m; base += 1024) {
        int32_t i = base + threadIdx.x;
        int32_t v = i < m ? sums[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < m) sums[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) k_scan_final(const int32_t *__restrict__ in, int32_t n,
                                                     const int32_t *__restrict__ sums,
                                                     int32_t *__restrict__ out) {
    __shared__ int32_t sh[1024];
    int32_t i = blockIdx.x * 1024 + threadIdx.x;
    int32_t v = i < n ? in[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = sums[blockIdx.x] + sh[threadIdx.x] - v;
}

// Destination slot of every particle (its bucket's cursor, one atomic per run of equal keys in a
// wave), recorded as perm[slot] = source index. After many steps of drift the runs are short and
// the slots of a wave's particles scatter; moving the particle state in a second pass, in slot
// order (k_permute), keeps the state's stores coalesced and leaves the scatter to the reads,
// which stay near their slots.
__global__ void k_sort_slots(int64_t n, const int32_t *__restrict__ tet, int32_t nt, int32_t *__restrict__ cursor,
                             int32_t *__restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    const int t = valid ? sort_key(tet[i], nt) : -1;
    int head, len, rank;
    wave_runs(t, valid, head, len, rank);
    int32_t first = 0;
    if (valid && rank == 0) first = atomicAdd(&cursor[t], len);
    first = __shfl(first, head, 64);
    if (valid) perm[first + rank] = (int32_t)i;
}

__global__ void k_permute(int64_t n, const int32_t *__restrict__ perm, const float *__restrict__ x,
                          const float *__restrict__ y, const float *__restrict__ z, const float *__restrict__ vx,
                          const float *__restrict__ vy, const float *__restrict__ vz,
                          const int32_t *__restrict__ tet, const int32_t *__restrict__ id, float *__restrict__ ox,
                          float *__restrict__ oy, float *__restrict__ oz, float *__restrict__ ovx,
                          float *__restrict__ ovy, float *__restrict__ ovz, int32_t *__restrict__ otet,
                          int32_t *__restrict__ oid) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t i = perm[j];
    ox[j] = x[i]; oy[j] = y[i]; oz[j] = z[i];
    ovx[j] = vx[i]; ovy[j] = vy[i]; ovz[j] = vz[i];
    otet[j] = tet[i]; oid[j] = id[i];
}

int qh_sort_species(qh_ctx *c, Species &s) {
    if (s.n == 0) return QH_OK;
    int32_t nt = (int32_t)c->hm.Nt;
    const int32_t nk = nt + 1;  // buckets: the tets, then the particles absorbed by a wall
    QH_HIP(c, hipMemsetAsync(c->hist, 0, sizeof(int32_t) * nk, c->stream));
    unsigned pb = (unsigned)((s.n + 255) / 256);
    hipLaunchKernelGGL(k_hist, dim3(pb), dim3(256), 0, c->stream, s.tet, s.n, nt, c->hist);
    int32_t chunks = (nk + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_sums, dim3(chunks), dim3(1024), 0, c->stream, c->hist, nk, c->scan_tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, c->stream, c->scan_tmp, chunks);
    hipLaunchKernelGGL(k_scan_final, dim3(chunks), dim3(1024), 0, c->stream, c->hist, nk, c->scan_tmp, c->cursor);
    const bool absorb = c->walls == QH_WALLS_ABSORB;
    int32_t live = (int32_t)s.n;  // the start of the last bucket
    if (absorb) QH_HIP(c, hipMemcpyAsync(&live, c->cursor + nt, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    if (c->perm_cap < s.n) {
        // queued work may still read the old index buffer: released after the stream passes it
        QH_HIP(c, hipStreamSynchronize(c->stream));
        qh_release(c, c->perm);
        c->perm_cap = 0;
        int rc = qh_alloc(c, &c->perm, (size_t)s.cap);
        if (rc) return rc;
        c->perm_cap = s.cap;
    }
    hipLaunchKernelGGL(k_sort_slots, dim3(pb), dim3(256), 0, c->stream, s.n, s.tet, nt, c->cursor, c->perm);
    hipLaunchKernelGGL(k_permute, dim3(pb), dim3(256), 0, c->stream, s.n, (const int32_t *)c->perm, s.x, s.y, s.zz,
                       s.vx, s.vy, s.vz, s.tet, s.id, s.sx, s.sy, s.sz, s.svx, s.svy, s.svz, s.stet, s.sid);
    QH_HIP(c, hipGetLastError());
    std::swap(s.x, s.sx); std::swap(s.y, s.sy); std::swap(s.zz, s.sz);
    std::swap(s.vx, s.svx); std::swap(s.vy, s.svy); std::swap(s.vz, s.svz);
    std::swap(s.tet, s.stet); std::swap(s.id, s.sid);
    if (absorb) {
        QH_HIP(c, hipStreamSynchronize(c->stream));
        s.n = live;  // the absorbed particles sit past the live ones and are dropped
        if (s.n == 0) return QH_OK;
    }
    int32_t nb = (int32_t)qh_species_blocks(s.n);
    hipLaunchKernelGGL(k_own, dim3((nb + 1 + 255) / 256), dim3(256), 0, c->stream, s.tet, s.n, nb, nt, s.own);
    QH_HIP(c, hipGetLastError());
    return QH_OK;
}
