// Implicit field update on gfx950 (Sec. IV.B): FP64 CSR products, preconditioned conjugate
// gradients with FP64 dot products reduced in a fixed order (deterministic iteration counts),
// the Gauss-law solve for the non-solenoidal part and the integer Faraday update.
//
// Edge system (trapezoidal rule on eq. maxwell_semi, b^{n+1} eliminated):
//   ([*eps] + tau S) e* = ([*eps] - tau S) e^n + dt C^T [*mu^-1] b^n - u_q g,   tau = dt^2/4
// Gauss law (eq. discreteGauss): G^T [*eps] G delta = rho^{n+1} - G^T [*eps] e*, e = e* + G delta
// Faraday: b^{n+1} = b^n - C round((dt/2)(e^{n+1} + e^n)/u_b)  (D C = 0 keeps D b fixed).
#include <algorithm>
#include <cmath>

#include "qh_internal.h"
#include "qh_spmv.h"

namespace {

constexpr int kThreads = 256;
constexpr int kLpr = 8;          // lanes per CSR row
constexpr int kMaxBlocks = 2048; // fixed grid of the reducing kernels (fixed summation order)

// device scalar slots of a CgWork: S_RZ + parity r.z (double-buffered), S_RR r.r, S_THR2 the
// target on r.r, S_BB b.b, S_RES the true-residual sums, S_SCALE the mixed-precision solve's
// residual scale, S_HIST a ring of r.r by iteration
// (the stall rule compares r.r with its value ten iterations before)
enum { S_RZ = 0, S_RZ1, S_RR, S_THR2, S_BB, S_RES = 8, S_SCALE = 10, S_HIST = 16, S_NSCAL = 32 };
constexpr int kHist = 16;
// flags[0] after a solve: why the iteration stopped
enum { CG_RUNNING = 0, CG_CONVERGED = 1, CG_STALLED = 2, CG_NONFINITE = 3 };
// stall rule of the learned solve: r.z <= 0, or ||r|| not 10 % lower than ten iterations before
constexpr int kStallWindow = 10;
constexpr double kStallRatio2 = 0.81;  // (1 - 0.1)^2 on r.r

__device__ __forceinline__ double wave_sum_lpr(double v) {
#pragma unroll
    for (int off = kLpr / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kLpr);
    return v;
}

inline unsigned grid_rows(int64_t nrows) {
    int64_t b = (nrows * kLpr + kThreads - 1) / kThreads;
    b = b < kMaxBlocks ? (b < 1 ? 1 : b) : kMaxBlocks;
    return (unsigned)((b + 7) / 8 * 8);
}
inline unsigned grid_elems(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b < kMaxBlocks ? (b < 1 ? 1 : b) : kMaxBlocks);
}

// Rows of a CSR kernel: each block takes one contiguous range, and the block index is
// remapped so that each of the 8 XCDs (which receive blocks round-robin) covers one
// contiguous span of rows: neighbouring rows share the vector entries they gather, and
// those then stay in one XCD's L2. Grids are multiples of 8 blocks.
struct Rows {
    int64_t begin, end;
};
__device__ __forceinline__ Rows block_rows(int64_t n) {
    const unsigned nb = gridDim.x, per_x = nb / 8;
    const unsigned lb = (blockIdx.x & 7) * per_x + (blockIdx.x >> 3);
    const int64_t per = (n + nb - 1) / nb;
    Rows r;
    r.begin = (int64_t)lb * per;
    r.end = r.begin + per < n ? r.begin + per : n;
    return r;
}

// ---------------------------------------------------------------------------------------
// CG kernels. Cross-block sums never use in-kernel synchronisation: a kernel writes one
// partial per block and every block of the NEXT kernel sums all partials itself in the same
// fixed order (a few KB from L2), so the result is identical in every block, deterministic,
// and needs no device-scope fence (which would write back the whole L2 on this part).
// Scalars: scal[S_RZ + parity] holds r.z of the current iterate (double-buffered by the
// iteration parity so no block reads a slot another block of the same kernel writes).

// Every block: sum of part[0..m) in a fixed order, returned to all threads.
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int m, double *sh) {
    double s = 0.0;
    for (int j = threadIdx.x; j < m; j += kThreads) s += part[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += sh[w];
    return t;
}

// Block-wide sum of NV values, written as this block's partials part[k * kMaxBlocks + block].
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *__restrict__ part) {
    __shared__ double sh[NV][kThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += sh[threadIdx.x][w];
        part[threadIdx.x * kMaxBlocks + blockIdx.x] = t;
    }
}

// init: r = b - A x, z = D^-1 r, p_old = 0; partials of r.z, r.r, b.b
__global__ void __launch_bounds__(kThreads) k_cg_init(const int2 *__restrict__ tiles, int32_t ntiles,
                                                      const int32_t *__restrict__ ptr,
                                                      const TileCols cols,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ b,
                                                      const double *__restrict__ dinv,
                                                      double *__restrict__ r, double *__restrict__ z,
                                                      double *__restrict__ p_old, double *__restrict__ part) {
    __shared__ double prod[kTileCap];
    double acc[3] = {0.0, 0.0, 0.0};
    tile_spmv(tiles, ntiles, ptr, cols, val, x, prod, [&](int32_t row) { return make_double2(b[row], dinv[row]); },
              [&](int32_t row, double s, double2 bd) {
        const double bb = bd.x;
        const double rr = bb - s;
        const double zz = rr * bd.y;
        r[row] = rr;
        z[row] = zz;
        p_old[row] = 0.0;
        acc[0] += rr * zz;
        acc[1] += rr * rr;
        acc[2] += bb * bb;
    });
    write_partials<3>(acc, part);
}

// Why an iteration stops, from r.r and r.z of the present iterate (the same sums, so the same
// decision, in every block): non-finite values, convergence, and for the learned
// preconditioner the stall rule (r.z <= 0 means M is not positive definite on r; ||r|| less
// than 10 % lower than ten iterations before). hist: r.r by iteration (ring), or null.
__device__ __forceinline__ int cg_state(double rr, double rz, double thr2, int stall, int32_t k, const double *hist) {
    if (!(rr == rr) || !(rz == rz) || rr > 1.7976931348623157e308) return CG_NONFINITE;
    if (rr <= thr2) return CG_CONVERGED;
    if (stall) {
        if (!(rz > 0.0)) return CG_STALLED;
        if (hist && k >= kStallWindow && rr > kStallRatio2 * hist[(k - kStallWindow) & (kHist - 1)]) return CG_STALLED;
    }
    return CG_RUNNING;
}

// one block: totals of the init partials; threshold; convergence flag
__global__ void __launch_bounds__(kThreads) k_cg_start(const double *__restrict__ part, int m,
                                                       const double *__restrict__ rz_part, int m_rz, double *scal,
                                                       int32_t *flags, double tol2, const double *abs_thr2, int stall) {
    __shared__ double sh[kThreads / 64];
    double rz = sum_partials(rz_part, m_rz, sh);
    double rr = sum_partials(part + kMaxBlocks, m, sh);
    double bb = sum_partials(part + 2 * kMaxBlocks, m, sh);
    if (threadIdx.x == 0) {
        double thr2 = abs_thr2 ? *abs_thr2 : tol2 * bb;
        scal[S_RZ] = rz;
        scal[S_RR] = rr;
        scal[S_BB] = bb;
        scal[S_THR2] = thr2;
        scal[S_HIST] = rr;
        flags[0] = cg_state(rr, rz, thr2, stall, 0, nullptr);
        flags[1] = 0;
    }
}

// Iteration k (parity par = k & 1). For k > 0 first finish the previous update: r.z and
// r.r from its partials, convergence test, beta. Then, with w = A z (the only gathered
// vector), p = z + beta p and q = A p = w + beta q in place (own rows only), and the
// partials of p.q. Gathering one vector instead of z and p halves the scattered loads.
// VT, XT: the matrix values' and the vectors' types (FP64, or FP32 in the inner iterations of
// the mixed-precision solve; products, sums and dot products are FP64 either way).
template <typename VT, typename XT>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) k_cg_spmv(int32_t n, const int2 *__restrict__ tiles, int32_t ntiles,
                                                      const int32_t *__restrict__ ptr,
                                                      const TileCols cols,
                                                      const VT *__restrict__ val,
                                                      const XT *__restrict__ z,
                                                      XT *__restrict__ p, XT *__restrict__ q,
                                                      const double *__restrict__ rz_part, int m_rz,
                                                      const double *__restrict__ rr_part, int m_rr,
                                                      double *__restrict__ part, double *scal, int32_t *flags,
                                                      int32_t k, int32_t par, int stall) {
    if (flags[0]) return;
    __shared__ double sh[kThreads / 64];
    __shared__ double prod[kTileCap];
    double beta = 0.0;
    if (k > 0) {
        double rz_new = sum_partials(rz_part, m_rz, sh);
        double rr = sum_partials(rr_part, m_rr, sh);
        // the ring slot read (k - 10) differs from the one written (k): no block reads what
        // block 0 writes in this launch
        const int state = cg_state(rr, rz_new, scal[S_THR2], stall, k, scal + S_HIST);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[S_RZ + (par ^ 1)] = rz_new;
            scal[S_RR] = rr;
            scal[S_HIST + (k & (kHist - 1))] = rr;
            flags[1] = k;
            if (state) flags[0] = state;
        }
        if (state) return;  // the same decision in every block (same sums, same order)
        beta = rz_new / scal[S_RZ + par];
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[S_RZ + 1] = scal[S_RZ];
    }
    double acc[1] = {0.0};
    tile_spmv(tiles, ntiles, ptr, cols, val, z, prod, [&](int32_t) { return 0; },
              [&](int32_t row, double s, int) {
        const XT pn = (XT)(k > 0 ? (double)z[row] + beta * (double)p[row] : (double)z[row]);
        const XT qn = (XT)(k > 0 ? s + beta * (double)q[row] : s);
        p[row] = pn;
        q[row] = qn;
        acc[0] += (double)pn * (double)qn;
    });
    write_partials<1>(acc, part);
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; with Jacobi also z = D^-1 r; partials of
// r.z (Jacobi) and r.r of the stored values. XT: the vectors' type, as in k_cg_spmv.
template <bool JAC, typename XT>
__global__ void __launch_bounds__(kThreads) k_cg_update(int32_t n, XT *__restrict__ x,
                                                        XT *__restrict__ r, XT *__restrict__ z,
                                                        const XT *__restrict__ p,
                                                        const XT *__restrict__ q,
                                                        const XT *__restrict__ dinv,
                                                        const double *__restrict__ qpart, double *__restrict__ part,
                                                        int m, const double *scal, const int32_t *flags, int32_t par) {
    if (flags[0]) return;
    __shared__ double sh[kThreads / 64];
    const double alpha = scal[S_RZ + (par ^ 1)] / sum_partials(qpart, m, sh);
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        x[i] = (XT)((double)x[i] + alpha * (double)p[i]);
        const XT ri = (XT)((double)r[i] - alpha * (double)q[i]);
        r[i] = ri;
        if (JAC) {
            const XT zi = (XT)((double)ri * (double)dinv[i]);
            z[i] = zi;
            acc[0] += (double)ri * (double)zi;
        }
        acc[1] += (double)ri * (double)ri;
    }
    write_partials<2>(acc, part);
}

// Mixed-precision solve. Outer step: r = b - A x in FP64, stored, with partials of r.r and b.b.
__global__ void __launch_bounds__(kThreads) k_res_store(const int2 *__restrict__ tiles, int32_t ntiles,
                                                        const int32_t *__restrict__ ptr, const TileCols cols,
                                                        const double *__restrict__ val, const double *__restrict__ x,
                                                        const double *__restrict__ b, double *__restrict__ r,
                                                        double *__restrict__ part) {
    __shared__ double prod[kTileCap];
    double acc[2] = {0.0, 0.0};
    tile_spmv(tiles, ntiles, ptr, cols, val, x, prod, [&](int32_t row) { return b[row]; },
              [&](int32_t row, double s, double bb) {
        const double ri = bb - s;
        r[row] = ri;
        acc[0] += ri * ri;
        acc[1] += bb * bb;
    });
    write_partials<2>(acc, part);
}

// Mixed-precision solve. Start: the FP32 system A d = r0 / s, s = ||r0|| (a unit right-hand
// side), from d = 0: r32 = r0 / s, d = p = 0, with Jacobi z = D^-1 r32; partials of r.z (Jacobi),
// r.r and b.b (= r.r here). rr: ||r0||^2 on the device; s is kept in scal[S_SCALE] for the solve.
template <bool JAC>
__global__ void __launch_bounds__(kThreads) k_inner_init(int32_t n, const double *__restrict__ r, const double *rr,
                                                         double *scal, float *__restrict__ r32,
                                                         float *__restrict__ x32, float *__restrict__ z32,
                                                         float *__restrict__ p32, const float *__restrict__ dinv32,
                                                         double *__restrict__ part) {
    const double s = sqrt(*rr), inv = 1.0 / s;
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_SCALE] = s;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const float ri = (float)(r[i] * inv);
        r32[i] = ri;
        x32[i] = 0.0f;
        p32[i] = 0.0f;
        if (JAC) {
            const float zi = (float)((double)ri * (double)dinv32[i]);
            z32[i] = zi;
            acc[0] += (double)ri * (double)zi;
        }
        acc[1] += (double)ri * (double)ri;
    }
    acc[2] = acc[1];
    write_partials<3>(acc, part);
}

// Reliable update, first half: x += s d in FP64 and d = 0.
__global__ void k_refine(int32_t n, double *__restrict__ x, float *__restrict__ d, const double *scal) {
    const double s = scal[S_SCALE];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += s * (double)d[i];
        d[i] = 0.0f;
    }
}

// Reliable update, second half (after r = b - A x in FP64): the recurrence's residual replaced by
// r32 = r / s, with Jacobi z = D^-1 r32, and the partials of r.z (Jacobi) and r.r written where
// the update kernel writes them, so the iteration continues with the next product (its beta
// from the new r.z), and the stop flag is cleared. The stall rule's history of r.r goes on: the
// replaced residual differs from the recurrence's by its FP32 drift only, far below the rule's
// 10 % over ten iterations while the solve converges, and a stalled solve stays stalled.
template <bool JAC>
__global__ void __launch_bounds__(kThreads) k_replace(int32_t n, const double *__restrict__ r, double *scal,
                                                      float *__restrict__ r32, float *__restrict__ z32,
                                                      const float *__restrict__ dinv32, double *__restrict__ part,
                                                      int32_t *flags) {
    const double inv = 1.0 / scal[S_SCALE];
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const float ri = (float)(r[i] * inv);
        r32[i] = ri;
        if (JAC) {
            const float zi = (float)((double)ri * (double)dinv32[i]);
            z32[i] = zi;
            acc[0] += (double)ri * (double)zi;
        }
        acc[1] += (double)ri * (double)ri;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) flags[0] = CG_RUNNING;
    write_partials<2>(acc, part);
}

template <typename S, typename D>
__global__ void k_convert(int64_t n, const S *__restrict__ in, D *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (D)in[i];
}

// one block, after a batch: finish the last update's convergence test
__global__ void __launch_bounds__(kThreads) k_cg_check(const double *__restrict__ upart, int m, double *scal,
                                                       int32_t *flags, int32_t k) {
    if (flags[0]) return;
    __shared__ double sh[kThreads / 64];
    double rr = sum_partials(upart + kMaxBlocks, m, sh);
    if (threadIdx.x == 0) {
        scal[S_RR] = rr;
        flags[1] = k;
        // convergence or a non-finite residual; the stall rule waits for the next product
        // kernel, which also has r.z
        const int state = cg_state(rr, 1.0, scal[S_THR2], 0, k, nullptr);
        if (state) flags[0] = state;
    }
}

__global__ void k_diag_inv(int32_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, double *__restrict__ dinv) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int32_t j = ptr[i]; j < ptr[i + 1]; ++j)
        if (col[j] == i) d = val[j];
    dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
}

// A = [*eps] + tau S and the right-hand-side matrix [*eps] - tau S on one pattern
__global__ void k_axpy_vals(int64_t n, const double *__restrict__ a, const double *__restrict__ s, double tau,
                            double *__restrict__ out, double *__restrict__ out_m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        out[i] = a[i] + tau * s[i];
        out_m[i] = a[i] - tau * s[i];
    }
}

// Edge right-hand side in two tiled passes over the interior edges:
//   rhs_i = sum_j ([*eps] - tau S)_ij e_j - u_q g[int_edge_i]          (k_edge_rhs_e)
//   rhs_i += dt u_b sum_f (C^T [*mu^-1])_if b_f                          (k_edge_rhs_b)
__global__ void __launch_bounds__(kThreads) k_edge_rhs_e(const int2 *__restrict__ tiles, int32_t ntiles,
                                                         const int32_t *__restrict__ ptr,
                                                         const TileCols cols,
                                                         const double *__restrict__ mval,
                                                         const double *__restrict__ e,
                                                         const int64_t *__restrict__ g,
                                                         const int32_t *__restrict__ int_edges, double u_q,
                                                         double *__restrict__ rhs) {
    __shared__ double prod[kTileCap];
    tile_spmv(tiles, ntiles, ptr, cols, mval, e, prod, [&](int32_t row) { return g[int_edges[row]]; },
              [&](int32_t row, double s, int64_t gi) { rhs[row] = s - u_q * (double)gi; });
}

__global__ void __launch_bounds__(kThreads) k_edge_rhs_b(const int2 *__restrict__ tiles, int32_t ntiles,
                                                         const int32_t *__restrict__ ptr,
                                                         const TileCols cols,
                                                         const double *__restrict__ cval,
                                                         const int64_t *__restrict__ b, double dtub,
                                                         double *__restrict__ rhs) {
    __shared__ double prod[kTileCap];
    tile_spmv(tiles, ntiles, ptr, cols, cval, b, prod, [&](int32_t row) { return rhs[row]; },
              [&](int32_t row, double t, double r0) { rhs[row] = r0 + dtub * t; });
}

// Gauss residual rg = rho - G^T [*eps] e on interior nodes, rho = u_q (Q_bg - Q);
// threshold thr2 = (tol_n (||rho|| + || |G^T [*eps]| |e| ||))^2: the residual is measured
// against the size of the terms that cancel in G^T [*eps] e (normwise backward error), so
// the tolerance stays above the FP64 rounding floor when the charge is small against E.
__global__ void __launch_bounds__(kThreads) k_gauss_rhs(int32_t n, const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ e,
                                                        const int64_t *__restrict__ Qbg,
                                                        const int64_t *__restrict__ Q,
                                                        const int32_t *__restrict__ int_nodes, double u_q,
                                                        const double *__restrict__ dbnd,
                                                        double *__restrict__ rg, double *__restrict__ rho_out,
                                                        double *__restrict__ part) {
    const int sub = threadIdx.x % kLpr;
    const Rows rr_ = block_rows(n);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t row = rr_.begin + threadIdx.x / kLpr; row < rr_.end; row += kThreads / kLpr) {
        double s = 0.0, sa = 0.0;
        for (int32_t j = ptr[row] + sub; j < ptr[row + 1]; j += kLpr) {
            double t = val[j] * e[col[j]];
            s += t;
            sa += fabs(t);
        }
        s = wave_sum_lpr(s);
        sa = wave_sum_lpr(sa);
        if (sub == 0) {
            int32_t gn = int_nodes[row];
            // charge, plus the normal flux a plane wave brought in through a natural boundary
            double rho = u_q * (double)(Qbg[gn] - Q[gn]) + (dbnd ? dbnd[gn] : 0.0);
            double r = rho - s;
            rg[row] = r;
            if (rho_out) rho_out[row] = rho;
            acc[0] += rho * rho;
            acc[1] += sa * sa;
            acc[2] += r * r;
        }
    }
    write_partials<3>(acc, part);
}

// one block: out[0] = (tol_n scale)^2, out[1] = scale, out[2] = ||r||^2, out[3] = ||rho||
__global__ void __launch_bounds__(kThreads) k_gauss_finish(const double *__restrict__ part, int m, double *out,
                                                           double tol_n) {
    __shared__ double sh[kThreads / 64];
    double a = sum_partials(part, m, sh);
    double b = sum_partials(part + kMaxBlocks, m, sh);
    double c = sum_partials(part + 2 * kMaxBlocks, m, sh);
    if (threadIdx.x == 0) {
        double scale = sqrt(a) + sqrt(b);
        out[0] = tol_n * tol_n * scale * scale;
        out[1] = scale;
        out[2] = c;
        out[3] = sqrt(a);
    }
}

// e_i += delta[head] - delta[tail] (wall nodes carry 0)
__global__ void k_gauss_apply(int32_t n, const int32_t *__restrict__ int_edges,
                              const int32_t *__restrict__ edge_nodes, const int32_t *__restrict__ int_node_of,
                              const double *__restrict__ delta, double *__restrict__ e) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t ge = int_edges[i];
    int32_t a = int_node_of[edge_nodes[2 * ge]], b = int_node_of[edge_nodes[2 * ge + 1]];
    double d = (b >= 0 ? delta[b] : 0.0) - (a >= 0 ? delta[a] : 0.0);
    e[i] += d;
}

// u = round((dt/2)(e_new + e_old)/u_b) per interior edge; e (global) <- e_new
__global__ void k_faraday_u(int32_t n, const int32_t *__restrict__ int_edges, const double *__restrict__ enew,
                            const double *__restrict__ eold, double half_dt_over_ub, int64_t *__restrict__ u,
                            double *__restrict__ eglob) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t ge = int_edges[i];
    u[ge] = (int64_t)llrint(half_dt_over_ub * (enew[i] + eold[i]));
    eglob[ge] = enew[i];
}

// b_f -= u_bc - u_ac + u_ab
__global__ void k_faraday_b(int64_t nf, const int32_t *__restrict__ fe, const int64_t *__restrict__ u,
                            int64_t *__restrict__ b) {
    int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    b[f] -= u[fe[3 * f + 2]] - u[fe[3 * f + 1]] + u[fe[3 * f]];
}

// ||b - A x||^2 and ||b||^2 (partials)
__global__ void __launch_bounds__(kThreads) k_true_res(const int2 *__restrict__ tiles, int32_t ntiles,
                                                       const int32_t *__restrict__ ptr,
                                                       const TileCols cols,
                                                       const double *__restrict__ val,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ b, double *__restrict__ part) {
    __shared__ double prod[kTileCap];
    double acc[2] = {0.0, 0.0};
    tile_spmv(tiles, ntiles, ptr, cols, val, x, prod, [&](int32_t row) { return b[row]; },
              [&](int32_t row, double s, double bb) {
        const double r = bb - s;
        acc[0] += r * r;
        acc[1] += bb * bb;
    });
    write_partials<2>(acc, part);
}

__global__ void __launch_bounds__(kThreads) k_sum2(const double *__restrict__ part, int m, double *out) {
    __shared__ double sh[kThreads / 64];
    double a = sum_partials(part, m, sh);
    double b = sum_partials(part + kMaxBlocks, m, sh);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// Right-hand side of the wave-equation update (eq. wave_cont, Newmark beta = 1/4, gamma = 1/2)
// on the interior edges:
//   rhs = 2 ([*eps] - tau S) e^n - ([*eps] + tau S) e^{n-1} - u_q (g^{n+1/2} - g^{n-1/2}),
// the two products over the pattern of A in one kernel (the same thread owns the same row in
// both passes, so the second adds to what the first wrote).
__global__ void __launch_bounds__(kThreads) k_wave_rhs(const int2 *__restrict__ tiles, int32_t ntiles,
                                                       const int32_t *__restrict__ ptr, const TileCols cols,
                                                       const double *__restrict__ arhs,
                                                       const double *__restrict__ aval,
                                                       const double *__restrict__ e,
                                                       const double *__restrict__ e_prev,
                                                       const int64_t *__restrict__ g,
                                                       const int64_t *__restrict__ g_prev,
                                                       const int32_t *__restrict__ int_edges, double u_q,
                                                       double *__restrict__ rhs) {
    __shared__ double prod[kTileCap];
    tile_spmv(tiles, ntiles, ptr, cols, arhs, e, prod,
              [&](int32_t row) {
                  const int32_t ge = int_edges[row];
                  return (double)(g[ge] - g_prev[ge]);
              },
              [&](int32_t row, double s, double dg) { rhs[row] = 2.0 * s - u_q * dg; });
    tile_spmv(tiles, ntiles, ptr, cols, aval, e_prev, prod, [&](int32_t) { return 0; },
              [&](int32_t row, double s, int) { rhs[row] -= s; });
}

// Plane wave through the natural boundary. s'(tau) of the modulated Gaussian s(u) =
// exp(-(u - t0)^2 / (2 sig^2)) cos(2 pi f0 (u - t0)).
__device__ __forceinline__ double pw_ds(double tau, double f0, double sig, double t0) {
    const double u = tau - t0, om = 2.0 * M_PI * f0;
    const double env = exp(-u * u / (2.0 * sig * sig));
    return env * (-(u / (sig * sig)) * cos(om * u) - om * sin(om * u));
}

// s'(t - x/c) at the step's three times for each distinct x of the rule points.
__global__ void k_pw_table(int32_t nu, const double *__restrict__ xs, double f0, double sig, double t0, double c0,
                           double t_prev, double t_n, double t_next, double *__restrict__ tab) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nu) return;
    const double ret = xs[i] / c0;
    tab[3 * i] = pw_ds(t_prev - ret, f0, sig, t0);
    tab[3 * i + 1] = pw_ds(t_n - ret, f0, sig, t0);
    tab[3 * i + 2] = pw_ds(t_next - ret, f0, sig, t0);
}

// Boundary term h_i(t) = sum over the edge's rule points of coef * (E0/eta) s'(t - x/c), at the
// step's times (s' from the table); adds the update's share to the right-hand side
// (trapezoidal: dt/2 (h^n + h^{n+1}); wave equation: dt/2 (h^{n+1} - h^{n-1})) and keeps
// dt/2 (h^n + h^{n+1}) for the Gauss-law target.
__global__ void k_plane_wave(int32_t nb, const int32_t *__restrict__ ptr, const int32_t *__restrict__ edge,
                             const double *__restrict__ coef, const int32_t *__restrict__ xi,
                             const double *__restrict__ tab, double amp, double half_dt, int wave,
                             double *__restrict__ rhs, double *__restrict__ hsum) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    double hp = 0.0, hn = 0.0, hx = 0.0;
    for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const double w = coef[k];
        const double *s = tab + 3 * xi[k];
        hn += w * s[1];
        hx += w * s[2];
        if (wave) hp += w * s[0];
    }
    const double hs = half_dt * amp * (hn + hx);
    hsum[i] = hs;
    rhs[edge[i]] += wave ? half_dt * amp * (hx - hp) : hs;
}

// dbnd += G^T hsum on the boundary nodes (edge a -> b: +1 at b, -1 at a), one thread per node in
// a fixed order.
__global__ void k_boundary_flux(int32_t nn, const int32_t *__restrict__ nptr, const int32_t *__restrict__ nlist,
                                const int32_t *__restrict__ node, const double *__restrict__ hsum,
                                double *__restrict__ dbnd) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    double s = 0.0;
    for (int32_t k = nptr[i]; k < nptr[i + 1]; ++k) {
        const int32_t v = nlist[k];
        s += (v & 1) ? -hsum[v >> 1] : hsum[v >> 1];
    }
    dbnd[node[i]] += s;
}

}  // namespace

int qh_cg_alloc(qh_ctx *c, CgWork &w, int32_t n) {
    w.n = n;
    int rc;
    if ((rc = qh_alloc(c, &w.x, n)) || (rc = qh_alloc(c, &w.r, n)) || (rc = qh_alloc(c, &w.z, n)) ||
        (rc = qh_alloc(c, &w.q, n)) || (rc = qh_alloc(c, &w.p0, n)) || (rc = qh_alloc(c, &w.p1, n)) ||
        (rc = qh_alloc(c, &w.dinv, n)) || (rc = qh_alloc(c, &w.b, n)) ||
        (rc = qh_alloc(c, &w.partial, 8 * kMaxBlocks)) || (rc = qh_alloc(c, &w.scal, S_NSCAL)) ||
        (rc = qh_alloc(c, &w.counter, 4)) || (rc = qh_alloc(c, &w.flags, 4)))
        return rc;
    QH_HIP(c, hipMemsetAsync(w.counter, 0, 4 * sizeof(unsigned int), c->stream));
    QH_HIP(c, hipMemsetAsync(w.x, 0, n * sizeof(double), c->stream));
    QH_HIP(c, hipMemsetAsync(w.scal, 0, S_NSCAL * sizeof(double), c->stream));
    return QH_OK;
}

hipError_t launch_diag_inv(qh_ctx *c, const DevCsr &M, double *dinv) {
    hipLaunchKernelGGL(k_diag_inv, dim3((M.n + 255) / 256), dim3(256), 0, c->stream, M.n, M.ptr, M.col, M.val, dinv);
    return hipGetLastError();
}

int qh_cg_solve(qh_ctx *c, const DevCsr &M, CgWork &w, double tol, int max_it, int check_every,
                SolveResult &out, const double *abs_thr2_dev, bool node_system, bool learned) {
    const int k_spmv = node_system ? QK_NODE_SPMV : QK_CG_SPMV;
    const int k_upd = node_system ? QK_NODE_UPDATE : QK_CG_UPDATE;
    out = SolveResult();
    if (w.n == 0) {
        out.converged = true;
        out.flag = CG_CONVERGED;
        return QH_OK;
    }
    // partials: [0, 4K) init / update (slot 0 r.z with Jacobi, 1 r.r, 2 b.b), [4K, 5K) products,
    // [5K, 6K) r.z of the learned preconditioner
    double *upart = w.partial, *qpart = w.partial + 4 * kMaxBlocks, *ppart = w.partial + 5 * kMaxBlocks;
    const unsigned ge = grid_elems(w.n), gt = tile_grid(M.ntiles);
    const unsigned gp = learned ? qh_prec_grid(c) : 0;
    const int stall = learned ? 1 : 0;
    if (check_every <= 0) check_every = 8;
    // iterations after convergence return at once on the device; sizing the first batch from
    // the previous solve avoids most of them and most host reads of the flag
    int first = w.last_iters[learned ? 1 : 0];
    if (first > 0) ++first;  // one idle launch when the count repeats, no second batch when it grows by one
    int it = 0;
    // Recurrence residuals drift from the true one; a solve whose recurrence converged but whose
    // recomputed residual misses the target restarts from its iterate (at most kRestarts times)
    constexpr int kRestarts = 2;
    for (int restart = 0;; ++restart) {
        int t0 = qh_tbeg(c);
        hipLaunchKernelGGL(k_cg_init, dim3(gt), dim3(kThreads), 0, c->stream, M.tiles, M.ntiles, M.ptr, M.cols(), M.val,
                           w.x, w.b, w.dinv, w.r, w.z, w.p0, upart);
        if (learned) QH_HIP(c, launch_prec_apply(c, w.r, w.z, ppart, nullptr));
        hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kThreads), 0, c->stream, upart, (int)gt,
                           learned ? (const double *)ppart : (const double *)upart, learned ? (int)gp : (int)gt,
                           w.scal, w.flags, tol * tol, abs_thr2_dev, stall);
        qh_tend(c, t0, QK_CG_INIT);
        QH_HIP(c, hipGetLastError());
        // the start's verdict is read on the host only when the last solve needed no iteration
        // (or there was none); otherwise the first batch is launched at once, and its launches
        // return at once if the start already stopped the iteration
        int32_t hflags[2] = {0, 0};
        int m_up = (int)gt;
        if (!(first > 0 && restart == 0)) {
            QH_HIP(c, hipMemcpyAsync(hflags, w.flags, sizeof(hflags), hipMemcpyDeviceToHost, c->stream));
            QH_HIP(c, hipStreamSynchronize(c->stream));
        }
        const int it0 = it;  // the device counts this run's iterations from 0
        while (it < max_it && !hflags[0]) {
            int batch = std::min(it == it0 && first > 0 && restart == 0 ? first : check_every, max_it - it);
            for (int k = it - it0; k < it - it0 + batch; ++k) {
                int par = k & 1;
                int ta = qh_tbeg(c);
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_spmv<double, double>), dim3(gt), dim3(kThreads), 0, c->stream, w.n, M.tiles, M.ntiles, M.ptr,
                                   M.cols(), M.val, w.z, w.p0, w.q, learned ? (const double *)ppart : (const double *)upart,
                                   learned ? (int)gp : m_up, upart + kMaxBlocks, m_up, qpart, w.scal, w.flags, k, par,
                                   stall);
                qh_tend(c, ta, k_spmv);
                int tb = qh_tbeg(c);
                if (learned)
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_update<false, double>), dim3(ge), dim3(kThreads), 0, c->stream, w.n, w.x, w.r, w.z,
                                       w.p0, w.q, w.dinv, qpart, upart, (int)gt, w.scal, w.flags, par);
                else
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_update<true, double>), dim3(ge), dim3(kThreads), 0, c->stream, w.n, w.x, w.r, w.z,
                                       w.p0, w.q, w.dinv, qpart, upart, (int)gt, w.scal, w.flags, par);
                qh_tend(c, tb, k_upd);
                m_up = (int)ge;
                if (learned) {
                    int tp = qh_tbeg(c);
                    QH_HIP(c, launch_prec_apply(c, w.r, w.z, ppart, w.flags));
                    qh_tend(c, tp, QK_PREC);
                }
            }
            it += batch;
            hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(kThreads), 0, c->stream, upart, m_up, w.scal, w.flags,
                               it - it0);
            QH_HIP(c, hipGetLastError());
            QH_HIP(c, hipMemcpyAsync(hflags, w.flags, sizeof(hflags), hipMemcpyDeviceToHost, c->stream));
            QH_HIP(c, hipStreamSynchronize(c->stream));
        }
        it = it0 + hflags[1];
        out.iters = it;
        out.flag = hflags[0];
        // true residual, recomputed with a fresh FP64 product, against the same target
        int tr = qh_tbeg(c);
        hipLaunchKernelGGL(k_true_res, dim3(gt), dim3(kThreads), 0, c->stream, M.tiles, M.ntiles, M.ptr, M.cols(), M.val,
                           w.x, w.b, upart);
        hipLaunchKernelGGL(k_sum2, dim3(1), dim3(kThreads), 0, c->stream, upart, (int)gt, w.scal + S_RES);
        qh_tend(c, tr, QK_TRUE_RES);
        double sc[S_RES + 2];
        QH_HIP(c, hipMemcpyAsync(sc, w.scal, sizeof(sc), hipMemcpyDeviceToHost, c->stream));
        QH_HIP(c, hipStreamSynchronize(c->stream));
        const double res2 = sc[S_RES], bb2 = sc[S_RES + 1], thr2 = sc[S_THR2];
        out.res = bb2 > 0 ? sqrt(res2 / bb2) : 0.0;
        out.true_ok = res2 == res2 && res2 <= thr2;
        out.converged = out.flag == CG_CONVERGED && out.true_ok;
        if (out.converged || out.flag != CG_CONVERGED || it >= max_it || restart == kRestarts) break;
        out.restarts = restart + 1;
    }
    if (out.converged) w.last_iters[learned ? 1 : 0] = out.iters;
    return QH_OK;
}

// Mixed-precision solve: PCG in FP32 (the FP32 copy of A's values, FP32 vectors, FP64 products
// and dot products, the same preconditioner) on A d = r0 / s from the FP64 residual r0 = b - A x0,
// s = ||r0||, with reliable updates: at the end of each batch of iterations x += s d in FP64,
// r = b - A x is recomputed in FP64 (the convergence test: ||r|| <= tol ||b||, the FP64 solve's
// stopping rule) and, unless it is met, replaces the recurrence's residual, which then continues
// without a restart (its Krylov space and convergence rate are kept). A segment between updates
// may reduce the residual by about 1e-4 at most (the FP32 correction d holds the FP64 solution's
// change only to FP32 accuracy): its length comes from the last solve's rate of convergence, and
// the last batch ends at the last solve's iteration count (from the second segment on, taking in
// a remainder of at most an eighth of a segment), where the FP64 residual usually meets the
// target already (the recurrence aims a little lower), so a step of the benchmark takes two
// reliable updates. Without a history, batches of check_every iterations. A batch that meets non-finite values is not
// applied (flag 3); one stopped by the stall rule is applied and the solve returns (flag 2).
int qh_cg_alloc32(qh_ctx *c, CgWork &w, int32_t n) {
    if (w.n32 >= n) return QH_OK;
    int rc;
    if ((rc = qh_alloc(c, &w.x32, n)) || (rc = qh_alloc(c, &w.r32, n)) || (rc = qh_alloc(c, &w.z32, n)) ||
        (rc = qh_alloc(c, &w.p32, n)) || (rc = qh_alloc(c, &w.q32, n)) || (rc = qh_alloc(c, &w.dinv32, n)))
        return rc;
    w.n32 = n;
    return QH_OK;
}

int qh_cg_solve_mixed(qh_ctx *c, DevCsr &M, CgWork &w, double tol, int max_it, int check_every,
                      SolveResult &out, bool learned) {
    out = SolveResult();
    const int32_t n = w.n;
    if (n == 0) {
        out.converged = out.true_ok = true;
        out.flag = CG_CONVERGED;
        return QH_OK;
    }
    int rc;
    if ((rc = qh_cg_alloc32(c, w, n))) return rc;
    // FP32 copies: the matrix values once per time step size, the inverse diagonal every solve
    // (a work area may serve several systems)
    if (!M.val32 || M.val32_tau != c->tau_assembled) {
        if (!M.val32 && (rc = qh_alloc(c, &M.val32, (size_t)M.nnz))) return rc;
        const unsigned gc = (unsigned)std::min<int64_t>((M.nnz + 255) / 256, 8192);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_convert<double, float>), dim3(gc), dim3(256), 0, c->stream, M.nnz, M.val,
                           M.val32);
        M.val32_tau = c->tau_assembled;
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_convert<double, float>), dim3(grid_elems(n)), dim3(256), 0, c->stream,
                       (int64_t)n, (const double *)w.dinv, w.dinv32);
    QH_HIP(c, hipGetLastError());
    double *upart = w.partial, *qpart = w.partial + 4 * kMaxBlocks, *ppart = w.partial + 5 * kMaxBlocks;
    const unsigned ge = grid_elems(n), gt = tile_grid(M.ntiles);
    const unsigned gp = learned ? qh_prec_grid(c) : 0;
    const int stall = learned ? 1 : 0;
    if (check_every <= 0) check_every = 8;
    // r = b - A x in FP64 with ||r||^2 and ||b||^2 on the host
    double sc[2] = {0.0, 0.0};
    auto fp64_residual = [&]() -> int {
        int tr = qh_tbeg(c);
        hipLaunchKernelGGL(k_res_store, dim3(gt), dim3(kThreads), 0, c->stream, M.tiles, M.ntiles, M.ptr, M.cols(), M.val,
                           w.x, w.b, w.r, upart);
        hipLaunchKernelGGL(k_sum2, dim3(1), dim3(kThreads), 0, c->stream, upart, (int)gt, w.scal + S_RES);
        qh_tend(c, tr, QK_TRUE_RES);
        QH_HIP(c, hipGetLastError());
        QH_HIP(c, hipMemcpyAsync(sc, w.scal + S_RES, sizeof(sc), hipMemcpyDeviceToHost, c->stream));
        QH_HIP(c, hipStreamSynchronize(c->stream));
        return QH_OK;
    };
    if ((rc = fp64_residual())) return rc;
    const double rr0 = sc[0], bb = sc[1], thr2 = tol * tol * bb;
    out.res = bb > 0 ? sqrt(rr0 / bb) : 0.0;
    if (!(rr0 == rr0) || rr0 > 1.7976931348623157e308) {
        out.flag = CG_NONFINITE;
        return QH_OK;
    }
    if (rr0 <= thr2) {
        out.converged = out.true_ok = true;
        out.flag = CG_CONVERGED;
        return QH_OK;
    }
    // start of the FP32 recurrence; its target on the scaled residual: (0.9 tol ||b|| / s)^2, a
    // little below the FP64 target, which the reliable update then usually confirms at once
    int t0 = qh_tbeg(c);
    if (learned) {
        hipLaunchKernelGGL(k_inner_init<false>, dim3(ge), dim3(kThreads), 0, c->stream, n, w.r, w.scal + S_RES, w.scal,
                           w.r32, w.x32, w.z32, w.p32, w.dinv32, upart);
        QH_HIP(c, launch_prec_apply32(c, w.r32, w.z32, ppart, nullptr));
    } else {
        hipLaunchKernelGGL(k_inner_init<true>, dim3(ge), dim3(kThreads), 0, c->stream, n, w.r, w.scal + S_RES, w.scal,
                           w.r32, w.x32, w.z32, w.p32, w.dinv32, upart);
    }
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kThreads), 0, c->stream, upart, (int)ge,
                       learned ? (const double *)ppart : (const double *)upart, learned ? (int)gp : (int)ge,
                       w.scal, w.flags, 0.81 * thr2 / rr0, (const double *)nullptr, stall);
    qh_tend(c, t0, QK_CG_INIT);
    QH_HIP(c, hipGetLastError());
    const int prev = w.last_mixed[learned ? 1 : 0];     // iterations of the last converged solve
    const int seg = w.last_segment[learned ? 1 : 0];    // its iterations per 1e-4 of reduction
    int k = 0, flag = CG_RUNNING;
    for (int update = 0;; ++update) {
        // a batch: to the next segment end, at most to the last solve's iteration count (from
        // the second segment on, a last remainder of at most an eighth of a segment joins the
        // one before it), then check_every at a time
        int target = 0;
        if (prev > 0 && seg > 0) {
            target = std::min((update + 1) * seg, prev);
            if (update > 0 && prev - target <= seg / 8) target = prev;
        }
        const int batch = std::min(target > k ? target - k : check_every, max_it - k);
        int32_t hflags[2] = {0, 0};
        if (batch > 0) {
            for (int kk = k; kk < k + batch; ++kk) {
                const int par = kk & 1;
                int ta = qh_tbeg(c);
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_spmv<float, float>), dim3(gt), dim3(kThreads), 0, c->stream, n,
                                   M.tiles, M.ntiles, M.ptr, M.cols(), (const float *)M.val32, (const float *)w.z32,
                                   w.p32, w.q32, learned ? (const double *)ppart : (const double *)upart,
                                   learned ? (int)gp : (int)ge, upart + kMaxBlocks, (int)ge, qpart, w.scal, w.flags,
                                   kk, par, stall);
                qh_tend(c, ta, QK_CG_SPMV);
                int tb = qh_tbeg(c);
                if (learned)
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_update<false, float>), dim3(ge), dim3(kThreads), 0, c->stream, n,
                                       w.x32, w.r32, w.z32, (const float *)w.p32, (const float *)w.q32,
                                       (const float *)w.dinv32, qpart, upart, (int)gt, w.scal, w.flags, par);
                else
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_update<true, float>), dim3(ge), dim3(kThreads), 0, c->stream, n,
                                       w.x32, w.r32, w.z32, (const float *)w.p32, (const float *)w.q32,
                                       (const float *)w.dinv32, qpart, upart, (int)gt, w.scal, w.flags, par);
                qh_tend(c, tb, QK_CG_UPDATE);
                if (learned) {
                    int tp = qh_tbeg(c);
                    QH_HIP(c, launch_prec_apply32(c, w.r32, w.z32, ppart, w.flags));
                    qh_tend(c, tp, QK_PREC);
                }
            }
            hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(kThreads), 0, c->stream, upart, (int)ge, w.scal, w.flags,
                               k + batch);
            QH_HIP(c, hipGetLastError());
            QH_HIP(c, hipMemcpyAsync(hflags, w.flags, sizeof(hflags), hipMemcpyDeviceToHost, c->stream));
            QH_HIP(c, hipStreamSynchronize(c->stream));
            k = hflags[0] ? hflags[1] : k + batch;
        }
        if (hflags[0] == CG_NONFINITE) {
            flag = CG_NONFINITE;  // the batch is not applied: x keeps the last reliable update
            break;
        }
        // reliable update: x += s d, r = b - A x in FP64
        int tf = qh_tbeg(c);
        hipLaunchKernelGGL(k_refine, dim3(ge), dim3(kThreads), 0, c->stream, n, w.x, w.x32, (const double *)w.scal);
        qh_tend(c, tf, QK_TRUE_RES);
        QH_HIP(c, hipGetLastError());
        if ((rc = fp64_residual())) return rc;
        out.refinements = update + 1;
        const double rr = sc[0];
        out.res = bb > 0 ? sqrt(rr / bb) : 0.0;
        if (rr == rr && rr <= thr2) {
            flag = CG_CONVERGED;
            break;
        }
        if (!(rr == rr) || rr > 1.7976931348623157e308) {
            flag = CG_NONFINITE;
            break;
        }
        if (hflags[0] == CG_STALLED) {
            flag = CG_STALLED;
            break;
        }
        if (k >= max_it) break;
        // the recurrence continues from the FP64 residual
        int tq = qh_tbeg(c);
        if (learned) {
            hipLaunchKernelGGL(k_replace<false>, dim3(ge), dim3(kThreads), 0, c->stream, n, (const double *)w.r, w.scal,
                               w.r32, w.z32, (const float *)w.dinv32, upart, w.flags);
            QH_HIP(c, launch_prec_apply32(c, w.r32, w.z32, ppart, nullptr));
        } else {
            hipLaunchKernelGGL(k_replace<true>, dim3(ge), dim3(kThreads), 0, c->stream, n, (const double *)w.r, w.scal,
                               w.r32, w.z32, (const float *)w.dinv32, upart, w.flags);
        }
        qh_tend(c, tq, QK_CG_INIT);
        QH_HIP(c, hipGetLastError());
    }
    out.iters = k;
    out.flag = flag;
    out.converged = out.true_ok = flag == CG_CONVERGED;
    if (out.converged) {
        w.last_mixed[learned ? 1 : 0] = k;
        // iterations per 1e-4 of residual reduction (1e-8 of r.r), at least check_every
        const double drop = sc[0] > 0 && k > 0 ? std::log(sc[0] / rr0) / k : 0.0;
        w.last_segment[learned ? 1 : 0] =
            drop < 0 ? (int)std::max<double>(check_every, std::min(1e6, std::ceil(std::log(1e-8) / drop))) : 0;
    }
    return QH_OK;
}

bool qh_make_tiles(const int32_t *ptr, int32_t n, std::vector<int2> &tiles) {
    tiles.clear();
    int32_t r = 0;
    tiles.push_back(make_int2(0, ptr[0]));
    while (r < n) {
        int32_t e = r;
        while (e < n && e - r < kTileRows && ptr[e + 1] - ptr[r] <= kTileCap) ++e;
        if (e == r) return false;
        tiles.push_back(make_int2(e, ptr[e]));
        r = e;
    }
    return true;
}

int64_t qh_compact_cols(const int32_t *col, const std::vector<int2> &tiles, std::vector<int4> &tbase,
                        std::vector<uint16_t> &col16) {
    constexpr int32_t kSpan = 1 << 14;
    const size_t nt = tiles.size() - 1;
    tbase.assign(nt, make_int4(-1, 0, 0, 0));
    col16.assign((size_t)tiles[nt].y, 0);
    int64_t n16 = 0;
    std::vector<int32_t> cs;
    for (size_t k = 0; k < nt; ++k) {
        const int32_t e0 = tiles[k].y, e1 = tiles[k + 1].y;
        if (e1 <= e0) continue;
        cs.assign(col + e0, col + e1);
        std::sort(cs.begin(), cs.end());
        int32_t w[4];
        int nw = 0;
        bool fits = true;
        for (int32_t v : cs) {
            if (nw > 0 && v < w[nw - 1] + kSpan) continue;
            if (nw == 4) {
                fits = false;
                break;
            }
            w[nw++] = v;
        }
        if (!fits) continue;
        for (int i = nw; i < 4; ++i) w[i] = w[nw - 1];
        tbase[k] = make_int4(w[0], w[1], w[2], w[3]);
        for (int32_t e = e0; e < e1; ++e) {
            int i = nw - 1;
            while (col[e] < w[i]) --i;  // the last window starting at or below the column
            col16[e] = (uint16_t)((uint32_t)i << 14 | (uint32_t)(col[e] - w[i]));
        }
        n16 += e1 - e0;
    }
    return n16;
}

hipError_t launch_assemble_A(qh_ctx *c, double tau) {
    int64_t nnz = c->A.nnz;
    hipLaunchKernelGGL(k_axpy_vals, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, c->stream, nnz, c->A.val2,
                       c->A_S, tau, c->A.val, c->A_rhs);
    return hipGetLastError();
}

hipError_t launch_edge_rhs(qh_ctx *c) {
    hipLaunchKernelGGL(k_edge_rhs_e, dim3(tile_grid(c->A.ntiles)), dim3(kThreads), 0, c->stream, c->A.tiles,
                       c->A.ntiles, c->A.ptr, c->A.cols(), c->A_rhs, c->cge.x, c->g, c->int_edges, c->phys.u_q,
                       c->cge.b);
    hipLaunchKernelGGL(k_edge_rhs_b, dim3(tile_grid(c->CMb.ntiles)), dim3(kThreads), 0, c->stream, c->CMb.tiles,
                       c->CMb.ntiles, c->CMb.ptr, c->CMb.cols(), c->CMb.val, c->b, c->phys.dt * c->phys.u_b, c->cge.b);
    return hipGetLastError();
}

hipError_t launch_wave_rhs(qh_ctx *c) {
    hipLaunchKernelGGL(k_wave_rhs, dim3(tile_grid(c->A.ntiles)), dim3(kThreads), 0, c->stream, c->A.tiles,
                       c->A.ntiles, c->A.ptr, c->A.cols(), c->A_rhs, c->A.val, c->cge.x, c->e_prev, c->g, c->g_prev,
                       c->int_edges, c->phys.u_q, c->cge.b);
    return hipGetLastError();
}

hipError_t launch_plane_wave(qh_ctx *c, bool wave) {
    const double dt = c->phys.dt, tn = (double)c->step_index * dt;
    hipLaunchKernelGGL(k_pw_table, dim3((c->pw_nu + 255) / 256), dim3(256), 0, c->stream, c->pw_nu, c->pw_xs, c->pw_f0,
                       c->pw_sig, c->pw_t0, c->pw_c, tn - dt, tn, tn + dt, c->pw_tab);
    hipLaunchKernelGGL(k_plane_wave, dim3((c->pw_nb + 255) / 256), dim3(256), 0, c->stream, c->pw_nb, c->pw_ptr,
                       c->pw_edge, c->pw_coef, c->pw_xi, c->pw_tab, c->pw_amp, 0.5 * dt, wave ? 1 : 0, c->cge.b,
                       c->pw_hsum);
    hipLaunchKernelGGL(k_boundary_flux, dim3((c->pw_nn + 255) / 256), dim3(256), 0, c->stream, c->pw_nn, c->pw_nptr,
                       c->pw_nlist, c->pw_node, c->pw_hsum, c->dbnd);
    return hipGetLastError();
}

hipError_t launch_gauss_rhs(qh_ctx *c, double *out3, double tol_n) {
    int32_t n = c->GtM.n;
    unsigned gr = grid_rows(n);
    hipLaunchKernelGGL(k_gauss_rhs, dim3(gr), dim3(kThreads), 0, c->stream, n, c->GtM.ptr, c->GtM.col,
                       c->GtM.val, c->cge.x, c->Q_bg, c->Q, c->int_nodes, c->phys.u_q,
                       (const double *)c->dbnd, c->cgn.b, c->rho, c->cgn.partial);
    hipLaunchKernelGGL(k_gauss_finish, dim3(1), dim3(kThreads), 0, c->stream, c->cgn.partial, (int)gr, out3, tol_n);
    return hipGetLastError();
}

// Quasi-Helmholtz split: cgn.b = -G^T [*eps] e (the Gauss-law right-hand side with no charge
// and no boundary flux), with the node solve's threshold in out3 as for the correction.
hipError_t launch_div_e(qh_ctx *c, double *out3, double tol_n) {
    int32_t n = c->GtM.n;
    unsigned gr = grid_rows(n);
    hipLaunchKernelGGL(k_gauss_rhs, dim3(gr), dim3(kThreads), 0, c->stream, n, c->GtM.ptr, c->GtM.col, c->GtM.val,
                       c->cge.x, (const int64_t *)c->Q, (const int64_t *)c->Q, c->int_nodes, 0.0, (const double *)nullptr,
                       c->cgn.b, (double *)nullptr, c->cgn.partial);
    hipLaunchKernelGGL(k_gauss_finish, dim3(1), dim3(kThreads), 0, c->stream, c->cgn.partial, (int)gr, out3, tol_n);
    return hipGetLastError();
}

// e_int += G delta (interior edge values; delta on the unknown nodes)
hipError_t launch_grad_add(qh_ctx *c, const double *delta, double *e_int) {
    int32_t n = c->A.n;
    hipLaunchKernelGGL(k_gauss_apply, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->int_edges, c->edge_nodes,
                       c->int_node_of, delta, e_int);
    return hipGetLastError();
}

hipError_t launch_gauss_apply(qh_ctx *c) {
    int32_t n = c->A.n;
    hipLaunchKernelGGL(k_gauss_apply, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->int_edges, c->edge_nodes,
                       c->int_node_of, c->cgn.x, c->cge.x);
    return hipGetLastError();
}

hipError_t launch_faraday(qh_ctx *c) {
    int32_t n = c->A.n;
    hipLaunchKernelGGL(k_faraday_u, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->int_edges, c->cge.x,
                       c->e_old, 0.5 * c->phys.dt / c->phys.u_b, c->u_int, c->e);
    int64_t nf = c->hm.Nf;
    hipLaunchKernelGGL(k_faraday_b, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, c->stream, nf, c->face_edges,
                       c->u_int, c->b);
    return hipGetLastError();
}

hipError_t launch_true_residual(qh_ctx *c, const DevCsr &M, const double *x, const double *b, double *out2) {
    const unsigned gt = tile_grid(M.ntiles);
    hipLaunchKernelGGL(k_true_res, dim3(gt), dim3(kThreads), 0, c->stream, M.tiles, M.ntiles, M.ptr, M.cols(), M.val, x, b,
                       c->cge.partial);
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(kThreads), 0, c->stream, c->cge.partial, (int)gt, out2);
    return hipGetLastError();
}
