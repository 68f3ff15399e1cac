// Implicit field update on gfx950 (Sec. IV.B): FP64 CSR products, preconditioned conjugate
// gradients with FP64 dot products reduced in a fixed order (deterministic iteration counts),
// the Gauss-law solve for the non-solenoidal part and the integer Faraday update.
//
// Edge system (trapezoidal rule on eq. maxwell_semi, b^{n+1} eliminated):
//   ([*eps] + tau S) e* = ([*eps] - tau S) e^n + dt C^T [*mu^-1] b^n - u_q g,   tau = dt^2/4
// Gauss law (eq. discreteGauss): G^T [*eps] G delta = rho^{n+1} - G^T [*eps] e*, e = e* + G delta
// Faraday: b^{n+1} = b^n - C round((dt/2)(e^{n+1} + e^n)/u_b)  (D C = 0 keeps D b fixed).
#include "qh_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kLpr = 8;          // lanes per CSR row
constexpr int kMaxBlocks = 2048; // fixed grid of the reducing kernels (fixed summation order)

// device scalar slots of a CgWork
enum { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_THR2, S_BB, S_RZ0, S_NSLOT };

__device__ __forceinline__ double wave_sum_lpr(double v) {
#pragma unroll
    for (int off = kLpr / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kLpr);
    return v;
}

// Block-wide sum of NV doubles (thread 0 holds the result).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[kThreads / 64]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) s += sh[k][w];
            v[k] = s;
        }
    }
}

// Write NV block partials; the last block to finish sums all partials in a fixed order and
// returns true in every thread of that block (totals in tot[] of thread 0).
template <int NV>
__device__ bool last_block_reduce(double (&v)[NV], double *partial, unsigned int *counter,
                                  double (&tot)[NV]) {
    __shared__ double sh[NV][kThreads / 64];
    __shared__ bool am_last;
    block_sum<NV>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) partial[k * kMaxBlocks + blockIdx.x] = v[k];
        __threadfence();
        unsigned int prev = atomicAdd(counter, 1u);
        am_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!am_last) return false;
    __threadfence();
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        s[k] = 0.0;
        for (int j = threadIdx.x; j < (int)gridDim.x; j += kThreads) s[k] += partial[k * kMaxBlocks + j];
    }
    __syncthreads();
    block_sum<NV>(s, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] = s[k];
        *counter = 0u;
    }
    return true;
}

inline unsigned grid_rows(int64_t nrows) {
    int64_t b = (nrows * kLpr + kThreads - 1) / kThreads;
    return (unsigned)(b < kMaxBlocks ? (b < 1 ? 1 : b) : kMaxBlocks);
}
inline unsigned grid_elems(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b < kMaxBlocks ? (b < 1 ? 1 : b) : kMaxBlocks);
}

// ---------------------------------------------------------------------------------------
// CG kernels
// init: r = b - A x, z = D^-1 r, p_old = 0, beta = 0; rz, rr, bb; thr2 = tol^2 bb unless an
// absolute threshold is supplied.
__global__ void __launch_bounds__(kThreads) k_cg_init(int32_t n, const int32_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ b,
                                                      const double *__restrict__ dinv,
                                                      double *__restrict__ r, double *__restrict__ z,
                                                      double *__restrict__ p_old, double *partial,
                                                      unsigned int *counter, double *scal,
                                                      int32_t *flags, double tol2,
                                                      const double *abs_thr2) {
    const int sub = threadIdx.x % kLpr;
    const int64_t rows_per_grid = (int64_t)gridDim.x * (kThreads / kLpr);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t row = (int64_t)blockIdx.x * (kThreads / kLpr) + threadIdx.x / kLpr; row < n; row += rows_per_grid) {
        double s = 0.0;
        for (int32_t j = ptr[row] + sub; j < ptr[row + 1]; j += kLpr) s += val[j] * x[col[j]];
        s = wave_sum_lpr(s);
        if (sub == 0) {
            double rr = b[row] - s;
            double zz = rr * dinv[row];
            r[row] = rr;
            z[row] = zz;
            p_old[row] = 0.0;
            acc[0] += rr * zz;
            acc[1] += rr * rr;
            acc[2] += b[row] * b[row];
        }
    }
    double tot[3];
    if (last_block_reduce<3>(acc, partial, counter, tot) && threadIdx.x == 0) {
        scal[S_RZ] = tot[0];
        scal[S_RR] = tot[1];
        scal[S_BB] = tot[2];
        scal[S_RZ0] = tot[0];
        scal[S_BETA] = 0.0;
        double thr2 = abs_thr2 ? *abs_thr2 : tol2 * tot[2];
        scal[S_THR2] = thr2;
        flags[0] = (tot[1] <= thr2) ? 1 : 0;
        flags[1] = 0;
    }
}

// p_new = z + beta p_old (own rows); q = A p_new, gathered on the fly; pq.
__global__ void __launch_bounds__(kThreads) k_cg_spmv(int32_t n, const int32_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ val,
                                                      const double *__restrict__ z,
                                                      const double *__restrict__ p_old,
                                                      double *__restrict__ p_new, double *__restrict__ q,
                                                      double *partial, unsigned int *counter,
                                                      double *scal, const int32_t *flags) {
    if (flags[0]) return;
    const double beta = scal[S_BETA];
    const int sub = threadIdx.x % kLpr;
    const int64_t rows_per_grid = (int64_t)gridDim.x * (kThreads / kLpr);
    double acc[1] = {0.0};
    for (int64_t row = (int64_t)blockIdx.x * (kThreads / kLpr) + threadIdx.x / kLpr; row < n; row += rows_per_grid) {
        double s = 0.0;
        for (int32_t j = ptr[row] + sub; j < ptr[row + 1]; j += kLpr) {
            int32_t cj = col[j];
            s += val[j] * (z[cj] + beta * p_old[cj]);
        }
        s = wave_sum_lpr(s);
        if (sub == 0) {
            double pn = z[row] + beta * p_old[row];
            p_new[row] = pn;
            q[row] = s;
            acc[0] += pn * s;
        }
    }
    double tot[1];
    if (last_block_reduce<1>(acc, partial, counter, tot) && threadIdx.x == 0) {
        scal[S_PQ] = tot[0];
        scal[S_ALPHA] = scal[S_RZ] / tot[0];
    }
}

// x += alpha p; r -= alpha q; z = D^-1 r; rz, rr -> beta, convergence flag.
__global__ void __launch_bounds__(kThreads) k_cg_update(int32_t n, double *__restrict__ x,
                                                        double *__restrict__ r, double *__restrict__ z,
                                                        const double *__restrict__ p,
                                                        const double *__restrict__ q,
                                                        const double *__restrict__ dinv,
                                                        double *partial, unsigned int *counter,
                                                        double *scal, int32_t *flags) {
    if (flags[0]) return;
    const double alpha = scal[S_ALPHA];
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        x[i] += alpha * p[i];
        double ri = r[i] - alpha * q[i];
        r[i] = ri;
        double zi = ri * dinv[i];
        z[i] = zi;
        acc[0] += ri * zi;
        acc[1] += ri * ri;
    }
    double tot[2];
    if (last_block_reduce<2>(acc, partial, counter, tot) && threadIdx.x == 0) {
        scal[S_BETA] = tot[0] / scal[S_RZ];
        scal[S_RZ] = tot[0];
        scal[S_RR] = tot[1];
        flags[1] += 1;
        if (tot[1] <= scal[S_THR2] || !(tot[1] == tot[1])) flags[0] = 1;
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

__global__ void k_axpy_vals(int64_t n, const double *__restrict__ a, const double *__restrict__ s, double tau,
                            double *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + tau * s[i];
}

// rhs_i = sum_j (2 Meps_ij - A_ij) e_j + dt u_b sum_f CMb_if b_f - u_q g[int_edge_i]
__global__ void __launch_bounds__(kThreads) k_edge_rhs(int32_t n, const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ aval,
                                                       const double *__restrict__ mval,
                                                       const double *__restrict__ e,
                                                       const int32_t *__restrict__ cptr,
                                                       const int32_t *__restrict__ ccol,
                                                       const double *__restrict__ cval,
                                                       const int64_t *__restrict__ b,
                                                       const int64_t *__restrict__ g,
                                                       const int32_t *__restrict__ int_edges, double dtub,
                                                       double u_q, double *__restrict__ rhs) {
    const int sub = threadIdx.x % kLpr;
    const int64_t row = (int64_t)blockIdx.x * (kThreads / kLpr) + threadIdx.x / kLpr;
    if (row >= n) return;
    double s = 0.0, t = 0.0;
    for (int32_t j = ptr[row] + sub; j < ptr[row + 1]; j += kLpr) s += (2.0 * mval[j] - aval[j]) * e[col[j]];
    for (int32_t j = cptr[row] + sub; j < cptr[row + 1]; j += kLpr) t += cval[j] * (double)b[ccol[j]];
    s = wave_sum_lpr(s);
    t = wave_sum_lpr(t);
    if (sub == 0) rhs[row] = s + dtub * t - u_q * (double)g[int_edges[row]];
}

// Gauss residual rg = rho - G^T [*eps] e on interior nodes, rho = u_q (Q_bg - Q);
// threshold thr2 = (tol_n (||rho|| + ||G^T [*eps] e||))^2.
__global__ void __launch_bounds__(kThreads) k_gauss_rhs(int32_t n, const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ e,
                                                        const int64_t *__restrict__ Qbg,
                                                        const int64_t *__restrict__ Q,
                                                        const int32_t *__restrict__ int_nodes, double u_q,
                                                        double *__restrict__ rg, double *__restrict__ rho_out,
                                                        double *partial, unsigned int *counter,
                                                        double *out, double tol_n) {
    const int sub = threadIdx.x % kLpr;
    const int64_t rows_per_grid = (int64_t)gridDim.x * (kThreads / kLpr);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t row = (int64_t)blockIdx.x * (kThreads / kLpr) + threadIdx.x / kLpr; row < n; row += rows_per_grid) {
        double s = 0.0;
        for (int32_t j = ptr[row] + sub; j < ptr[row + 1]; j += kLpr) s += val[j] * e[col[j]];
        s = wave_sum_lpr(s);
        if (sub == 0) {
            int32_t gn = int_nodes[row];
            double rho = u_q * (double)(Qbg[gn] - Q[gn]);
            double r = rho - s;
            rg[row] = r;
            if (rho_out) rho_out[row] = rho;
            acc[0] += rho * rho;
            acc[1] += s * s;
            acc[2] += r * r;
        }
    }
    double tot[3];
    if (last_block_reduce<3>(acc, partial, counter, tot) && threadIdx.x == 0) {
        double scale = sqrt(tot[0]) + sqrt(tot[1]);
        out[0] = tol_n * tol_n * scale * scale;  // threshold on ||r||^2
        out[1] = scale;
        out[2] = tot[2];
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

// ||b - A x||^2 and ||b||^2
__global__ void __launch_bounds__(kThreads) k_true_res(int32_t n, const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ b, double *partial,
                                                       unsigned int *counter, double *out) {
    const int sub = threadIdx.x % kLpr;
    const int64_t rows_per_grid = (int64_t)gridDim.x * (kThreads / kLpr);
    double acc[2] = {0.0, 0.0};
    for (int64_t row = (int64_t)blockIdx.x * (kThreads / kLpr) + threadIdx.x / kLpr; row < n; row += rows_per_grid) {
        double s = 0.0;
        for (int32_t j = ptr[row] + sub; j < ptr[row + 1]; j += kLpr) s += val[j] * x[col[j]];
        s = wave_sum_lpr(s);
        if (sub == 0) {
            double r = b[row] - s;
            acc[0] += r * r;
            acc[1] += b[row] * b[row];
        }
    }
    double tot[2];
    if (last_block_reduce<2>(acc, partial, counter, tot) && threadIdx.x == 0) {
        out[0] = tot[0];
        out[1] = tot[1];
    }
}

}  // namespace

int qh_cg_alloc(qh_ctx *c, CgWork &w, int32_t n) {
    w.n = n;
    int rc;
    if ((rc = qh_alloc(c, &w.x, n)) || (rc = qh_alloc(c, &w.r, n)) || (rc = qh_alloc(c, &w.z, n)) ||
        (rc = qh_alloc(c, &w.q, n)) || (rc = qh_alloc(c, &w.p0, n)) || (rc = qh_alloc(c, &w.p1, n)) ||
        (rc = qh_alloc(c, &w.dinv, n)) || (rc = qh_alloc(c, &w.b, n)) ||
        (rc = qh_alloc(c, &w.partial, 4 * kMaxBlocks)) || (rc = qh_alloc(c, &w.scal, 16)) ||
        (rc = qh_alloc(c, &w.counter, 4)) || (rc = qh_alloc(c, &w.flags, 4)))
        return rc;
    QH_HIP(c, hipMemsetAsync(w.counter, 0, 4 * sizeof(unsigned int), c->stream));
    QH_HIP(c, hipMemsetAsync(w.x, 0, n * sizeof(double), c->stream));
    QH_HIP(c, hipMemsetAsync(w.scal, 0, 16 * sizeof(double), c->stream));
    return QH_OK;
}

hipError_t launch_diag_inv(qh_ctx *c, const DevCsr &M, double *dinv) {
    hipLaunchKernelGGL(k_diag_inv, dim3((M.n + 255) / 256), dim3(256), 0, c->stream, M.n, M.ptr, M.col, M.val, dinv);
    return hipGetLastError();
}

int qh_cg_solve(qh_ctx *c, const DevCsr &M, CgWork &w, double tol, int max_it, int check_every,
                SolveResult &out, const double *abs_thr2_dev) {
    out = SolveResult();
    if (w.n == 0) {
        out.converged = true;
        return QH_OK;
    }
    const unsigned gr = grid_rows(w.n), ge = grid_elems(w.n);
    hipLaunchKernelGGL(k_cg_init, dim3(gr), dim3(kThreads), 0, c->stream, w.n, M.ptr, M.col, M.val, w.x, w.b, w.dinv,
                       w.r, w.z, w.p0, w.partial, w.counter, w.scal, w.flags, tol * tol, abs_thr2_dev);
    QH_HIP(c, hipGetLastError());
    if (check_every <= 0) check_every = 8;
    int32_t hflags[2] = {0, 0};
    int it = 0;
    double *pa = w.p0, *pb = w.p1;
    while (it < max_it) {
        int batch = std::min(check_every, max_it - it);
        for (int k = 0; k < batch; ++k) {
            int t0 = qh_tbeg(c);
            hipLaunchKernelGGL(k_cg_spmv, dim3(gr), dim3(kThreads), 0, c->stream, w.n, M.ptr, M.col, M.val, w.z, pa, pb,
                               w.q, w.partial, w.counter, w.scal, w.flags);
            qh_tend(c, t0, QK_CG_SPMV);
            int t1 = qh_tbeg(c);
            hipLaunchKernelGGL(k_cg_update, dim3(ge), dim3(kThreads), 0, c->stream, w.n, w.x, w.r, w.z, pb, w.q, w.dinv,
                               w.partial, w.counter, w.scal, w.flags);
            qh_tend(c, t1, QK_CG_UPDATE);
            std::swap(pa, pb);
        }
        it += batch;
        QH_HIP(c, hipGetLastError());
        QH_HIP(c, hipMemcpyAsync(hflags, w.flags, sizeof(hflags), hipMemcpyDeviceToHost, c->stream));
        QH_HIP(c, hipStreamSynchronize(c->stream));
        if (hflags[0]) break;
    }
    out.iters = hflags[1];
    // true residual, recomputed
    hipLaunchKernelGGL(k_true_res, dim3(gr), dim3(kThreads), 0, c->stream, w.n, M.ptr, M.col, M.val, w.x, w.b,
                       w.partial, w.counter, w.scal + 8);
    double res2[2];
    QH_HIP(c, hipMemcpyAsync(res2, w.scal + 8, sizeof(res2), hipMemcpyDeviceToHost, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    out.res = res2[1] > 0 ? sqrt(res2[0] / res2[1]) : 0.0;
    out.converged = hflags[0] != 0;
    return QH_OK;
}

hipError_t launch_assemble_A(qh_ctx *c, double tau) {
    int64_t nnz = c->A.nnz;
    hipLaunchKernelGGL(k_axpy_vals, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, c->stream, nnz, c->A.val2,
                       c->A_S, tau, c->A.val);
    return hipGetLastError();
}

hipError_t launch_edge_rhs(qh_ctx *c) {
    int32_t n = c->A.n;
    unsigned gr = (unsigned)(((int64_t)n * kLpr + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_edge_rhs, dim3(gr), dim3(kThreads), 0, c->stream, n, c->A.ptr, c->A.col, c->A.val, c->A.val2,
                       c->cge.x, c->CMb.ptr, c->CMb.col, c->CMb.val, c->b, c->g, c->int_edges,
                       c->phys.dt * c->phys.u_b, c->phys.u_q, c->cge.b);
    return hipGetLastError();
}

hipError_t launch_gauss_rhs(qh_ctx *c, double *out3, double tol_n) {
    int32_t n = c->GtM.n;
    hipLaunchKernelGGL(k_gauss_rhs, dim3(grid_rows(n)), dim3(kThreads), 0, c->stream, n, c->GtM.ptr, c->GtM.col,
                       c->GtM.val, c->cge.x, c->Q_bg, c->Q, c->int_nodes, c->phys.u_q, c->cgn.b, c->rho,
                       c->cgn.partial, c->cgn.counter, out3, tol_n);
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
    hipLaunchKernelGGL(k_true_res, dim3(grid_rows(M.n)), dim3(kThreads), 0, c->stream, M.n, M.ptr, M.col, M.val, x, b,
                       c->cge.partial, c->cge.counter, out2);
    return hipGetLastError();
}
