// Field energy of the discrete fields (Sec. VI.A.1: without sources the trapezoidal update keeps
// 1/2 e^T [*eps] e + 1/2 b^T [*mu^-1] b unchanged; Sec. IV.A for the Whitney forms).
//
// Electric part: 1/2 sum_i e_i ([*eps] e)_i over the edge unknowns, with [*eps] from the
// device system matrix. Magnetic part: the Whitney 2-form field of fluxes with D b = 0 is
// constant in each tet (a divergence-free member of the local space), so its energy is
// |B_T|^2 |T| / (2 mu0) exactly, with B_T from the four face fluxes and FP64 geometry.
// Both sums are taken in FP64 with a fixed reduction tree: the result does not depend on
// scheduling.
#include <algorithm>

#include "qh_internal.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double block_sum(double v, double *lds) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kThreads / 64; ++k) s += lds[k];
    return s;
}

// part[blockIdx.x] = sum over this block's rows i of x_i * sum_j eps_ij x_j
__global__ void __launch_bounds__(kThreads) k_energy_e(int32_t n, const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ eps,
                                                       const double *__restrict__ x, double *__restrict__ part) {
    __shared__ double lds[kThreads / 64];
    const int32_t i = blockIdx.x * kThreads + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        double s = 0.0;
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) s += eps[k] * x[col[k]];
        v = x[i] * s;
    }
    v = block_sum(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// part[blockIdx.x] = sum over this block's tets of |B_T|^2 |T|, B_T in teslas
__global__ void __launch_bounds__(kThreads) k_energy_b(int32_t nt, const int4 *__restrict__ tnodes,
                                                       const int32_t *__restrict__ tfaces,
                                                       const double *__restrict__ xyz,
                                                       const int64_t *__restrict__ b, double u_b,
                                                       double *__restrict__ part) {
    __shared__ double lds[kThreads / 64];
    const int32_t t = blockIdx.x * kThreads + threadIdx.x;
    double v = 0.0;
    if (t < nt) {
        const int4 tn = tnodes[t];
        const int vid[4] = {tn.x, tn.y, tn.z, tn.w};
        double p[4][3];
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 3; ++d) p[a][d] = xyz[3 * vid[a] + d];
        double e1[3], e2[3], e3[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = p[1][d] - p[0][d];
            e2[d] = p[2][d] - p[0][d];
            e3[d] = p[3][d] - p[0][d];
        }
        // grad lambda_1..3 are the rows of the inverse of [e1 e2 e3]^T: (e2 x e3, e3 x e1, e1 x e2) / det
        double g[4][3];
        g[1][0] = e2[1] * e3[2] - e2[2] * e3[1];
        g[1][1] = e2[2] * e3[0] - e2[0] * e3[2];
        g[1][2] = e2[0] * e3[1] - e2[1] * e3[0];
        g[2][0] = e3[1] * e1[2] - e3[2] * e1[1];
        g[2][1] = e3[2] * e1[0] - e3[0] * e1[2];
        g[2][2] = e3[0] * e1[1] - e3[1] * e1[0];
        g[3][0] = e1[1] * e2[2] - e1[2] * e2[1];
        g[3][1] = e1[2] * e2[0] - e1[0] * e2[2];
        g[3][2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double det = e1[0] * g[1][0] + e1[1] * g[1][1] + e1[2] * g[1][2];
        for (int a = 1; a < 4; ++a)
            for (int d = 0; d < 3; ++d) g[a][d] /= det;
        for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
        // local face k is opposite vertex k, vertices ascending; its 2-form's mean over the tet
        // is (g_b - g_a) x (g_c - g_a) / 2
        const int LF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
        double B[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 4; ++k) {
            const double f = (double)b[tfaces[4 * t + k]] * u_b;
            const double *ga = g[LF[k][0]], *gb = g[LF[k][1]], *gc = g[LF[k][2]];
            const double u[3] = {gb[0] - ga[0], gb[1] - ga[1], gb[2] - ga[2]};
            const double w[3] = {gc[0] - ga[0], gc[1] - ga[1], gc[2] - ga[2]};
            B[0] += 0.5 * f * (u[1] * w[2] - u[2] * w[1]);
            B[1] += 0.5 * f * (u[2] * w[0] - u[0] * w[2]);
            B[2] += 0.5 * f * (u[0] * w[1] - u[1] * w[0]);
        }
        v = (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]) * fabs(det) / 6.0;
    }
    v = block_sum(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// out[0] = 1/2 sum pe, out[1] = sum pb / (2 mu0): one block, fixed order
__global__ void __launch_bounds__(kThreads) k_energy_finish(const double *__restrict__ pe, int32_t me,
                                                            const double *__restrict__ pb, int32_t mb,
                                                            double inv_mu0, double *__restrict__ out) {
    __shared__ double lds[kThreads / 64];
    double s = 0.0;
    for (int32_t k = threadIdx.x; k < me; k += kThreads) s += pe[k];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[0] = 0.5 * s;
    __syncthreads();
    s = 0.0;
    for (int32_t k = threadIdx.x; k < mb; k += kThreads) s += pb[k];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[1] = 0.5 * inv_mu0 * s;
}

}  // namespace

int32_t qh_energy_parts(const qh_ctx *c) {
    const int32_t me = (c->A.n + kThreads - 1) / kThreads, mb = (int32_t)((c->hm.Nt + kThreads - 1) / kThreads);
    return std::max<int32_t>(me, 1) + std::max<int32_t>(mb, 1);
}

hipError_t launch_field_energy(qh_ctx *c, double *part, double *out) {
    const int32_t n = c->A.n, nt = (int32_t)c->hm.Nt;
    const int32_t me = std::max<int32_t>((n + kThreads - 1) / kThreads, 1);
    const int32_t mb = std::max<int32_t>((nt + kThreads - 1) / kThreads, 1);
    hipLaunchKernelGGL(k_energy_e, dim3(me), dim3(kThreads), 0, c->stream, n, c->A.ptr, c->A.col, c->A.val2,
                       c->cge.x, part);
    hipLaunchKernelGGL(k_energy_b, dim3(mb), dim3(kThreads), 0, c->stream, nt, c->tnodes, c->tfaces, c->xyz_d,
                       c->b, c->phys.u_b, part + me);
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(kThreads), 0, c->stream, part, me, part + me, mb,
                       1.0 / c->phys.mu0, out);
    return hipGetLastError();
}
