// Learned preconditioner for the edge system on gfx950.
//
// M = G^T G, G sparse lower triangular on the pattern of A = [*eps] + dt^2/4 S (interior
// edges). A network 16 -> 64 -> 64 -> 1 (ReLU) maps local features of each pattern entry
// (i, j), j <= i, to o_ij; G_ij = o_ij / sqrt(A_jj) (j < i), G_ii = softplus(o_ii + s0) /
// sqrt(A_ii) with softplus(s0) = 1, so a zero output gives Jacobi and M is SPD by
// construction (plain PCG applies). Training minimises the Kaporin number of G A G^T,
// L = log(tr(G A G^T)/n) - (2/n) sum log G_ii, trace from Rademacher probes.
//
// The dense layers run on MFMA with BF16 operands and FP32 accumulation, activations kept
// feature-major (entries along the 16 accumulator columns). The accumulator tile of one layer
// (lane l holds rows 4(l/16)+j of column l%16) feeds the next layer's B operand without a
// shuffle: the 16-feature input layer uses v_mfma_f32_16x16x16_bf16; the 64-wide contractions
// use v_mfma_f32_16x16x32_bf16 (lane l holds k = 8(l/16)+j), whose B operand is two
// accumulator tiles side by side, with the weight columns permuted to match. Weight gradients
// contract over entries (32 per step) through a small per-wave LDS transpose.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>

#include "qh_internal.h"
#include "qh_spmv.h"

namespace {

constexpr int kF = 16, kH = 64;
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248, kOffB3 = 5312;
constexpr float kS0 = 0.54132485461291810f;  // log(e - 1): softplus(kS0) = 1
constexpr int kWaves = 4;                    // waves per block in the MLP kernels

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float f) {  // round to nearest even
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
// two floats to two BF16 (round to nearest even) in one instruction on gfx950 (low half = lo)
__device__ __forceinline__ unsigned pk_bf16(float lo, float hi) {
    const f32x2 f = {lo, hi};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f, b16x2));
}
__device__ __forceinline__ bf16x4 bf16x4_of(float a, float b, float c, float d) {
    const u32x2 u = {pk_bf16(a, b), pk_bf16(c, d)};
    return __builtin_bit_cast(bf16x4, u);
}
__device__ __forceinline__ bf16x4 bf16x4_relu(f32x4 z) {
    return bf16x4_of(fmaxf(z[0], 0.f), fmaxf(z[1], 0.f), fmaxf(z[2], 0.f), fmaxf(z[3], 0.f));
}
__device__ __forceinline__ float relu(float v) { return v > 0.f ? v : 0.f; }
// K = 16: A lane l holds A[l%16][4(l/16)+j], B lane l holds B[4(l/16)+j][l%16]
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// K = 32: A lane l holds A[l%16][8(l/16)+j], B lane l holds B[8(l/16)+j][l%16]
__device__ __forceinline__ f32x4 mfma32(bf16x8s a, bf16x8s b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
}
// B operand of a 32-wide contraction from accumulator tiles t0 (rows 0..15) and t1 (16..31):
// position k = 8(l/16)+j of the lane's group then stands for row hid32(l/16, j) of the pair
__device__ __forceinline__ bf16x8s cat8(bf16x4 t0, bf16x4 t1) {
    return __builtin_shufflevector(t0, t1, 0, 1, 2, 3, 4, 5, 6, 7);
}
__device__ __forceinline__ int hid32(int g, int j) { return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4); }
// Orders this wave's LDS accesses (a staging area private to one wave needs no block barrier:
// the wave's LDS instructions execute in program order once the compiler keeps that order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ float softplus_f(float x) { return x > 20.f ? x : log1pf(expf(x)); }
__device__ __forceinline__ float sigmoid_f(float x) { return 1.f / (1.f + expf(-x)); }

// Weight fragments of one wave. Layer 1: Z1^T = W1 X^T (A = rows 16mb.. of W1, k = features);
// layer 2: Z2^T = W2 H1^T (A = rows 16mb.. of W2, k block q = hidden units 32q + hid32).
struct Frags {
    bf16x4 w1[4];
    bf16x8s w2[4][2];
};

__device__ __forceinline__ void load_frags(const float *__restrict__ w, Frags &F) {
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
        for (int j = 0; j < 4; ++j) F.w1[mb][j] = f2bf(w[kOffW1 + (16 * mb + r) * kF + 4 * g + j]);
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int j = 0; j < 8; ++j) F.w2[mb][q][j] = f2bf(w[kOffW2 + (16 * mb + r) * kH + 32 * q + hid32(g, j)]);
    }
}

// b1, b2, w3 (64 each) and b3 of the block in LDS; every thread of the block must call it.
constexpr int kVecB1 = 0, kVecB2 = 64, kVecW3 = 128, kVecB3 = 192;
__device__ __forceinline__ void load_vecs(const float *__restrict__ w, float *vec) {
    for (int k = threadIdx.x; k < 193; k += blockDim.x)
        vec[k] = k < 64 ? w[kOffB1 + k] : k < 128 ? w[kOffB2 + k - 64] : k < 192 ? w[kOffW3 + k - 128] : w[kOffB3];
    __syncthreads();
}
// the lane's four values of rows 16mb + 4(l/16) + j of a vector in LDS
__device__ __forceinline__ f32x4 vec4(const float *vec, int off, int mb) {
    const int g = (threadIdx.x & 63) >> 4;
    return *(const f32x4 *)(vec + off + 16 * mb + 4 * g);
}

// Features of entry e0 + l%16 for this lane's quarter (4 BF16), zero past the end.
__device__ __forceinline__ bf16x4 load_x(const unsigned short *__restrict__ feats, int64_t e0, int64_t nnz) {
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    const int64_t e = e0 + r;
    u32x2 u = {0u, 0u};
    if (e < nnz) {
        const uint2 raw = *(const uint2 *)(feats + e * kF + 4 * g);
        u[0] = raw.x;
        u[1] = raw.y;
    }
    return __builtin_bit_cast(bf16x4, u);
}

// Forward pass of one 16-entry tile (entries e0 + l%16, features x). Returns o for entry
// e0 + l%16 in every lane; z1, z2 (pre-activations, feature-major) and H1 in BF16 are kept
// for the backward pass. Biases initialise the accumulators.
__device__ __forceinline__ float tile_forward(const Frags &F, const float *vec, bf16x4 x, f32x4 (&z1)[4],
                                              f32x4 (&z2)[4], bf16x4 (&h1b)[4]) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        z1[mb] = mfma16(F.w1[mb], x, vec4(vec, kVecB1, mb));
        h1b[mb] = bf16x4_relu(z1[mb]);
    }
    float s = 0.f;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        f32x4 c = vec4(vec, kVecB2, mb);
#pragma unroll
        for (int q = 0; q < 2; ++q) c = mfma32(F.w2[mb][q], cat8(h1b[2 * q], h1b[2 * q + 1]), c);
        z2[mb] = c;
        const f32x4 w3 = vec4(vec, kVecW3, mb);
#pragma unroll
        for (int j = 0; j < 4; ++j) s += relu(c[j]) * w3[j];
    }
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    return s + vec[kVecB3];
}

// G value of entry e from the network output
__device__ __forceinline__ float g_of(float o, bool diag, float scale) {
    return diag ? softplus_f(o + kS0) * scale : o * scale;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Inference: G values for all pattern entries (and G^T values through the permutation).
__global__ void __launch_bounds__(64 * kWaves) k_mlp_factor(const float *__restrict__ w,
                                                            const unsigned short *__restrict__ feats,
                                                            const int32_t *__restrict__ grow,
                                                            const int32_t *__restrict__ gcol,
                                                            const float *__restrict__ gscale, int64_t nnz,
                                                            float *__restrict__ o_out, float *__restrict__ gval) {
    __shared__ __align__(16) float vec[196];
    load_vecs(w, vec);
    Frags F;
    load_frags(w, F);
    const int l = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * kWaves;
    // two 16-entry tiles per step (two independent MFMA chains); the next step's features and
    // output scales are always in flight
    auto load_out = [&](int64_t e0, float &gs, bool &dg) {
        const int64_t e = e0 + l;
        gs = 0.f;
        dg = false;
        if (l < 32 && e < nnz) {
            gs = gscale[e];
            dg = grow[e] == gcol[e];
        }
    };
    bf16x4 xn[2] = {load_x(feats, wave * 32, nnz), load_x(feats, wave * 32 + 16, nnz)};
    float gsn;
    bool dgn;
    load_out(wave * 32, gsn, dgn);
    for (int64_t e0 = wave * 32; e0 < nnz; e0 += nwaves * 32) {
        const bf16x4 x0 = xn[0], x1 = xn[1];
        const float gs = gsn;
        const bool dg = dgn;
        xn[0] = load_x(feats, e0 + nwaves * 32, nnz);
        xn[1] = load_x(feats, e0 + nwaves * 32 + 16, nnz);
        load_out(e0 + nwaves * 32, gsn, dgn);
        f32x4 z1[4], z2[4];
        bf16x4 h1b[4];
        const float o0 = tile_forward(F, vec, x0, z1, z2, h1b);
        const float o1 = tile_forward(F, vec, x1, z1, z2, h1b);
        const int64_t e = e0 + l;
        if (l < 32 && e < nnz) {
            const float o = l < 16 ? o0 : o1;
            if (o_out) o_out[e] = o;
            gval[e] = g_of(o, dg, gs);
        }
    }
}

// G^T values out[k] = in[src[k]], and BF16 copies of G and G^T for the application
__global__ void k_gather_f32(int64_t n, const int32_t *__restrict__ src, const float *__restrict__ in,
                             float *__restrict__ out, uint16_t *__restrict__ in_h, uint16_t *__restrict__ out_h,
                             const uint16_t *__restrict__ in_c16, const uint16_t *__restrict__ out_c16,
                             uint32_t *__restrict__ in_pk, uint32_t *__restrict__ out_pk) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        const float v = in[src[k]];
        out[k] = v;
        const uint32_t vo = (uint16_t)f2bf(v), vi = (uint16_t)f2bf(in[k]);
        out_h[k] = (uint16_t)vo;
        in_h[k] = (uint16_t)vi;
        // packed with the compact columns (BF16 bits high, column low)
        out_pk[k] = vo << 16 | out_c16[k];
        in_pk[k] = vi << 16 | in_c16[k];
    }
}

// ---------------------------------------------------------------------------------------
// Preconditioner application: y = G r (rows of G), then z = G^T y (rows of G^T) with the
// partials of r.z, from BF16 copies of G and G^T (the network's own precision; the products
// and sums are FP64, so M = G^T G stays one fixed SPD operator), both as tiled products (each block a contiguous, XCD-grouped range of row
// tiles). Grids are multiples of 8 blocks, at most 2048.
// T: the vectors' type (FP64, or FP32 in the inner iterations of the mixed-precision solve; the
// products and sums are FP64 either way, and the dot product takes the stored values).
template <bool DOT, typename T>
__global__ void __launch_bounds__(kTileThreads) k_prec_g(const int2 *__restrict__ tiles, int32_t ntiles,
                                                         const int32_t *__restrict__ ptr,
                                                         const TileCols cols, const uint16_t *__restrict__ val,
                                                         const T *__restrict__ in, T *__restrict__ out,
                                                         const T *__restrict__ r, double *__restrict__ part,
                                                         const int32_t *__restrict__ done) {
    if (done && done[0]) return;  // the solve has converged: nothing left to precondition
    __shared__ double prod[kTileCap];
    double acc = 0.0;
    auto pre = [&](int32_t row) { return DOT ? r[row] : (T)0; };
    auto epi = [&](int32_t row, double s, T rr) {
        const T st = (T)s;
        out[row] = st;
        if (DOT) acc += (double)st * (double)rr;
    };
    if (cols.all_pk)  // packed words only: the next tile's loaded during this one
        tile_spmv_pk(tiles, ntiles, ptr, cols, in, prod, pre, epi);
    else
        tile_spmv(tiles, ntiles, ptr, cols, val, in, prod, pre, epi);
    if (DOT) {
        __shared__ double sh[kTileThreads / 64];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
    }
}

// ---------------------------------------------------------------------------------------
// Kaporin loss pieces. Probes V and products W = G^T V, AW = A W are stored node-major
// [n][P] in FP32; sums are FP64.
constexpr int kP = 16;  // probes per training step

__global__ void k_probes(int32_t n, uint64_t seed, float *__restrict__ V) {
    // Rademacher signs from a counter-based hash of (seed, row, probe) (splitmix64 finaliser)
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)n * kP) return;
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (uint64_t)(k + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    V[k] = (z >> 63) ? 1.f : -1.f;
}

// out[row][p] = sum_k M_row,k in[k][p]; one lane per probe, 16 rows per block and pass. With
// DOT, also per-block partials of sum_row other[row][p] * out[row][p] (for the trace).
// The row's entries go through LDS eight at a time (one coalesced load per group of 16 lanes,
// then broadcast reads), so the eight gathers of in[] are independent loads in flight together;
// the products are summed in entry order, as a plain row loop would.
template <typename VT, bool DOT>
__global__ void __launch_bounds__(256) k_spmm16(int32_t n, const int32_t *__restrict__ ptr,
                                                const int32_t *__restrict__ col, const VT *__restrict__ val,
                                                const float *__restrict__ in, float *__restrict__ out,
                                                const float *__restrict__ other, double *__restrict__ part) {
    struct Ent {
        int32_t c;
        VT v;
    };
    __shared__ Ent ent[16][8];  // per group of 16 lanes (one row): the current eight entries
    const int p = threadIdx.x & 15, grp = threadIdx.x >> 4;
    double d = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * 16 + grp; row < n; row += (int64_t)gridDim.x * 16) {
        const int32_t beg = ptr[row], end = ptr[row + 1];
        double s = 0.0;
        for (int32_t j0 = beg; j0 < end; j0 += 8) {
            if (p < 8) {
                // past the row's end: a zero weight on column of the row's first entry
                const bool ok = j0 + p < end;
                ent[grp][p] = Ent{col[ok ? j0 + p : beg], ok ? val[j0 + p] : (VT)0};
            }
            wave_lds_sync();
            float x[8];
            VT v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const Ent q = ent[grp][k];
                v[k] = q.v;
                x[k] = in[(int64_t)q.c * kP + p];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) s += (double)v[k] * (double)x[k];
            wave_lds_sync();
        }
        out[row * kP + p] = (float)s;
        if (DOT) d += s * (double)other[row * kP + p];
    }
    if (DOT) {
        __shared__ double sh[256];
        sh[threadIdx.x] = d;
        __syncthreads();
        if (threadIdx.x < 16) {
            double t = 0.0;
            for (int k = 0; k < 16; ++k) t += sh[16 * k + threadIdx.x];
            part[(int64_t)blockIdx.x * kP + threadIdx.x] = t;
        }
    }
}

// Sum of m partials by one 256-thread block: eight independent strided loads in flight per
// thread, then a fixed-order tree (deterministic).
__device__ __forceinline__ double block_sum(const double *__restrict__ part, int32_t m, double *sh) {
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int32_t b = threadIdx.x;
    for (; b + 7 * 256 < m; b += 8 * 256)
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += part[b + u * 256];
    for (; b < m; b += 256) s[0] += part[b];
    sh[threadIdx.x] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
        __syncthreads();
    }
    return sh[0];
}

// T = sum of the trace partials / (P n) into loss[1]
__global__ void __launch_bounds__(256) k_trace_finish(const double *__restrict__ part, int32_t m, int32_t n,
                                                      double *loss) {
    __shared__ double sh[256];
    const double t = block_sum(part, m * kP, sh);
    if (threadIdx.x == 0) loss[1] = t / ((double)kP * (double)n);
}

// T = mean_p t_p / |v_p|^2 (|v_p|^2 = n); dG and d o per entry; partials of sum log G_ii.
__global__ void __launch_bounds__(256) k_kaporin_grad(int64_t nnz, int32_t n, const int32_t *__restrict__ grow,
                                                      const int32_t *__restrict__ gcol,
                                                      const float *__restrict__ gscale, const float *__restrict__ o,
                                                      const float *__restrict__ gval, const float *__restrict__ V,
                                                      const float *__restrict__ AW, float *__restrict__ d_o,
                                                      double *__restrict__ lpart, const double *__restrict__ loss) {
    __shared__ double sh[256];
    const double T = loss[1];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lg = 0.0;
    if (e < nnz) {
        const int32_t i = grow[e], j = gcol[e];
        // rows of 16 floats, 64-byte aligned: four 16-byte loads each
        const float4 *aw4 = reinterpret_cast<const float4 *>(AW + (int64_t)j * kP);
        const float4 *v4 = reinterpret_cast<const float4 *>(V + (int64_t)i * kP);
        float4 a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = aw4[q];
            b[q] = v4[q];
        }
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            s += (double)a[q].x * (double)b[q].x;
            s += (double)a[q].y * (double)b[q].y;
            s += (double)a[q].z * (double)b[q].z;
            s += (double)a[q].w * (double)b[q].w;
        }
        double dG = 2.0 / ((double)kP * T * (double)n) * s;
        const bool diag = i == j;
        float d;
        if (diag) {
            const double gi = gval[e];
            dG -= 2.0 / ((double)n * gi);
            lg = log(gi);
            d = (float)(dG * sigmoid_f(o[e] + kS0) * gscale[e]);
        } else {
            d = (float)(dG * gscale[e]);
        }
        d_o[e] = d;
    }
    sh[threadIdx.x] = lg;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------------------------------
// Solver pairs in the objective: the energy-norm loss
//   L_E = mean_k ||x_k - G^T G b_k||_A^2 / ||x_k||_A^2
// over a batch of QH_PAIR_BATCH recorded pairs (b_k, x_k), A x_k = b_k, so ||x_k||_A^2 = x_k.b_k
// (kept per pair). With Y = G B, V = X - G^T Y, AV = A V, GAV = G AV (node-major [n][16]):
//   dL_E/dG_ij = -(2/P) sum_k (Y_ik AV_jk + GAV_ik B_jk) / x_k.b_k,
// added with a weight to the Kaporin gradient in d o (through G's dependence on o).

// one pair into bank slot k: FP32 copies of b and x, and x.b (FP64) as per-block partials
__global__ void __launch_bounds__(256) k_pair_store(int32_t n, const double *__restrict__ b, const double *__restrict__ x,
                                                    float *__restrict__ pb, float *__restrict__ px,
                                                    double *__restrict__ part) {
    __shared__ double sh[256];
    double d = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double bi = b[i], xi = x[i];
        pb[i] = (float)bi;
        px[i] = (float)xi;
        d += bi * xi;
    }
    sh[threadIdx.x] = d;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_pair_store_finish(const double *__restrict__ part, int32_t m,
                                                           double *__restrict__ out) {
    __shared__ double sh[256];
    const double t = block_sum(part, m, sh);
    if (threadIdx.x == 0) *out = t;
}

static_assert(QH_PAIR_BATCH == kP, "a pair batch fills the 16 columns of the probe products");
struct PairIdx {
    int32_t k[QH_PAIR_BATCH];
};

// the batch's pairs node-major: B[i][p] = b_{idx p, i}, X likewise
__global__ void __launch_bounds__(256) k_pair_gather(int32_t n, PairIdx idx, const float *__restrict__ pb,
                                                     const float *__restrict__ px, float *__restrict__ B,
                                                     float *__restrict__ X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * QH_PAIR_BATCH) return;
    const int64_t i = t / QH_PAIR_BATCH;
    const int p = (int)(t - i * QH_PAIR_BATCH);
    const int64_t src = (int64_t)idx.k[p] * n + i;
    B[t] = pb[src];
    X[t] = px[src];
}

// V = X - V in place (V holds G^T Y)
__global__ void k_pair_residual(int64_t m, const float *__restrict__ X, float *__restrict__ V) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) V[t] = X[t] - V[t];
}

// per pair: v.Av from the product partials, weight 1/(x.b), and L_E into loss[2]
__global__ void __launch_bounds__(256) k_pair_finish(const double *__restrict__ part, int32_t m, PairIdx idx,
                                                     const double *__restrict__ xb, double *__restrict__ pw,
                                                     double *loss) {
    __shared__ double sh[256];
    double tot = 0.0;
    for (int p = 0; p < QH_PAIR_BATCH; ++p) {
        double s = 0.0;
        for (int32_t b = threadIdx.x; b < m; b += 256) s += part[(int64_t)b * kP + p];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
            __syncthreads();
        }
        const double w = 1.0 / xb[idx.k[p]];
        tot += sh[0] * w;
        if (threadIdx.x == 0) pw[p] = w;
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[2] = tot / QH_PAIR_BATCH;
}

// d o += lambda dL_E/do per entry
__global__ void __launch_bounds__(256) k_pair_grad(int64_t nnz, const int32_t *__restrict__ grow,
                                                   const int32_t *__restrict__ gcol, const float *__restrict__ gscale,
                                                   const float *__restrict__ o, const float *__restrict__ Y,
                                                   const float *__restrict__ AV, const float *__restrict__ GAV,
                                                   const float *__restrict__ B, const double *__restrict__ pw,
                                                   double lambda, float *__restrict__ d_o) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int32_t i = grow[e], j = gcol[e];
    const float *y = Y + (int64_t)i * kP, *g = GAV + (int64_t)i * kP;
    const float *av = AV + (int64_t)j * kP, *bb = B + (int64_t)j * kP;
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < QH_PAIR_BATCH; ++p)
        s += ((double)y[p] * (double)av[p] + (double)g[p] * (double)bb[p]) * pw[p];
    const double dG = -2.0 / QH_PAIR_BATCH * s;
    const double chain = i == j ? (double)sigmoid_f(o[e] + kS0) * gscale[e] : (double)gscale[e];
    d_o[e] += (float)(lambda * dG * chain);
}

// one block of 256: strided per-thread sums, then a tree (fixed order)
__global__ void __launch_bounds__(256) k_loss_finish(const double *__restrict__ lpart, int32_t m, int32_t n,
                                                     double *loss) {
    __shared__ double sh[256];
    const double lg = block_sum(lpart, m, sh);
    if (threadIdx.x == 0) loss[0] = log(loss[1]) - 2.0 / (double)n * lg;
}

// ---------------------------------------------------------------------------------------
// Backward pass over all entries: per-wave partial gradients of sum_e d_o[e] o[e].
// Layout of a wave's partial (kParams floats): same as the weights.
// A wave takes 32 entries per step (two 16-entry tiles): forward, dZ2^T = w3 d_o (z2 > 0),
// dH1^T = W2^T dZ2^T, dZ1^T = dH1^T (z1 > 0); then dZ2^T, H1^T, dZ1^T and X^T of both tiles go
// to the wave's LDS area as [row][entry] and the weight gradients contract over the 32 entries:
// dW2 += dZ2^T H1, dW1 += dZ1^T X. Bias and w3 gradients are per-lane sums.
constexpr int kTrStride = 40;               // BF16 per staged row: 32 entries + 8 (16-byte aligned rows, spread banks)
constexpr int kTrRows = 3 * kH + kF;        // dZ2^T, H1^T, dZ1^T, X^T
constexpr int kTrDZ2 = 0, kTrH1 = kH, kTrDZ1 = 2 * kH, kTrX = 3 * kH;
__global__ void __launch_bounds__(64 * kWaves) k_mlp_backward(const float *__restrict__ w,
                                                              const unsigned short *__restrict__ feats,
                                                              const float *__restrict__ d_o, int64_t nnz,
                                                              float *__restrict__ gpart) {
    __shared__ __align__(16) unsigned short tr[kWaves][kTrRows][kTrStride];
    __shared__ __align__(16) float vec[196];
    load_vecs(w, vec);
    Frags F;
    load_frags(w, F);
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    bf16x8s w2t[4][2];  // W2^T fragments for dH1^T = W2^T dZ2^T (k block q = outputs 32q + hid32)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int j = 0; j < 8; ++j) w2t[mb][q][j] = f2bf(w[kOffW2 + (32 * q + hid32(g, j)) * kH + 16 * mb + r]);
    const int wv = threadIdx.x >> 6;
    unsigned short(*T)[kTrStride] = tr[wv];
    const int64_t wave = (int64_t)blockIdx.x * kWaves + wv;
    f32x4 gW2[4][4], gW1[4];
    float gb1[4][4], gb2[4][4], gw3[4][4], gb3 = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gW2[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
            gb1[a][b] = gb2[a][b] = gw3[a][b] = 0.f;
        }
    }
    const int64_t nwaves = (int64_t)gridDim.x * kWaves;
    // the next step's features and output gradients are always in flight
    auto load_d = [&](int64_t e) { return e < nnz ? d_o[e] : 0.f; };
    bf16x4 xn[2] = {load_x(feats, wave * 32, nnz), load_x(feats, wave * 32 + 16, nnz)};
    float dn[2] = {load_d(wave * 32 + r), load_d(wave * 32 + 16 + r)};
    for (int64_t e0 = wave * 32; e0 < nnz; e0 += nwaves * 32) {
        const bf16x4 xt[2] = {xn[0], xn[1]};
        const float dt[2] = {dn[0], dn[1]};
        xn[0] = load_x(feats, e0 + nwaves * 32, nnz);
        xn[1] = load_x(feats, e0 + nwaves * 32 + 16, nnz);
        dn[0] = load_d(e0 + nwaves * 32 + r);
        dn[1] = load_d(e0 + nwaves * 32 + 16 + r);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            f32x4 z1[4], z2[4];
            bf16x4 h1b[4];
            (void)tile_forward(F, vec, xt[s], z1, z2, h1b);
            const float dout = dt[s];
            bf16x4 dz2b[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const f32x4 w3 = vec4(vec, kVecW3, mb);
                float dz[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    dz[j] = z2[mb][j] > 0.f ? w3[j] * dout : 0.f;
                    gb2[mb][j] += dz[j];
                    gw3[mb][j] += relu(z2[mb][j]) * dout;
                }
                dz2b[mb] = bf16x4_of(dz[0], dz[1], dz[2], dz[3]);
            }
            if (g == 0) gb3 += dout;
            bf16x4 dz1b[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q < 2; ++q) c = mfma32(w2t[mb][q], cat8(dz2b[2 * q], dz2b[2 * q + 1]), c);
                float dz[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    dz[j] = z1[mb][j] > 0.f ? c[j] : 0.f;
                    gb1[mb][j] += dz[j];
                }
                dz1b[mb] = bf16x4_of(dz[0], dz[1], dz[2], dz[3]);
            }
            // stage this tile's columns (entry 16s + l%16)
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mb + 4 * g + j;
                    T[kTrDZ2 + row][16 * s + r] = (unsigned short)dz2b[mb][j];
                    T[kTrH1 + row][16 * s + r] = (unsigned short)h1b[mb][j];
                    T[kTrDZ1 + row][16 * s + r] = (unsigned short)dz1b[mb][j];
                }
#pragma unroll
            for (int j = 0; j < 4; ++j) T[kTrX + 4 * g + j][16 * s + r] = (unsigned short)xt[s][j];
        }
        wave_lds_sync();
        // dW2[o][i] += sum_e dZ2^T[o][e] H1^T[i][e]: A = dZ2^T (o x e), B = H1 (e x i), k = 8(l/16)+j
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            const bf16x8s a = *(const bf16x8s *)&T[kTrDZ2 + 16 * ob + r][8 * g];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) {
                const bf16x8s b = *(const bf16x8s *)&T[kTrH1 + 16 * ib + r][8 * g];
                gW2[ob][ib] = mfma32(a, b, gW2[ob][ib]);
            }
        }
        // dW1[o][f] += sum_e dZ1^T[o][e] X[e][f]
        const bf16x8s xb = *(const bf16x8s *)&T[kTrX + r][8 * g];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            const bf16x8s a = *(const bf16x8s *)&T[kTrDZ1 + 16 * ob + r][8 * g];
            gW1[ob] = mfma32(a, xb, gW1[ob]);
        }
        wave_lds_sync();
    }
    // wave partials: C tiles directly; vector terms summed over the 16 entry lanes
    float *out = gpart + wave * 5313;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            out[kOffW1 + (16 * ob + 4 * g + j) * kF + r] = gW1[ob][j];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) out[kOffW2 + (16 * ob + 4 * g + j) * kH + 16 * ib + r] = gW2[ob][ib][j];
        }
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float a = gb1[mb][j], b = gb2[mb][j], c = gw3[mb][j];
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) {
                a += __shfl_xor(a, off, 16);
                b += __shfl_xor(b, off, 16);
                c += __shfl_xor(c, off, 16);
            }
            if (r == 0) {
                out[kOffB1 + 16 * mb + 4 * g + j] = a;
                out[kOffB2 + 16 * mb + 4 * g + j] = b;
                out[kOffW3 + 16 * mb + 4 * g + j] = c;
            }
        }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) gb3 += __shfl_xor(gb3, off, 16);
    if (l == 0) out[kOffB3] = gb3;
}

// Sum of the wave partials in a fixed order (one thread per parameter).
// Sum of the per-wave partial gradients in two fixed-order passes: chunk c of the waves
// (blockIdx.y) into part2[c][k], then the kGradChunks chunks per parameter.
constexpr int kGradChunks = 64;
__global__ void k_grad_reduce(const float *__restrict__ gpart, int64_t nwaves, double *__restrict__ part2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 5313) return;
    const int64_t per = (nwaves + kGradChunks - 1) / kGradChunks;
    const int64_t w0 = (int64_t)blockIdx.y * per, w1 = w0 + per < nwaves ? w0 + per : nwaves;
    double s = 0.0;
    for (int64_t wv = w0; wv < w1; ++wv) s += gpart[wv * 5313 + k];
    part2[(int64_t)blockIdx.y * 5313 + k] = s;
}
__global__ void k_grad_finish(const double *__restrict__ part2, float *__restrict__ grad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 5313) return;
    double s = 0.0;
    for (int c = 0; c < kGradChunks; ++c) s += part2[(int64_t)c * 5313 + k];
    grad[k] = (float)s;
}

__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, float lr, float b1, float b2, float eps, int32_t t) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 5313) return;
    const float gk = grad[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.f - powf(b1, (float)t));
    const float vh = vk / (1.f - powf(b2, (float)t));
    w[k] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------------------
// Host side
namespace {

float host_bf16_round(double x) {
    float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    std::memcpy(&f, &u, 4);
    return f;
}

}  // namespace

int qh_learned_setup(qh_ctx *c) {
    if (c->lp.built && c->lp.tau == c->tau_assembled) return QH_OK;
    const HostMesh &m = c->hm;
    const HostCsr &A = c->hA;
    const double tau = c->tau_assembled;
    const int32_t n = (int32_t)A.nrow;
    LearnedPrec &L = c->lp;
    int rc;
    if (!L.built) {
        // pattern of G (lower triangle of A, row-major, sorted) and of G^T
        std::vector<int32_t> gptr(n + 1, 0), gcol, grow;
        for (int32_t i = 0; i < n; ++i) {
            for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                if (A.col[k] <= i) {
                    gcol.push_back(A.col[k]);
                    grow.push_back(i);
                }
            gptr[i + 1] = (int32_t)gcol.size();
        }
        const int64_t nnz = (int64_t)gcol.size();
        std::vector<int32_t> tptr(n + 1, 0), tcol(nnz), tsrc(nnz);
        for (int64_t e = 0; e < nnz; ++e) tptr[gcol[e] + 1]++;
        for (int32_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
        std::vector<int32_t> cur(tptr.begin(), tptr.end() - 1);
        for (int64_t e = 0; e < nnz; ++e) {
            int32_t k = cur[gcol[e]]++;
            tcol[k] = grow[e];
            tsrc[k] = (int32_t)e;
        }
        L.n = n;
        L.nnz = nnz;
        L.h_row = grow;
        L.h_col = gcol;
        if ((rc = qh_alloc(c, &L.gptr, n + 1)) || (rc = qh_alloc(c, &L.gcol, nnz)) || (rc = qh_alloc(c, &L.grow, nnz)) ||
            (rc = qh_alloc(c, &L.tptr, n + 1)) || (rc = qh_alloc(c, &L.tcol, nnz)) || (rc = qh_alloc(c, &L.tsrc, nnz)) ||
            (rc = qh_alloc(c, &L.feats, nnz * kF)) || (rc = qh_alloc(c, &L.gscale, nnz)) ||
            (rc = qh_alloc(c, &L.gval, nnz)) || (rc = qh_alloc(c, &L.tval, nnz)) ||
            (rc = qh_alloc(c, &L.gval_h, nnz)) || (rc = qh_alloc(c, &L.tval_h, nnz)) || (rc = qh_alloc(c, &L.o, nnz)) ||
            (rc = qh_alloc(c, &L.d_o, nnz)) || (rc = qh_alloc(c, &L.y, n)) || (rc = qh_alloc(c, &L.w, 5313)) ||
            (rc = qh_alloc(c, &L.adam_m, 5313)) || (rc = qh_alloc(c, &L.adam_v, 5313)) ||
            (rc = qh_alloc(c, &L.grad, 5313)) || (rc = qh_alloc(c, &L.loss, 4)))
            return rc;
        QH_HIP(c, hipMemcpyAsync(L.gptr, gptr.data(), 4 * (n + 1), hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.gcol, gcol.data(), 4 * nnz, hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.grow, grow.data(), 4 * nnz, hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.tptr, tptr.data(), 4 * (n + 1), hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.tcol, tcol.data(), 4 * nnz, hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.tsrc, tsrc.data(), 4 * nnz, hipMemcpyHostToDevice, c->stream));
        std::vector<int2> gt, tt;
        if (!qh_make_tiles(gptr.data(), n, gt) || !qh_make_tiles(tptr.data(), n, tt))
            return qh_fail(c, QH_EINVAL, "factor row longer than a product tile");
        L.ngtiles = (int32_t)gt.size() - 1;
        L.nttiles = (int32_t)tt.size() - 1;
        if ((rc = qh_alloc(c, &L.gtiles, gt.size())) || (rc = qh_alloc(c, &L.ttiles, tt.size()))) return rc;
        QH_HIP(c, hipMemcpyAsync(L.gtiles, gt.data(), sizeof(int2) * gt.size(), hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.ttiles, tt.data(), sizeof(int2) * tt.size(), hipMemcpyHostToDevice, c->stream));
        std::vector<int4> gb, tb;
        std::vector<uint16_t> g16, t16;
        L.nnz_c16 = qh_compact_cols(gcol.data(), gt, gb, g16) + qh_compact_cols(tcol.data(), tt, tb, t16);
        auto all_compact = [](const std::vector<int4> &b) {
            for (const int4 &q : b)
                if (q.x < 0) return false;
            return !b.empty();
        };
        L.g_all_pk = all_compact(gb);
        L.t_all_pk = all_compact(tb);
        if ((rc = qh_alloc(c, &L.gtbase, gb.size())) || (rc = qh_alloc(c, &L.ttbase, tb.size())) ||
            (rc = qh_alloc(c, &L.gcol16, g16.size())) || (rc = qh_alloc(c, &L.tcol16, t16.size())) ||
            (rc = qh_alloc(c, &L.gpk, g16.size())) || (rc = qh_alloc(c, &L.tpk, t16.size())))
            return rc;
        QH_HIP(c, hipMemcpyAsync(L.gtbase, gb.data(), sizeof(int4) * gb.size(), hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.ttbase, tb.data(), sizeof(int4) * tb.size(), hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.gcol16, g16.data(), 2 * g16.size(), hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipMemcpyAsync(L.tcol16, t16.data(), 2 * t16.size(), hipMemcpyHostToDevice, c->stream));
        QH_HIP(c, hipStreamSynchronize(c->stream));
        if (!L.have_weights) {
            // He-normal hidden layers, zero output layer: the initial network is Jacobi
            std::mt19937_64 gen(12345);
            std::normal_distribution<double> n1(0.0, std::sqrt(2.0 / kF)), n2(0.0, std::sqrt(2.0 / kH));
            std::vector<float> w(5313, 0.f);
            for (int k = 0; k < kH * kF; ++k) w[kOffW1 + k] = (float)n1(gen);
            for (int k = 0; k < kH * kH; ++k) w[kOffW2 + k] = (float)n2(gen);
            QH_HIP(c, hipMemcpyAsync(L.w, w.data(), 4 * 5313, hipMemcpyHostToDevice, c->stream));
            L.have_weights = true;
        }
        L.built = true;
    }
    // features and scales depend on dt
    const int64_t nnz = L.nnz;
    std::vector<double> dA(n), dM(n), dS(n), off(n, 0.0), rl(n);
    for (int32_t i = 0; i < n; ++i) {
        rl[i] = A.ptr[i + 1] - A.ptr[i];
        double s = 0.0;
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            const double a = A.val[k] + tau * A.val2[k];
            s += std::fabs(a);
            if (A.col[k] == i) {
                dA[i] = a;
                dM[i] = A.val[k];
                dS[i] = tau * A.val2[k];
            }
        }
        off[i] = s / dA[i] - 1.0;
    }
    std::vector<double> tv(3 * (int64_t)n), ell(n);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t e = m.int_edges[i];
        const double *pa = &m.xyz[3 * (int64_t)m.edges[2 * e]], *pb = &m.xyz[3 * (int64_t)m.edges[2 * e + 1]];
        for (int d = 0; d < 3; ++d) tv[3 * i + d] = pb[d] - pa[d];
        ell[i] = std::sqrt(tv[3 * i] * tv[3 * i] + tv[3 * i + 1] * tv[3 * i + 1] + tv[3 * i + 2] * tv[3 * i + 2]);
    }
    std::vector<uint16_t> fh(nnz * kF);
    std::vector<float> sc(nnz);
    int64_t e = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            const int32_t j = A.col[k];
            if (j > i) continue;
            const double a = A.val[k] + tau * A.val2[k], mm = A.val[k], ss = tau * A.val2[k];
            double f[kF];
            const double cosang = (tv[3 * i] * tv[3 * j] + tv[3 * i + 1] * tv[3 * j + 1] + tv[3 * i + 2] * tv[3 * j + 2]) /
                                  (ell[i] * ell[j]);
            f[0] = i == j ? 1.0 : 0.0;
            f[1] = a / std::sqrt(dA[i] * dA[j]);
            f[2] = mm / std::sqrt(dM[i] * dM[j]);
            f[3] = ss / std::sqrt(dA[i] * dA[j]);
            f[4] = dS[i] / dA[i];
            f[5] = dS[j] / dA[j];
            f[6] = cosang;
            f[7] = std::log(ell[j] / ell[i]);
            f[8] = rl[i] / 20.0;
            f[9] = rl[j] / 20.0;
            f[10] = off[i];
            f[11] = off[j];
            f[12] = std::fabs(f[1]);
            f[13] = f[1] * f[1];
            f[14] = f[4] * f[5];
            f[15] = 1.0;
            for (int q = 0; q < kF; ++q) {
                float bf = host_bf16_round(f[q]);
                uint32_t u;
                std::memcpy(&u, &bf, 4);
                fh[e * kF + q] = (uint16_t)(u >> 16);
            }
            sc[e] = (float)(1.0 / std::sqrt(i == j ? dA[i] : dA[j]));
            ++e;
        }
    QH_HIP(c, hipMemcpyAsync(L.feats, fh.data(), 2 * nnz * kF, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, hipMemcpyAsync(L.gscale, sc.data(), 4 * nnz, hipMemcpyHostToDevice, c->stream));
    QH_HIP(c, hipStreamSynchronize(c->stream));
    L.tau = c->tau_assembled;
    L.factor_valid = false;
    return QH_OK;
}

static unsigned mlp_grid(int64_t nnz) {
    int64_t tiles = (nnz + 15) / 16;
    int64_t blocks = (tiles + kWaves - 1) / kWaves;
    return (unsigned)std::min<int64_t>(blocks, 2048);
}

int qh_learned_factor(qh_ctx *c) {
    LearnedPrec &L = c->lp;
    hipLaunchKernelGGL(k_mlp_factor, dim3(mlp_grid(L.nnz)), dim3(64 * kWaves), 0, c->stream, L.w, L.feats, L.grow,
                       L.gcol, L.gscale, L.nnz, L.o, L.gval);
    hipLaunchKernelGGL(k_gather_f32, dim3((unsigned)((L.nnz + 255) / 256)), dim3(256), 0, c->stream, L.nnz, L.tsrc,
                       L.gval, L.tval, L.gval_h, L.tval_h, (const uint16_t *)L.gcol16, (const uint16_t *)L.tcol16,
                       L.gpk, L.tpk);
    QH_HIP(c, hipGetLastError());
    L.factor_valid = true;
    return QH_OK;
}

unsigned qh_prec_grid(qh_ctx *c) { return tile_grid(c->lp.nttiles); }

// z = G^T (G r); part[block] = partial r.z (qh_prec_grid blocks). With done != null both
// passes return at once when done[0] is set (a converged solve).
hipError_t launch_prec_apply(qh_ctx *c, const double *r, double *z, double *part, const int32_t *done) {
    LearnedPrec &L = c->lp;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_prec_g<false, double>), dim3(tile_grid(L.ngtiles)), dim3(kTileThreads), 0, c->stream, L.gtiles,
                       L.ngtiles, L.gptr, TileCols{L.gcol, L.gcol16, L.gtbase, L.gpk, L.g_all_pk}, L.gval_h, r, L.y, (const double *)nullptr, (double *)nullptr, done);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_prec_g<true, double>), dim3(tile_grid(L.nttiles)), dim3(kTileThreads), 0, c->stream, L.ttiles,
                       L.nttiles, L.tptr, TileCols{L.tcol, L.tcol16, L.ttbase, L.tpk, L.t_all_pk}, L.tval_h, L.y, z, r, part, done);
    return hipGetLastError();
}

hipError_t launch_prec_apply32(qh_ctx *c, const float *r, float *z, double *part, const int32_t *done) {
    LearnedPrec &L = c->lp;
    if (!L.y32) {
        float *y = nullptr;
        if (hipMalloc((void **)&y, sizeof(float) * (size_t)std::max<int32_t>(1, L.n)) != hipSuccess)
            return hipErrorOutOfMemory;
        c->allocations.push_back((void *)y);
        L.y32 = y;
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_prec_g<false, float>), dim3(tile_grid(L.ngtiles)), dim3(kTileThreads), 0, c->stream, L.gtiles,
                       L.ngtiles, L.gptr, TileCols{L.gcol, L.gcol16, L.gtbase, L.gpk, L.g_all_pk}, L.gval_h, r, L.y32, (const float *)nullptr, (double *)nullptr, done);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_prec_g<true, float>), dim3(tile_grid(L.nttiles)), dim3(kTileThreads), 0, c->stream, L.ttiles,
                       L.nttiles, L.tptr, TileCols{L.tcol, L.tcol16, L.ttbase, L.tpk, L.t_all_pk}, L.tval_h, L.y32, z, r, part, done);
    return hipGetLastError();
}

// Loss and gradient for the current weights with probes V (device, [n][16] floats).
int qh_learned_record_pair(qh_ctx *c, const double *rhs, const double *sol) {
    LearnedPrec &L = c->lp;
    if (!L.pair_rec || L.pair_n >= L.pair_cap) return QH_OK;
    const int32_t n = c->A.n;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    const int64_t off = (int64_t)L.pair_n * n;
    hipLaunchKernelGGL(k_pair_store, dim3(g), dim3(256), 0, c->stream, n, rhs, sol, L.pair_b + off, L.pair_x + off,
                       L.ppart);
    hipLaunchKernelGGL(k_pair_store_finish, dim3(1), dim3(256), 0, c->stream, L.ppart, (int32_t)g,
                       L.pair_xb + L.pair_n);
    QH_HIP(c, hipGetLastError());
    L.pair_n++;
    return QH_OK;
}

int qh_learned_loss_grad(qh_ctx *c, const float *V_dev, bool want_grad, double pair_weight, const int32_t *pair_idx) {
    LearnedPrec &L = c->lp;
    int rc;
    if ((rc = qh_learned_factor(c))) return rc;
    const int32_t n = L.n;
    if (!L.W) {
        if ((rc = qh_alloc(c, &L.W, (int64_t)n * kP)) || (rc = qh_alloc(c, &L.AW, (int64_t)n * kP)) ||
            (rc = qh_alloc(c, &L.tpart, 2048 * kP)) ||
            (rc = qh_alloc(c, &L.lpart, (L.nnz + 255) / 256)) ||
            (rc = qh_alloc(c, &L.gpart, (int64_t)mlp_grid(L.nnz) * kWaves * 5313)) ||
            (rc = qh_alloc(c, &L.gpart2, (int64_t)kGradChunks * 5313)))
            return rc;
    }
    const unsigned gr = (unsigned)std::min<int64_t>((n + 15) / 16, 2048);
    const unsigned ge = (unsigned)((L.nnz + 255) / 256);
    if (V_dev) {
        // W = G^T V, AW = A W (+ partial traces)
        hipLaunchKernelGGL((k_spmm16<float, false>), dim3(gr), dim3(256), 0, c->stream, n, L.tptr, L.tcol, L.tval, V_dev,
                           L.W, (const float *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL((k_spmm16<double, true>), dim3(gr), dim3(256), 0, c->stream, n, c->A.ptr, c->A.col, c->A.val,
                           L.W, L.AW, L.W, L.tpart);
        hipLaunchKernelGGL(k_trace_finish, dim3(1), dim3(256), 0, c->stream, L.tpart, (int32_t)gr, n, L.loss);
        hipLaunchKernelGGL(k_kaporin_grad, dim3(ge), dim3(256), 0, c->stream, L.nnz, n, L.grow, L.gcol, L.gscale, L.o,
                           L.gval, V_dev, L.AW, L.d_o, L.lpart, L.loss);
        hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, c->stream, L.lpart, (int32_t)ge, n, L.loss);
    } else {
        // the pair term alone: its gradient is added to zero
        QH_HIP(c, hipMemsetAsync(L.d_o, 0, sizeof(float) * L.nnz, c->stream));
    }
    if (pair_weight > 0.0 && pair_idx) {
        // the batch of recorded pairs: Y = G B, V = X - G^T Y, AV = A V (+ v.Av partials), GAV = G AV
        if (!L.PB) {
            const int64_t m = (int64_t)n * kP;
            if ((rc = qh_alloc(c, &L.PB, m)) || (rc = qh_alloc(c, &L.PX, m)) || (rc = qh_alloc(c, &L.PY, m)) ||
                (rc = qh_alloc(c, &L.PV, m)) || (rc = qh_alloc(c, &L.PAV, m)) || (rc = qh_alloc(c, &L.PGAV, m)) ||
                (rc = qh_alloc(c, &L.pw, QH_PAIR_BATCH)))
                return rc;
        }
        PairIdx idx;
        for (int p = 0; p < QH_PAIR_BATCH; ++p) idx.k[p] = pair_idx[p];
        const int64_t m = (int64_t)n * kP;
        hipLaunchKernelGGL(k_pair_gather, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c->stream, n, idx, L.pair_b,
                           L.pair_x, L.PB, L.PX);
        hipLaunchKernelGGL((k_spmm16<float, false>), dim3(gr), dim3(256), 0, c->stream, n, L.gptr, L.gcol, L.gval, L.PB,
                           L.PY, (const float *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL((k_spmm16<float, false>), dim3(gr), dim3(256), 0, c->stream, n, L.tptr, L.tcol, L.tval, L.PY,
                           L.PV, (const float *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL(k_pair_residual, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c->stream, m, L.PX, L.PV);
        hipLaunchKernelGGL((k_spmm16<double, true>), dim3(gr), dim3(256), 0, c->stream, n, c->A.ptr, c->A.col, c->A.val,
                           L.PV, L.PAV, L.PV, L.tpart);
        hipLaunchKernelGGL((k_spmm16<float, false>), dim3(gr), dim3(256), 0, c->stream, n, L.gptr, L.gcol, L.gval, L.PAV,
                           L.PGAV, (const float *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL(k_pair_finish, dim3(1), dim3(256), 0, c->stream, L.tpart, (int32_t)gr, idx, L.pair_xb, L.pw,
                           L.loss);
        hipLaunchKernelGGL(k_pair_grad, dim3(ge), dim3(256), 0, c->stream, L.nnz, L.grow, L.gcol, L.gscale, L.o, L.PY,
                           L.PAV, L.PGAV, L.PB, L.pw, pair_weight, L.d_o);
    }
    if (want_grad) {
        const unsigned gm = mlp_grid(L.nnz);
        hipLaunchKernelGGL(k_mlp_backward, dim3(gm), dim3(64 * kWaves), 0, c->stream, L.w, L.feats, L.d_o, L.nnz, L.gpart);
        hipLaunchKernelGGL(k_grad_reduce, dim3((5313 + 255) / 256, kGradChunks), dim3(256), 0, c->stream, L.gpart,
                           (int64_t)gm * kWaves, L.gpart2);
        hipLaunchKernelGGL(k_grad_finish, dim3((5313 + 255) / 256), dim3(256), 0, c->stream, L.gpart2, L.grad);
    }
    QH_HIP(c, hipGetLastError());
    return QH_OK;
}

int qh_learned_adam(qh_ctx *c, float lr, int32_t t) {
    LearnedPrec &L = c->lp;
    hipLaunchKernelGGL(k_adam, dim3((5313 + 255) / 256), dim3(256), 0, c->stream, L.w, L.adam_m, L.adam_v, L.grad, lr,
                       0.9f, 0.999f, 1e-8f, t);
    QH_HIP(c, hipGetLastError());
    L.factor_valid = false;
    return QH_OK;
}

int qh_learned_probes(qh_ctx *c, float *V_dev, uint64_t seed) {
    const int64_t tot = (int64_t)c->lp.n * kP;
    hipLaunchKernelGGL(k_probes, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, c->lp.n, seed, V_dev);
    QH_HIP(c, hipGetLastError());
    return QH_OK;
}
