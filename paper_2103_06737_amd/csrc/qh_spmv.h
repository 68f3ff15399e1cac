// Tiled CSR products y_i = sum_j a_ij x_j for the solvers (FP64 or FP32 values and vectors,
// FP64 products and sums) and the learned factor (BF16 entries); shared by qh_solver.hip and
// qh_learned.hip.
//
// A tile is a run of at most kTileRows consecutive rows holding at most kTileCap entries.
// One 256-thread block walks a contiguous range of tiles. Per tile, every thread first forms
// kTileCap / 256 products a_ij * x_j over the tile's entries in storage order (the value and
// column loads are coalesced and independent of the row structure, so many are in flight at
// once), keeping them in LDS; then thread t adds up the products of row (first row + t) and
// hands the sum to an epilogue. Against one row per lane group this removes the chain of
// dependent loads (row pointer -> entries -> gathered vector) per row. Column indices are read
// as 16 bits (a window of the tile and an offset in it) wherever the tile allows it (TileCols).
#pragma once

#include <type_traits>

#include "qh_internal.h"

constexpr int kTileThreads = 256;
constexpr int kTileRows = kTileThreads;  // one row per thread in the summing pass
constexpr int kTileCap = 2048;           // products per tile (16 KB of LDS)
constexpr int kTileUnroll = 8;           // product loads issued together per thread

// Tile starts {first row, first entry}; tiles[ntiles] = {n, nnz}. Rows longer than kTileCap
// entries are not supported (returns false).
bool qh_make_tiles(const int32_t *ptr, int32_t n, std::vector<int2> &tiles);

// Compact columns of every tile (TileCols): the windows of tile k are laid greedily from its
// smallest column up (each starts at the smallest column not yet covered); a tile that needs more
// than four keeps 32-bit columns (tbase[k].x = -1). Returns the number of entries in compact tiles.
int64_t qh_compact_cols(const int32_t *col, const std::vector<int2> &tiles, std::vector<int4> &tbase,
                        std::vector<uint16_t> &col16);

// Entry values: FP64, FP32, or BF16 (stored as its 16 bits), all widened to FP64.
__device__ __forceinline__ double tile_val(double v) { return v; }
__device__ __forceinline__ double tile_val(float v) { return (double)v; }
__device__ __forceinline__ double tile_val(uint16_t h) { return (double)__uint_as_float((unsigned)h << 16); }

// Contiguous tile range of this block; the block index is remapped so that each of the 8
// XCDs (which receive blocks round-robin) covers one contiguous span of tiles. The grid must
// be a multiple of 8 blocks.
__device__ __forceinline__ void tile_range(int32_t ntiles, int32_t &tb, int32_t &te) {
    const unsigned nb = gridDim.x, per_x = nb / 8;
    const unsigned lb = (blockIdx.x & 7) * per_x + (blockIdx.x >> 3);
    const int32_t per = (int32_t)((ntiles + nb - 1) / nb);
    tb = (int32_t)lb * per;
    te = tb + per < ntiles ? tb + per : ntiles;
    if (tb > ntiles) tb = ntiles;
}

// Tile headers and window bases are the same for the whole block: kept in scalar registers.
__device__ __forceinline__ int2 uniform2(int2 v) {
    return make_int2(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y));
}
__device__ __forceinline__ int4 uniform4(int4 v) {
    return make_int4(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y),
                     __builtin_amdgcn_readfirstlane(v.z), __builtin_amdgcn_readfirstlane(v.w));
}

// For every row of this block's tiles: epi(row, sum_j a_row,j xg(j), pre(row)). pre(row) loads
// what the epilogue needs from the row's own entries; it is issued with the tile's entry loads,
// and the next tile's header is fetched one tile ahead, so a tile costs
// two dependent memory round trips (entries, then gathered vector). All threads of the block
// must call it (it synchronises the block).
template <typename VT, typename XG, typename Pre, typename Epi>
__device__ __forceinline__ void tile_spmv_g(const int2 *__restrict__ tiles, int32_t ntiles,
                                            const int32_t *__restrict__ ptr, const TileCols cols,
                                            const VT *__restrict__ val, XG &&xg,
                                            double *prod /* LDS, kTileCap */, Pre &&pre, Epi &&epi) {
    using PF = decltype(pre(0));
    int32_t tb, te;
    tile_range(ntiles, tb, te);
    if (tb >= te) return;  // the same for every thread of the block
    const int tid = threadIdx.x;
    int2 t0 = uniform2(tiles[tb]), t1 = uniform2(tiles[tb + 1]);
    int4 base0 = uniform4(cols.tbase ? cols.tbase[tb] : make_int4(-1, 0, 0, 0));
    for (int32_t ti = tb; ti < te; ++ti) {
        const int2 t2 = uniform2(tiles[ti + 2 <= ntiles ? ti + 2 : ntiles]);
        const int4 base1 = uniform4(cols.tbase && ti + 1 < ntiles ? cols.tbase[ti + 1] : make_int4(-1, 0, 0, 0));
        const int32_t row = t0.x + tid;
        int32_t js = 0, je = 0;
        PF pf{};
        if (row < t1.x) {
            js = ptr[row] - t0.y;
            je = ptr[row + 1] - t0.y;
            pf = pre(row);
        }
        const int32_t cnt = t1.y - t0.y;  // >= 1 whenever the tile has rows with entries
        for (int32_t b = 0; b < cnt; b += kTileUnroll * kTileThreads) {
            VT v[kTileUnroll];
            int32_t c[kTileUnroll];
            bool packed = false;
            if constexpr (std::is_same<VT, uint16_t>::value) packed = cols.pk != nullptr;
            if (base0.x >= 0 && packed) {  // the same for the whole block
#pragma unroll
                for (int u = 0; u < kTileUnroll; ++u) {
                    int32_t j = b + u * kTileThreads + tid;
                    j = j < cnt ? j : cnt - 1;  // clamped: every load stays inside the tile
                    const uint32_t e = cols.pk[t0.y + j];
                    v[u] = (VT)(e >> 16);
                    const uint32_t h = e & 0xffffu;
                    const uint32_t w = h >> 14;
                    c[u] = (w == 0 ? base0.x : w == 1 ? base0.y : w == 2 ? base0.z : base0.w) + (int32_t)(h & 0x3fffu);
                }
            } else if (base0.x >= 0) {
#pragma unroll
                for (int u = 0; u < kTileUnroll; ++u) {
                    int32_t j = b + u * kTileThreads + tid;
                    j = j < cnt ? j : cnt - 1;  // clamped: every load stays inside the tile
                    v[u] = val[t0.y + j];
                    const uint32_t h = cols.col16[t0.y + j];
                    const uint32_t w = h >> 14;
                    c[u] = (w == 0 ? base0.x : w == 1 ? base0.y : w == 2 ? base0.z : base0.w) + (int32_t)(h & 0x3fffu);
                }
            } else {
#pragma unroll
                for (int u = 0; u < kTileUnroll; ++u) {
                    int32_t j = b + u * kTileThreads + tid;
                    j = j < cnt ? j : cnt - 1;
                    v[u] = val[t0.y + j];
                    c[u] = cols.col[t0.y + j];
                }
            }
            double xv[kTileUnroll];
#pragma unroll
            for (int u = 0; u < kTileUnroll; ++u) xv[u] = xg(c[u]);
#pragma unroll
            for (int u = 0; u < kTileUnroll; ++u) {
                const int32_t j = b + u * kTileThreads + tid;
                if (j < cnt) prod[j] = tile_val(v[u]) * xv[u];
            }
        }
        __syncthreads();
        if (row < t1.x) {
            double s = 0.0;
            for (int32_t j = js; j < je; ++j) s += prod[j];
            epi(row, s, pf);
        }
        __syncthreads();
        t0 = t1;
        t1 = t2;
        base0 = base1;
    }
}

// Block barrier that orders LDS only: a wave waits for its own LDS operations, not for its
// global loads in flight (a plain __syncthreads also waits for those).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// BF16 entries with packed words (cols.pk: value bits << 16 | 16-bit column), for matrices
// whose tiles are all compact and non-empty (cols.all_pk): a tile's words are one load per
// thread and unroll slot (a tile holds at most kTileUnroll * kTileThreads entries), so the next
// tile's words are loaded while this tile's vector gathers, products and row sums run. They
// are issued after the gathers, with the next tile's row bounds (the memory counter completes
// in order, so waiting for the gathers does not wait for them); the block barriers order LDS
// only, so these loads stay in flight across them. Per tile one
// dependent memory round trip remains exposed (the gathers) instead of two. epi and pre as in
// tile_spmv_g.
static_assert(kTileCap == kTileUnroll * kTileThreads, "a tile is one round of loads");
template <typename XT, typename Pre, typename Epi>
__device__ __forceinline__ void tile_spmv_pk(const int2 *__restrict__ tiles, int32_t ntiles,
                                             const int32_t *__restrict__ ptr, const TileCols cols,
                                             const XT *__restrict__ x, double *prod /* LDS, kTileCap */,
                                             Pre &&pre, Epi &&epi) {
    using PF = decltype(pre(0));
    int32_t tb, te;
    tile_range(ntiles, tb, te);
    if (tb >= te) return;  // the same for every thread of the block
    const int tid = threadIdx.x;
    const uint32_t *__restrict__ pk = cols.pk;
    // the words of the tile whose entries start at first (cnt >= 1 of them; cnt = 0 asks for
    // none, and the loads then repeat entry 0, unused); the slots past cnt repeat the tile's last
    // entry, so every load stays inside the array
    auto load_words = [&](uint32_t w[kTileUnroll], int32_t first, int32_t cnt) {
        if (cnt < 1) first = 0, cnt = 1;
#pragma unroll
        for (int u = 0; u < kTileUnroll; ++u) {
            const int32_t j = u * kTileThreads + tid;
            w[u] = pk[first + (j < cnt ? j : cnt - 1)];
        }
    };
    int2 t0 = uniform2(tiles[tb]), t1 = uniform2(tiles[tb + 1]);
    int4 base0 = uniform4(cols.tbase[tb]);
    uint32_t w[kTileUnroll];
    load_words(w, t0.y, t1.y - t0.y);
    int32_t row = t0.x + tid, js = 0, je = 0;  // this thread's row of the tile and its entries
    PF pf{};
    if (row < t1.x) {
        js = ptr[row];
        je = ptr[row + 1];
        pf = pre(row);
    }
    for (int32_t ti = tb; ti < te; ++ti) {
        const bool more = ti + 1 < te;
        const int2 t2 = uniform2(tiles[ti + 2 <= ntiles ? ti + 2 : ntiles]);
        const int4 base1 = more ? uniform4(cols.tbase[ti + 1]) : base0;
        float v[kTileUnroll];  // BF16 values, exact in FP32
        int32_t c[kTileUnroll];
#pragma unroll
        for (int u = 0; u < kTileUnroll; ++u) {
            v[u] = __uint_as_float(w[u] & 0xffff0000u);
            const uint32_t h = w[u] & 0xffffu;
            const uint32_t q = h >> 14;
            c[u] = (q == 0 ? base0.x : q == 1 ? base0.y : q == 2 ? base0.z : base0.w) + (int32_t)(h & 0x3fffu);
        }
        XT xv[kTileUnroll];
#pragma unroll
        for (int u = 0; u < kTileUnroll; ++u) xv[u] = x[c[u]];
        // the next tile's row bounds and words
        const int32_t rn = t1.x + tid;
        int32_t jsn = 0, jen = 0;
        PF pfn{};
        if (more && rn < t2.x) {
            jsn = ptr[rn];
            jen = ptr[rn + 1];
            pfn = pre(rn);
        }
        load_words(w, t1.y, more ? t2.y - t1.y : 0);
        // every slot is stored (those past the tile's entries repeat its last one, and no row
        // reads them)
#pragma unroll
        for (int u = 0; u < kTileUnroll; ++u) prod[u * kTileThreads + tid] = (double)v[u] * (double)xv[u];
        lds_barrier();
        if (row < t1.x) {
            double s = 0.0;
            for (int32_t j = js - t0.y; j < je - t0.y; ++j) s += prod[j];
            epi(row, s, pf);
        }
        lds_barrier();
        row = rn;
        js = jsn;
        je = jen;
        pf = pfn;
        t0 = t1;
        t1 = t2;
        base0 = base1;
    }
}

// The same with the gathered vector read from memory (converted to FP64).
template <typename VT, typename XT, typename Pre, typename Epi>
__device__ __forceinline__ void tile_spmv(const int2 *__restrict__ tiles, int32_t ntiles,
                                          const int32_t *__restrict__ ptr, const TileCols cols,
                                          const VT *__restrict__ val, const XT *__restrict__ x,
                                          double *prod /* LDS, kTileCap */, Pre &&pre, Epi &&epi) {
    tile_spmv_g(tiles, ntiles, ptr, cols, val, [&](int32_t j) { return (double)x[j]; }, prod, pre, epi);
}

// Grid of a tiled product: one block per tile up to 2048 blocks, a multiple of 8.
inline unsigned tile_grid(int32_t ntiles) {
    int64_t b = ntiles < 2048 ? ntiles : 2048;
    if (b < 8) b = 8;
    return (unsigned)((b + 7) / 8 * 8);
}
