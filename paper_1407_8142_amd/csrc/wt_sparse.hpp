// Node tables over the nonempty nodes only, for 32-bit alphabets much
// larger than the sequence (and for sigma up to 2^32, L up to 32, where a
// dense table of 2^(L+1) entries per build cannot exist).
//
// The nonempty nodes of level l are the distinct top-l-bit prefixes of the
// symbols present (Fig. 1 keeps only nonempty nodes too), at most
// min(n, 2^l) of them.  With U the sorted distinct symbols (from C), level
// l's nodes in order are the distinct values of U[j] >> (L-l); for node j:
//   NID[j]  = its prefix p (the node id within the level),
//   NS[j]   = its first position C[p * 2^(L-l)] (NS[m] = n),
//   D[2j]   = ones of B_l before it,  D[2j+1] = zeros of B_l before node j+1.
// The level pass finds a symbol's node j inside its tile's node range (a
// tile of S_l holds a contiguous run of nodes, found by position) by its
// prefix; everything else is the generic level pass.
#pragma once

#include "wt_kernels.hpp"

namespace wt {

// Distinct symbols: U[r] = the r-th c < sigma with C[c+1] > C[c]; *u = |U|.
struct CompactOp {
    const uint64_t *C;
    uint64_t sigma;
    uint32_t *U;
    uint64_t *u;
    __device__ uint64_t value(uint64_t c) const { return C[c + 1] > C[c] ? 1u : 0u; }
    __device__ void store(uint64_t c, uint64_t ex) const {
        if (C[c + 1] > C[c]) U[ex] = (uint32_t)c;
        if (c + 1 == sigma) *u = ex + (C[c + 1] > C[c] ? 1u : 0u);
    }
    __device__ uint64_t seg_start(uint64_t) const { return 0; }
    __device__ uint64_t chunk_seg_first(uint64_t) const { return 0; }
};

// Level l's nodes (shift s = L - l >= 1): NID[r] = distinct U >> s, *m = count.
struct NodeIdOp {
    const uint32_t *U;
    const uint64_t *u;
    uint32_t s;
    uint32_t *NID;
    uint64_t *m;
    __device__ bool head(uint64_t g) const {
        const uint64_t nu = *u;
        if (g >= nu) return false;
        return g == 0 || ((uint64_t)U[g] >> s) != ((uint64_t)U[g - 1] >> s);
    }
    __device__ uint64_t value(uint64_t g) const { return head(g) ? 1u : 0u; }
    __device__ void store(uint64_t g, uint64_t ex) const {
        const bool h = head(g);
        if (h) NID[ex] = (uint32_t)((uint64_t)U[g] >> s);
        if (g + 1 == *u) *m = ex + (h ? 1u : 0u);
    }
    __device__ uint64_t seg_start(uint64_t) const { return 0; }
    __device__ uint64_t chunk_seg_first(uint64_t) const { return 0; }
};

// Level l's table from C: zeros of node j = symbols of its left half.
struct SparseTableOp {
    const uint64_t *C;
    uint64_t sigma, n;
    const uint32_t *NID;
    const uint64_t *m;
    uint32_t s;            // L - l
    uint64_t *NS, *D;
    uint64_t *level_zeros; // this level's zeros (the last node's D[2j+1])
    __device__ uint64_t Cc(uint64_t x) const { return C[x < sigma ? x : sigma]; }
    __device__ uint64_t value(uint64_t j) const {
        if (j >= *m) return 0;
        const uint64_t p = NID[j];
        return Cc((2 * p + 1) << (s - 1)) - Cc(p << s);
    }
    __device__ void store(uint64_t j, uint64_t ex) const {
        const uint64_t nm = *m;
        if (j >= nm) return;
        const uint64_t p = NID[j];
        const uint64_t start = Cc(p << s), z = Cc((2 * p + 1) << (s - 1)) - start;
        NS[j] = start;
        D[2 * j] = start - ex;
        D[2 * j + 1] = ex + z;
        if (j + 1 == nm) {
            NS[nm] = n;
            *level_zeros = ex + z;
        }
    }
    __device__ uint64_t seg_start(uint64_t) const { return 0; }
    __device__ uint64_t chunk_seg_first(uint64_t) const { return 0; }
};

struct SparseArgs {
    const uint32_t *NID;  // level l's node ids, in order
    const uint64_t *NS;   // their first positions (NS[m] = n)
    const uint64_t *m;    // number of nodes
    const uint64_t *level_zeros;
};

// Last j in [lo, hi) with NS[j] <= x (NS[lo] <= x assumed).
__device__ __forceinline__ uint64_t node_at(const uint64_t *NS, uint64_t lo, uint64_t hi, uint64_t x) {
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (NS[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

constexpr int kSparseCache = 1024;  // node ids of a tile's range kept in LDS

template <typename TIN>
struct LdsSparse {
    __align__(16) unsigned char stage[TileCfg<TIN>::kBytes];
    uint64_t words[TileCfg<TIN>::kWords];
    uint32_t zpre[TileCfg<TIN>::kWords];
    uint32_t nid[kSparseCache];
    uint64_t j0, nj;  // the tile's first node and its node count
    uint64_t Z0;
    uint32_t Zt;
    CountTable ct;
};

// The generic level pass (any width, any n) with the sparse node table;
// with a.tails the blocks also write the level's directory tail.
template <typename TIN, typename TOUT, bool SCATTER, bool DIRS>
__device__ __forceinline__ void level_tile_sparse(const LevelArgs &a, const SparseArgs &sp, uint64_t tile,
                                                  LdsSparse<TIN> &s) {
    using Cfg = TileCfg<TIN>;
    constexpr int kTile = Cfg::kTile, kIt = Cfg::kItems, kWPL = Cfg::kWPL;

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint64_t t0 = tile * kTile;
    const uint32_t len = (uint32_t)min((uint64_t)kTile, a.n - t0);
    const uint32_t k = a.k;

    TIN *stage_in = reinterpret_cast<TIN *>(s.stage);
    const TIN *in = reinterpret_cast<const TIN *>(a.in) + t0;
    for (uint32_t e = tid; e < len; e += kBlock) stage_in[e] = in[e];
    if (SCATTER) {
        count_init(s.ct, tid);
        if (tid == 0) {
            const uint64_t m = *sp.m;
            const uint64_t j0 = node_at(sp.NS, 0, m, t0);
            const uint64_t j1 = node_at(sp.NS, j0, m, t0 + len - 1);
            s.j0 = j0;
            s.nj = j1 - j0 + 1;
        }
    }
    if (*a.status) return;
    if (DIRS && a.tails) {
        const uint64_t zeros = *sp.level_zeros;
        dir_tail(0, zeros, a.n, a.L, a.rank, a.rank_len, a.sel1, a.sel0, a.cap, a.sel_counts + a.level,
                 tile * kBlock + tid, (uint64_t)gridDim.x * kBlock);
    }
    __syncthreads();
    if (SCATTER && s.nj <= (uint64_t)kSparseCache)
        for (uint32_t j = tid; j < (uint32_t)s.nj; j += kBlock) s.nid[j] = sp.NID[s.j0 + j];

    // Bits and zero counts per word (striped view, as the generic pass).
    uint32_t pk[kIt];
#pragma unroll
    for (int r = 0; r < kIt; ++r) {
        const uint32_t e = (uint32_t)(r * kBlock + tid);
        const bool valid = e < len;
        const uint32_t sym = valid ? (uint32_t)stage_in[e] : 0u;
        pk[r] = sym;
        const bool bit = valid && ((sym >> k) & 1u);
        const uint64_t vm = __ballot(valid), w = __ballot(bit);
        if (lane == 0) {
            s.words[r * kWaves + wave] = w;
            s.zpre[r * kWaves + wave] = (uint32_t)(__popcll(vm) - __popcll(w));
        }
    }
    __syncthreads();

    if (wave == 0) {
        uint32_t zp[kWPL];
        uint64_t wd[kWPL];
        uint32_t own = 0;
#pragma unroll
        for (int m = 0; m < kWPL; ++m) {
            zp[m] = own;
            own += s.zpre[lane * kWPL + m];
            wd[m] = s.words[lane * kWPL + m];
        }
        const uint32_t inc = wave_incl_scan_u32(own, lane);
        const uint32_t Zt = __shfl(inc, kWave - 1, kWave);
        const uint64_t Z0 = a.tile_prefix[tile];
        const uint32_t ex = inc - own;
#pragma unroll
        for (int m = 0; m < kWPL; ++m) {
            zp[m] += ex;
            s.zpre[lane * kWPL + m] = zp[m];
        }
        if (lane == 0) {
            s.Z0 = Z0;
            s.Zt = Zt;
        }
#pragma unroll
        for (int m = 0; m < kWPL; ++m) {
            const uint32_t w = (uint32_t)lane * kWPL + m;
            if (w * 64u < len) a.bits[(t0 >> 6) + w] = wd[m];
        }
        if (DIRS) emit_directories<kWPL>(wd, zp, Z0, t0, len, Zt, a.n, a.rank, a.sel1, a.sel0, lane);
    }
    if (!SCATTER) return;
    __syncthreads();
    const uint64_t Z0 = s.Z0;
    const uint32_t Zt = s.Zt;

    // Stable split into LDS (zeros first), as the generic pass.
    TOUT *stage_out = reinterpret_cast<TOUT *>(s.stage);
    const uint64_t lt = lanemask_lt(lane);
#pragma unroll
    for (int r = 0; r < kIt; ++r) {
        const uint32_t e = (uint32_t)(r * kBlock + tid);
        if (e < len) {
            const uint64_t w = s.words[r * kWaves + wave];
            const uint32_t zl = s.zpre[r * kWaves + wave] + (uint32_t)__popcll(~w & lt);
            const uint32_t slot = ((w >> lane) & 1ull) ? Zt + (e - zl) : zl;
            stage_out[slot] = (TOUT)pk[r];
        }
    }
    __syncthreads();

    // Scatter: node j of the symbol by its prefix inside the tile's node
    // range, then Fig. 1's destinations through the table (see level_tile).
    TOUT *out = reinterpret_cast<TOUT *>(a.out);
    const uint64_t O0 = t0 - Z0;
    const uint32_t kn = k - 1;
    const uint64_t j0 = s.j0, nj = s.nj;
    const bool cached = nj <= (uint64_t)kSparseCache;
    LaneCount lc;
    for (int r = 0; r < kIt; ++r) {
        const uint32_t sp_ = (uint32_t)(r * kBlock + tid);
        if (sp_ < len) {
            const uint32_t v = (uint32_t)stage_out[sp_];
            const uint64_t prefix = (uint64_t)v >> (k + 1);
            uint64_t lo = 0, hi = nj;  // id(lo) <= prefix < id(hi)
            while (hi - lo > 1) {
                const uint64_t mid = lo + (hi - lo) / 2;
                const uint64_t id = cached ? s.nid[mid] : sp.NID[j0 + mid];
                if (id <= prefix) lo = mid;
                else hi = mid;
            }
            const uint64_t j = j0 + lo;
            const uint32_t b = (v >> k) & 1u;
            const uint64_t base = a.D[2 * j + b];
            const uint64_t dest = base + (sp_ < Zt ? Z0 + sp_ : O0 + (sp_ - Zt));
            if (dest < a.n) {
                out[dest] = (TOUT)v;
                lc.add(s.ct, a.next_cnt, (uint32_t)(dest >> a.next_shift), ((v >> kn) & 1u) ^ 1u);
            }
        }
    }
    lc.flush_wave(s.ct, a.next_cnt, lane);
    __syncthreads();
    count_flush(s.ct, a.next_cnt, tid);
}

}  // namespace wt
