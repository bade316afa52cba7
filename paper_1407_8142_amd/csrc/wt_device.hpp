// Device-side building blocks shared by the library's kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wt {

constexpr int kWave = 64;

// Tile-state words of the decoupled look-back scan (Merrill & Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back"): the status
// and the value share one 64-bit word, so a single relaxed agent-scope
// atomic carries both and no fence is needed.
constexpr uint64_t kStAgg = 1ull << 62;  // value = this tile's own total
constexpr uint64_t kStInc = 2ull << 62;  // value = inclusive prefix through this tile
constexpr uint64_t kStVal = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Valid elements of a group of k that starts at `start` in a range of `len`:
// min(k, len - start), and 0 when start >= len.  Computed in signed
// arithmetic (len, start < 2^31): the form `start >= len ? 0 : min(k, len -
// start)` has been compiled with the unsigned subtraction hoisted out of
// its guard and then used as if it could not wrap, which made every guard
// built on the count pass for groups past the end.
__device__ __forceinline__ uint32_t clamp_count(uint32_t len, uint32_t start, uint32_t k) {
    const int32_t rem = (int32_t)len - (int32_t)start;
    return (uint32_t)min(max(rem, 0), (int32_t)k);
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// Sum over the 64 lanes of a wave (all lanes active), in every lane: quad,
// half-row and row sums by DPP lane permutations, then rows 0+1 and 2+3
// through the row broadcasts, read from lane 63.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Position of the set bit of x with 0-based ordinal r (r < popcount(x)).
__device__ __forceinline__ uint32_t select_in_word(uint64_t x, uint32_t r) {
    uint32_t pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        uint64_t low = x & ((1ull << w) - 1ull);
        uint32_t c = (uint32_t)__popcll(low);
        if (r >= c) {
            r -= c;
            x >>= w;
            pos += (uint32_t)w;
        }
    }
    return pos;
}

// Decoupled look-back with fallback, run by one full wave.  Publishes `agg`
// for `tile` and returns the exclusive prefix (sum of the aggregates of all
// earlier tiles).  Each poll reads a window of 64*LBM predecessors (LBM
// loads in flight per lane), so a long run of tiles that have published
// only their aggregates costs few round trips.  Tile numbers are block
// indices, so nothing guarantees that an earlier tile's block has been
// scheduled: when the closest predecessor still missing has not published
// after `spin_limit` polls, the wave computes that tile's aggregate itself
// with `agg_of(tile)` (a pure function of the input) and counts it locally
// (Smith, Levien & Owens, "Decoupled Fallback: A Portable Single-Pass GPU
// Scan").  Every wait therefore ends, whatever the dispatch order, and the
// only words written are this tile's own (relaxed agent-scope stores).
template <int LBM, typename AggOf>
__device__ __forceinline__ uint64_t lookback_exclusive(uint64_t *state, uint64_t tile, uint64_t agg, int lane,
                                                       int spin_limit, AggOf agg_of) {
    constexpr int kWin = LBM * kWave;
    if (tile == 0) {
        if (lane == 0) st_relaxed(state, kStInc | agg);
        return 0;
    }
    if (lane == 0) st_relaxed(state + tile, kStAgg | agg);
    uint64_t excl = 0;
    int64_t base = (int64_t)tile - 1;  // closest predecessor not yet counted
    int spins = 0;
    for (;;) {
        uint64_t v[LBM];
#pragma unroll
        for (int m = 0; m < LBM; ++m) {
            int64_t idx = base - (m * kWave + lane);
            v[m] = idx >= 0 ? ld_relaxed(state + idx) : kStInc;  // "tile -1" is an empty inclusive prefix
        }
        int f = kWin, b = kWin;  // closest inclusive, closest missing (distance from base)
#pragma unroll
        for (int m = 0; m < LBM; ++m) {
            uint32_t st = (uint32_t)(v[m] >> 62);
            uint64_t inc = __ballot(st == 2u), bad = __ballot(st == 0u);
            if (f == kWin && inc) f = m * kWave + __ffsll((unsigned long long)inc) - 1;
            if (b == kWin && bad) b = m * kWave + __ffsll((unsigned long long)bad) - 1;
        }
        uint64_t part = 0;
        const int lim = b < f ? b : f + 1;  // count distances < lim
#pragma unroll
        for (int m = 0; m < LBM; ++m)
            if (m * kWave + lane < lim) part += v[m] & kStVal;
        excl += wave_sum_u64(part);
        if (b < f) {
            // Counted the ready aggregates before the missing tile; now wait
            // for it or reduce it here.
            base -= b;
            if (b > 0) {
                spins = 0;
            } else if (++spins >= spin_limit) {
                excl += agg_of((uint64_t)base);
                base -= 1;
                spins = 0;
            } else {
                __builtin_amdgcn_s_sleep(2);
            }
            continue;
        }
        if (f < kWin) break;
        base -= kWin;
    }
    if (lane == 0) st_relaxed(state + tile, kStInc | (excl + agg));
    return excl;
}

// Directory entries for one tile of up to 64*WPL level words, run by one
// wave; lane j holds words j*WPL .. j*WPL+WPL-1 (position order).
// zpre[m] = zeros before word m of the lane inside the tile, Z0 = zeros of
// the level before the tile, t0 = first position of the tile (a multiple of
// 4096), len = valid positions in the tile, n = level length (an ordinal
// >= n cannot exist, so it is never written).
template <int WPL>
__device__ __forceinline__ void emit_directories(const uint64_t (&word)[WPL], const uint32_t (&zpre)[WPL],
                                                 uint64_t Z0, uint64_t t0, uint32_t len, uint32_t Ztile,
                                                 uint64_t n, uint64_t *rank, uint64_t *sel1, uint64_t *sel0,
                                                 int lane) {
    constexpr uint64_t S = 4096;
    const uint64_t O0 = t0 - Z0;
    const uint32_t Otile = len - Ztile;
#pragma unroll
    for (int m = 0; m < WPL; ++m) {
        const uint32_t w = (uint32_t)lane * WPL + m;
        // rank[j] = ones before position 512 j (positions before the word are all valid).
        if (w * 64u < len && (w & 7u) == 0)
            rank[(t0 >> 9) + (w >> 3)] = (t0 + (uint64_t)w * 64u) - (Z0 + zpre[m]);
    }
    // Targets are counted by their offset inside the tile, so the loops run
    // at most Otile/S + 1 (resp. Ztile/S + 1) times whatever O0 and Z0 hold.
    for (uint64_t loc64 = (S - O0 % S) % S; loc64 < Otile; loc64 += S) {
        const uint32_t loc = (uint32_t)loc64;
        const uint64_t o = O0 + loc64;
#pragma unroll
        for (int m = 0; m < WPL; ++m) {
            const uint32_t w = (uint32_t)lane * WPL + m;
            const uint32_t opre = w * 64u - zpre[m];
            const uint32_t ow = w * 64u < len ? (uint32_t)__popcll(word[m]) : 0u;
            if (o < n && opre <= loc && loc < opre + ow)
                sel1[o / S] = t0 + (uint64_t)w * 64u + select_in_word(word[m], loc - opre);
        }
    }
    for (uint64_t loc64 = (S - Z0 % S) % S; loc64 < Ztile; loc64 += S) {
        const uint32_t loc = (uint32_t)loc64;
        const uint64_t o = Z0 + loc64;
#pragma unroll
        for (int m = 0; m < WPL; ++m) {
            const uint32_t w = (uint32_t)lane * WPL + m;
            const uint32_t nb = clamp_count(len, w * 64u, 64u);
            const uint64_t vmask = nb >= 64u ? ~0ull : ((1ull << nb) - 1ull);
            const uint64_t zword = ~word[m] & vmask;
            const uint32_t zw = (uint32_t)__popcll(zword);
            if (o < n && zpre[m] <= loc && loc < zpre[m] + zw)
                sel0[o / S] = t0 + (uint64_t)w * 64u + select_in_word(zword, loc - zpre[m]);
        }
    }
}

}  // namespace wt
