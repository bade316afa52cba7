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

// Decoupled look-back, run by one full wave.  Publishes `agg` for `tile`
// and returns the exclusive prefix (sum of the aggregates of all earlier
// tiles).  Tiles are numbered in the order blocks obtained them from an
// atomic ticket, so every tile this one waits on belongs to a block that is
// already running and publishes its aggregate without waiting itself.
__device__ __forceinline__ uint64_t lookback_exclusive(uint64_t *state, uint64_t tile, uint64_t agg,
                                                       int lane) {
    if (tile == 0) {
        if (lane == 0) st_relaxed(state, kStInc | agg);
        return 0;
    }
    if (lane == 0) st_relaxed(state + tile, kStAgg | agg);
    uint64_t excl = 0;
    int64_t base = (int64_t)tile - 1;
    for (;;) {
        int64_t idx = base - lane;
        uint64_t v = idx >= 0 ? ld_relaxed(state + idx) : kStInc;
        uint32_t st = (uint32_t)(v >> 62);
        uint64_t inc_mask = __ballot(st == 2u);
        uint64_t bad_mask = __ballot(st == 0u);
        int first_inc = inc_mask ? __ffsll((unsigned long long)inc_mask) - 1 : kWave;
        uint64_t need = first_inc >= kWave - 1 ? ~0ull : ((2ull << first_inc) - 1ull);
        if (bad_mask & need) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t val = lane <= first_inc ? (v & kStVal) : 0ull;
        excl += wave_sum_u64(val);
        if (first_inc < kWave) break;
        base -= kWave;
    }
    if (lane == 0) st_relaxed(state + tile, kStInc | (excl + agg));
    return excl;
}

// Directory entries for one tile of up to 64 level words, run by one wave
// (lane j holds word j of the tile).  zpre = zeros before word j inside the
// tile, Z0 = zeros of the level before the tile, t0 = first position of the
// tile (a multiple of 4096), len = valid positions in the tile, n = level
// length (an ordinal >= n cannot exist, so it is never written).
__device__ __forceinline__ void emit_directories(uint64_t word, uint32_t zpre, uint64_t Z0, uint64_t t0,
                                                 uint32_t len, uint32_t Ztile, uint64_t n, uint64_t *rank,
                                                 uint64_t *sel1, uint64_t *sel0, int lane) {
    const bool has = (uint32_t)lane * 64u < len;
    const uint32_t nb = has ? min(64u, len - (uint32_t)lane * 64u) : 0u;
    const uint64_t vmask = nb >= 64u ? ~0ull : ((1ull << nb) - 1ull);
    // rank[j] = ones before position 512 j (positions before the word are all valid).
    if (has && (lane & 7) == 0)
        rank[(t0 >> 9) + (uint64_t)(lane >> 3)] = (t0 + (uint64_t)lane * 64u) - (Z0 + zpre);
    const uint64_t O0 = t0 - Z0;
    const uint32_t Otile = len - Ztile;
    const uint32_t opre = (uint32_t)lane * 64u - zpre;
    const uint32_t ow = (uint32_t)__popcll(word);
    const uint64_t zword = ~word & vmask;
    const uint32_t zw = (uint32_t)__popcll(zword);
    constexpr uint64_t S = 4096;
    for (uint64_t o = (O0 + S - 1) / S * S; o < O0 + Otile; o += S) {
        uint32_t loc = (uint32_t)(o - O0);
        if (has && o < n && opre <= loc && loc < opre + ow)
            sel1[o / S] = t0 + (uint64_t)lane * 64u + select_in_word(word, loc - opre);
    }
    for (uint64_t o = (Z0 + S - 1) / S * S; o < Z0 + Ztile; o += S) {
        uint32_t loc = (uint32_t)(o - Z0);
        if (has && o < n && zpre <= loc && loc < zpre + zw)
            sel0[o / S] = t0 + (uint64_t)lane * 64u + select_in_word(zword, loc - zpre);
    }
}

}  // namespace wt
