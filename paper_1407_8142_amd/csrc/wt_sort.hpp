// sortWT on the GPU (section "sortWT"), a second construction of the same
// tree, independent of the level passes: level l of the tree is bit L-1-l
// of S stably sorted by its top l bits, so every level is built on its own
// and all levels run in the same launches (grid.y = level).  Byte symbols
// (L <= 8, at most 128 keys per level); per level l, key = x >> (L - l):
//   sort_count:   the count of each key per 16 KiB tile of S;
//   sort_scan:    per key, the exclusive prefix of its tile counts, plus the
//                 key's start C[key << (L - l)] in the sorted order;
//   sort_scatter: per tile, the stable rank of each element among the
//                 tile's elements of its key (each wave ranks its quarter in
//                 order: lanes holding the same key are found by a ballot
//                 per key bit, and a per-wave running count per key lives
//                 in LDS), then S_l[start + rank] = x;
//   sort_bits:    B_l from S_l, a bit word per thread from four 16-byte loads.
// The directories come from the standalone builder.  The paper finds sortWT
// slower than levelWT (it writes every level's sorted copy); here it serves
// as a cross-check of the level passes at any size.
#pragma once

#include "wt_kernels.hpp"

namespace wt {

constexpr int kSortTile = 16384;
constexpr int kSortKeys = 128;

__device__ __forceinline__ uint32_t sort_key(uint32_t x, uint32_t L, uint32_t l) {
    return (x >> (L - l)) & ((1u << l) - 1u);  // masked: a symbol >= 2^L (a rejected input) stays in range
}

__global__ __launch_bounds__(kBlock) void sort_count(const uint8_t *S, uint64_t n, uint32_t L, uint64_t T,
                                                     uint32_t *cnt) {
    __shared__ uint32_t h[kSortKeys];
    const uint32_t l = blockIdx.y, tile = blockIdx.x, tid = threadIdx.x;
    if (tid < kSortKeys) h[tid] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)tile * kSortTile;
    const uint32_t len = (uint32_t)min((uint64_t)kSortTile, n - t0);
    for (uint32_t p = 16u * tid; p < len; p += 16u * kBlock) {
        if (p + 16u <= len) {
            const uint4 v = *reinterpret_cast<const uint4 *>(S + t0 + p);
            const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int b = 0; b < 16; ++b) atomicAdd(&h[sort_key((dw[b >> 2] >> (8 * (b & 3))) & 0xFFu, L, l)], 1u);
        } else {
            for (uint32_t e = p; e < len; ++e) atomicAdd(&h[sort_key(S[t0 + e], L, l)], 1u);
        }
    }
    __syncthreads();
    if (tid < (1u << l)) cnt[((uint64_t)l * kSortKeys + tid) * T + tile] = h[tid];
}

__global__ __launch_bounds__(kBlock) void sort_scan(const uint32_t *cnt, const uint64_t *C, uint64_t sigma, uint32_t L,
                                                    uint64_t T, uint64_t *base) {
    __shared__ BlockScanTmp tmp;
    const uint32_t key = blockIdx.x, l = blockIdx.y;
    if (key >= (1u << l)) return;
    const uint64_t x = (uint64_t)key << (L - l);
    uint64_t carry = C[x < sigma ? x : sigma];
    const uint32_t *c = cnt + ((uint64_t)l * kSortKeys + key) * T;
    uint64_t *b = base + ((uint64_t)l * kSortKeys + key) * T;
    for (uint64_t c0 = 0; c0 < T; c0 += (uint64_t)kBlock * kItems) {
        const uint64_t i0 = c0 + (uint64_t)threadIdx.x * kItems;
        uint64_t v[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) v[j] = i0 + j < T ? c[i0 + j] : 0;
        uint64_t total;
        block_excl_scan(v, tmp, total);
#pragma unroll
        for (int j = 0; j < kItems; ++j)
            if (i0 + j < T) b[i0 + j] = carry + v[j];
        carry += total;
        __syncthreads();
    }
}

struct LdsSort {
    uint8_t x[kSortTile];
    uint16_t lr[kSortTile];           // rank among the same key in the wave's quarter
    uint32_t wc[kWaves][kSortKeys];   // per wave, elements of each key
    uint64_t tb[kSortKeys];           // this tile's start per key in S_l
};

__global__ __launch_bounds__(kBlock) void sort_scatter(const uint8_t *S, uint64_t n, uint32_t L, uint64_t T,
                                                       const uint64_t *base, uint8_t *out, uint64_t stride) {
    __shared__ LdsSort s;
    constexpr uint32_t kQuarter = kSortTile / kWaves;
    const uint32_t l = blockIdx.y, tile = blockIdx.x, tid = threadIdx.x, wave = tid / kWave;
    const int lane = lane_id();
    const uint64_t t0 = (uint64_t)tile * kSortTile;
    const uint32_t len = (uint32_t)min((uint64_t)kSortTile, n - t0);
    for (uint32_t e = tid; e < len; e += kBlock) s.x[e] = S[t0 + e];
    for (uint32_t i = tid; i < kWaves * kSortKeys; i += kBlock) s.wc[i / kSortKeys][i % kSortKeys] = 0;
    if (tid < (1u << l)) s.tb[tid] = base[((uint64_t)l * kSortKeys + tid) * T + tile];
    __syncthreads();
    // Each wave ranks its quarter in position order, 64 elements at a time.
    for (uint32_t it = 0; it < kQuarter / kWave; ++it) {
        const uint32_t e = wave * kQuarter + it * kWave + (uint32_t)lane;
        const bool valid = e < len;
        const uint32_t key = valid ? sort_key(s.x[e], L, l) : 0u;
        uint64_t peers = __ballot(valid);
        for (uint32_t b = 0; b < l; ++b) {
            const uint64_t bb = __ballot(valid && ((key >> b) & 1u));
            peers &= ((key >> b) & 1u) ? bb : ~bb;
        }
        if (!valid) peers = 0;
        const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt(lane));
        const uint32_t before = valid ? s.wc[wave][key] : 0u;
        if (valid) s.lr[e] = (uint16_t)(before + below);
        if (valid && below == 0) s.wc[wave][key] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    for (uint32_t e = tid; e < len; e += kBlock) {
        const uint32_t x = s.x[e], key = sort_key(x, L, l), w = e / kQuarter;
        uint32_t wb = 0;
        for (uint32_t v = 0; v < w; ++v) wb += s.wc[v][key];
        const uint64_t pos = s.tb[key] + wb + s.lr[e];
        if (pos < n) out[(uint64_t)l * stride + pos] = (uint8_t)x;
    }
}

// Thread t of the grid makes bit word t of level l from 64 sorted symbols:
// four 16-byte loads, the bit of four bytes at a time gathered by shifts and
// ORs.  The copy is padded to 256 bytes; bits past n are masked off.
__global__ __launch_bounds__(kBlock) void sort_bits(const uint8_t *Sl, uint64_t n, uint32_t L, uint64_t stride,
                                                    uint64_t *bits, uint64_t W) {
    const uint32_t l = blockIdx.y, k = L - 1 - l;
    const uint64_t w = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (w >= W) return;
    const uint4 *src = reinterpret_cast<const uint4 *>(Sl + (uint64_t)l * stride + (w << 6));
    uint64_t word = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 v = src[q];
        const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // bit k of byte i of dw[j] -> bit 4j + i of the 16-bit group
            uint32_t x = (dw[j] >> k) & 0x01010101u;
            x = (x | (x >> 7) | (x >> 14) | (x >> 21)) & 0xFu;
            word |= (uint64_t)x << (16 * q + 4 * j);
        }
    }
    const uint64_t rem = n - (w << 6);
    if (rem < 64) word &= (1ull << rem) - 1ull;
    bits[(uint64_t)l * W + w] = word;
}

}  // namespace wt
