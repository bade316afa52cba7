// Histogram of a wide alphabet (L > 16 levels, 32-bit symbols) in two
// phases that each read the sequence once, instead of one sliced pass that
// reads it once per 2^16 symbols of the alphabet.
//   coarse: with c = L - 16, levels 0..c-1 need C only at multiples of
//           2^(L-c), the starts of the 2^c groups of symbols sharing their
//           top c bits (node boundaries down to level c).  One pass counts
//           those groups (and checks the symbols, and counts the zeros of
//           the top bit per level-0 tile); one block turns the counts into
//           those entries of C.
//   fine:   after level c-1, S_c holds each group as one contiguous
//           segment [C[s 2^16], C[(s+1) 2^16]).  A block counts its share of
//           S_c, segment by segment, in 2^16 packed 16-bit LDS counters; the
//           first segment of the block becomes its row of counts, later
//           ones (a block crosses at most 2^c - 1 boundaries in all) go to
//           a count array by atomics.  Rows of one segment belong to
//           consecutive blocks, so one sum per symbol over those rows gives
//           every count.
#pragma once

#include "wt_kernels.hpp"

namespace wt {

constexpr uint32_t kCoarseMaxBits = 9;    // 2^c + 1 entries of C from one block of 1024 threads
constexpr uint32_t kCoarseTab = 2048;     // LDS words of the coarse table (replicas x (2^c + 1)): 8 KiB, 8 blocks per CU
constexpr uint32_t kFineBits = 16;        // symbols per segment: 2^16 packed counters = 128 KiB of LDS
constexpr int kFineThreads = 1024;
constexpr uint32_t kNoSeg = 0xFFFFFFFFu;

// Coarse pass over level-0 tiles (grid-stride): cnt0[tile] = zeros of the
// top bit in the tile; cc[g] += symbols whose top c bits are g; a symbol
// >= sigma sets the status.  Replica r of the LDS table serves the lanes
// with lane % reps == r (stride 2^c + 1: the replicas of one group fall in
// different banks).
template <typename T>
__global__ __launch_bounds__(kBlock) void hist_coarse(const T *__restrict__ S, uint64_t n, uint64_t sigma, uint32_t L,
                                                      uint32_t c, uint32_t reps, uint32_t tile_shift, uint64_t ntiles,
                                                      uint32_t *cnt0, unsigned long long *cc, uint32_t *status) {
    __shared__ uint32_t tab[kCoarseTab];
    __shared__ uint32_t s_red[kWaves];
    constexpr int V = 16 / sizeof(T);
    const int tid = threadIdx.x;
    const uint32_t ng = 1u << c, stride = ng + 1u, fb = L - c;
    for (uint32_t i = tid; i < reps * stride; i += kBlock) tab[i] = 0;
    __syncthreads();
    uint32_t *h = tab + (uint32_t)(lane_id() % reps) * stride;
    bool bad = false;
    auto one = [&](uint32_t x) -> uint32_t {
        const bool ok = x < sigma;
        bad |= !ok;
        atomicAdd(h + (ok ? (x >> fb) : ng), 1u);  // a rejected symbol goes to the spare slot ng
        return ((x >> (L - 1u)) & 1u) ^ 1u;
    };
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t base = tile << tile_shift;
        const uint32_t len = (uint32_t)min(1ull << tile_shift, n - base);
        const uint32_t nvec = len / V;
        const uint4 *src = reinterpret_cast<const uint4 *>(S + base);
        uint32_t zeros = 0;
        constexpr int kU = 4;
        for (uint32_t v0 = tid; v0 < nvec; v0 += kBlock * kU) {
            uint4 q[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) q[u] = v0 + u * kBlock < nvec ? src[v0 + u * kBlock] : make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (v0 + u * kBlock >= nvec) break;
                union {
                    uint4 q;
                    T e[V];
                } w;
                w.q = q[u];
#pragma unroll
                for (int e = 0; e < V; ++e) zeros += one((uint32_t)w.e[e]);
            }
        }
        for (uint32_t e = nvec * V + tid; e < len; e += kBlock) zeros += one((uint32_t)S[base + e]);
        const uint32_t t = block_sum_u32(zeros, s_red);
        if (tid == 0) cnt0[tile] = t;
    }
    if (__ballot(bad) && lane_id() == 0) atomicMax(status, kStatusSymbol);
    __syncthreads();
    for (uint32_t g = tid; g < ng; g += kBlock) {
        uint32_t sum = 0;
        for (uint32_t r = 0; r < reps; ++r) sum += tab[r * stride + g];
        if (sum) atomicAdd(cc + g, (unsigned long long)sum);
    }
}

// C[min(g 2^(L-c), sigma)] = symbols of the groups before g, g = 0..2^c
// (one block of 1024 threads; c <= kCoarseMaxBits).  Groups at or past
// sigma are empty, so every g that lands on C[sigma] writes the same total.
__global__ __launch_bounds__(1024) void coarse_to_C(const unsigned long long *cc, uint32_t c, uint32_t L,
                                                    uint64_t sigma, uint64_t *C) {
    __shared__ uint64_t s[1024];
    const uint32_t t = threadIdx.x, ng = 1u << c;
    s[t] = t < ng ? (uint64_t)cc[t] : 0ull;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint64_t v = t >= off ? s[t - off] : 0ull;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    if (t <= ng) {
        const uint64_t x = (uint64_t)t << (L - c);
        C[x < sigma ? x : sigma] = t ? s[t - 1] : 0ull;
    }
}

// Fine pass: block b counts positions [b per, (b+1) per) of S_c (32-bit
// symbols), piece by piece, one piece per segment it meets.  Segment s
// starts at C[min(s 2^16, sigma)] (entries the coarse phase wrote, or the
// full C: the same values).  A packed counter that reaches 2^15 hands 2^15
// to extra[] (the thread whose add crossed the mark does it).
__global__ __launch_bounds__(kFineThreads) void hist_fine(const uint32_t *__restrict__ S, uint64_t n, uint64_t sigma,
                                                          uint32_t c, const uint64_t *C, uint64_t per,
                                                          uint32_t *rows, uint32_t *tags, unsigned long long *extra,
                                                          const uint32_t *status) {
    __shared__ uint32_t bins[1u << (kFineBits - 1)];
    __shared__ uint32_t s_first;
    const uint32_t b = blockIdx.x, tid = threadIdx.x;
    const uint64_t lo = min(n, (uint64_t)b * per), hi = min(n, lo + per);
    const uint32_t nseg = 1u << c;
    constexpr uint32_t kMask = (1u << kFineBits) - 1u;
    auto bound = [&](uint32_t s) -> uint64_t {
        const uint64_t x = (uint64_t)s << kFineBits;
        return C[x < sigma ? x : sigma];
    };
    if (*status || lo >= hi) {  // a rejected input leaves C unused; an empty share has no row
        if (tid == 0) tags[b] = kNoSeg;
        return;
    }
    if (tid == 0) {  // the segment holding lo: the last s with bound(s) <= lo
        uint32_t a = 0, e = nseg - 1u;
        while (a < e) {
            const uint32_t m = (a + e + 1u) >> 1;
            if (bound(m) <= lo) a = m;
            else e = m - 1u;
        }
        s_first = a;
        tags[b] = a;
    }
    __syncthreads();
    const uint32_t s0 = s_first;
    for (uint32_t s = s0; s < nseg; ++s) {
        const uint64_t sb = bound(s), se = s + 1u < nseg ? bound(s + 1u) : n;
        if (sb >= hi) break;
        const uint64_t a = max(lo, sb), e = min(hi, se);
        if (a >= e) continue;
        for (uint32_t i = tid; i < (1u << (kFineBits - 1)); i += kFineThreads) bins[i] = 0;
        __syncthreads();
        const uint64_t sym0 = (uint64_t)s << kFineBits;
        auto one = [&](uint32_t x) {
            const uint32_t v = x & kMask, hb = v & 1u, inc = hb ? 0x10000u : 1u;
            const uint32_t old = atomicAdd(bins + (v >> 1), inc);
            if (((old >> (16u * hb)) & 0xFFFFu) == 0x7FFFu) {
                atomicSub(bins + (v >> 1), inc << 15);
                atomicAdd(extra + sym0 + v, 0x8000ull);
            }
        };
        // Head up to a 16-byte boundary, 16-byte body, tail.
        const uint64_t a4 = min(e, align_up(a, 4)), e4 = max(a4, e & ~3ull);
        for (uint64_t i = a + tid; i < a4; i += kFineThreads) one(S[i]);
        const uint4 *src = reinterpret_cast<const uint4 *>(S + a4);
        const uint64_t nv = (e4 - a4) / 4;
        constexpr int kU = 4;
        for (uint64_t v0 = tid; v0 < nv; v0 += (uint64_t)kFineThreads * kU) {
            uint4 q[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint64_t vi = v0 + (uint64_t)u * kFineThreads;
                q[u] = vi < nv ? src[vi] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (v0 + (uint64_t)u * kFineThreads >= nv) break;
                one(q[u].x);
                one(q[u].y);
                one(q[u].z);
                one(q[u].w);
            }
        }
        for (uint64_t i = e4 + tid; i < e; i += kFineThreads) one(S[i]);
        __syncthreads();
        if (s == s0) {
            uint32_t *row = rows + (uint64_t)b * (1u << kFineBits);
            for (uint32_t i = tid; i < (1u << kFineBits); i += kFineThreads) row[i] = (bins[i >> 1] >> (16u * (i & 1u))) & 0xFFFFu;
        } else {
            const uint32_t nb = (uint32_t)min((uint64_t)1u << kFineBits, sigma - sym0);
            for (uint32_t i = tid; i < nb; i += kFineThreads) {
                const uint32_t v = (bins[i >> 1] >> (16u * (i & 1u))) & 0xFFFFu;
                if (v) atomicAdd(extra + sym0 + i, (unsigned long long)v);
            }
        }
        __syncthreads();
    }
}

// Cp1[x] = extra[x] + the rows of the blocks whose first segment holds x
// (consecutive blocks: tags never decrease, kNoSeg ones come last).
__global__ __launch_bounds__(kBlock) void hist_fine_reduce(const uint32_t *__restrict__ rows, const uint32_t *tags,
                                                           uint32_t nblocks, const unsigned long long *extra,
                                                           uint64_t sigma, uint64_t *Cp1) {
    __shared__ uint32_t s_tags[1024];
    for (uint32_t i = threadIdx.x; i < nblocks; i += kBlock) s_tags[i] = tags[i];
    __syncthreads();
    auto lower = [&](uint32_t key) -> uint32_t {  // first block with tag >= key
        uint32_t a = 0, e = nblocks;
        while (a < e) {
            const uint32_t m = (a + e) >> 1;
            if (s_tags[m] < key) a = m + 1u;
            else e = m;
        }
        return a;
    };
    for (uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x; x < sigma; x += (uint64_t)gridDim.x * kBlock) {
        const uint32_t s = (uint32_t)(x >> kFineBits), v = (uint32_t)x & ((1u << kFineBits) - 1u);
        const uint32_t b0 = lower(s), b1 = lower(s + 1u);
        uint64_t t = extra[x];
        for (uint32_t bb = b0; bb < b1; ++bb) t += rows[(uint64_t)bb * (1u << kFineBits) + v];
        Cp1[x] = t;
    }
}

}  // namespace wt
