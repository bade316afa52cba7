// Wavelet-tree construction on gfx950: levelWT (Fig. 1 of "Parallel Wavelet
// Tree Construction") as one HBM pass per level, plus rank/select directories.
//
// Pipeline of wt_build on one stream:
//   zero_fill      status word, look-back tile states, C
//   histogram      counts of every symbol into C[1..sigma] and the symbol check
//   scan (C)       C[c] = #{S[i] < c}, a device-wide prefix sum
//   node tables    per level l and node p: D_l[2p] = ones of B_l before node p,
//                  D_l[2p+1] = zeros of B_l before node p+1 (from C alone)
//   level_pass x L one kernel per level: bit extraction into B_l (wave
//                  ballots), zero-count scan with decoupled look-back, stable
//                  split of every node (Fig. 1 left/right offsets) staged in
//                  LDS and scattered to S_{l+1}; optionally the directory
//                  entries of B_l; the last level writes bits only.
//   dir_finish     per-level directory tails and counts (from the tables)
//
// Node offsets come from C rather than from Fig. 1's node list: the node of
// a symbol at level l is its top l bits (the observation behind sortWT and
// FEFS), so every node boundary of every level is known once C is known.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/wt.h"
#include "wt_device.hpp"
#include "wt_kernels.hpp"
#include "wt_pair.hpp"
#include "wt_quad.hpp"
#include "wt_hist2.hpp"
#include "wt_huff.hpp"
#include "wt_sort.hpp"
#include "wt_stats.hpp"
#include "wt_sparse.hpp"
#include "wt_u16.hpp"
#include "wt_u32.hpp"

namespace wt {

constexpr int kDirTile = 4096;  // bits per tile of the standalone directory builder

// ---------------------------------------------------------------------------
// zero_fill: clears up to two word ranges.
__global__ void zero_fill(uint64_t *a, uint64_t na, uint64_t *b, uint64_t nb) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
        if (i < na) a[i] = 0;
        else b[i - na] = 0;
    }
}

// ---------------------------------------------------------------------------
// histogram: counts into Cp1[c] = C[c+1] (zeroed), the symbol check, and the
// zeros of the top bit per level-0 tile.  Blocks take whole tiles of level 0
// (grid-stride); the LDS table (replicas or hash, see hist_count) lives
// across the block's tiles and is flushed once at the end.
// With DIG, the per-tile output is the packed counts of the top two bits'
// digit (the prefixes a first pass over two levels needs) instead of the
// zeros of the top bit.
// Byte symbols with LDS replicas (the common case): every byte is one LDS
// add (its result unused) into its lane's replica, and the zeros of the top
// bit (or the digit counts) are tallied by SWAR over the sixteen bytes of a
// load, fewer instructions per byte than merging runs.  The four loads of a
// thread's share of a whole tile are issued together; a ragged tile end is
// counted byte by byte.
// CHECK: sigma < 256, so a byte can be out of range (then it is counted in
// the spare bin sigma and flagged).
template <bool DIG, bool CHECK>
__device__ __forceinline__ std::conditional_t<DIG, uint64_t, uint32_t> hist_count_u8(
    const uint8_t *__restrict__ S, uint64_t base, uint32_t len, uint64_t sigma, uint32_t reps, uint32_t ktop,
    uint32_t *tab, bool &bad) {
    const int tid = threadIdx.x;
    uint32_t *h = tab + (uint32_t)(lane_id() % reps) * (uint32_t)(sigma + 1);
    const uint32_t smax = (uint32_t)sigma;
    std::conditional_t<DIG, uint64_t, uint32_t> acc = 0;
    auto one = [&](uint32_t x) {
        if constexpr (CHECK) {
            bad |= x >= smax;
            x = min(x, smax);
        }
        atomicAdd(h + x, 1u);
    };
    auto count16 = [&](const uint4 &q) {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int b = 0; b < 4; ++b) one((w[i] >> (8 * b)) & 0xFFu);
        if constexpr (DIG) acc += digit_inc16(q, ktop - 1u);
        else acc += zeros16(q, ktop);
    };
    const uint4 *src = reinterpret_cast<const uint4 *>(S + base);
    const uint32_t nvec = len / 16;
    constexpr int kU = 4;
    for (uint32_t v0 = tid; v0 < nvec; v0 += kBlock * kU) {
        uint4 q[kU];
        if (v0 + (uint32_t)((kU - 1) * kBlock) < nvec) {
#pragma unroll
            for (int k = 0; k < kU; ++k) q[k] = src[v0 + k * kBlock];
#pragma unroll
            for (int k = 0; k < kU; ++k) count16(q[k]);
        } else {
            for (uint32_t v = v0; v < nvec; v += kBlock) count16(src[v]);
        }
    }
    for (uint32_t e = nvec * 16 + tid; e < len; e += kBlock) {
        const uint32_t x = S[base + e];
        one(x);
        if constexpr (DIG) acc += digit_inc(x, ktop - 1u);
        else acc += ((x >> ktop) & 1u) ^ 1u;
    }
    return acc;
}

template <typename T, bool DIG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void histogram(const T *__restrict__ S, uint64_t n, uint64_t sigma,
                                                    unsigned long long *Cp1, uint32_t *status, uint32_t reps,
                                                    uint32_t ktop, void *cnt0, uint32_t tile_shift,
                                                    uint64_t ntiles) {
    constexpr uint32_t kH = 4096;
    extern __shared__ uint32_t s_dyn[];
    __shared__ uint64_t s_red[kWaves];
    __shared__ uint32_t s_nused;
    hist_init<kH>(s_dyn, &s_nused, reps, sigma);
    bool bad = false;
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t base = tile << tile_shift;
        const uint32_t len = (uint32_t)min(1ull << tile_shift, n - base);
        std::conditional_t<DIG, uint64_t, uint32_t> zeros;
        if constexpr (sizeof(T) == 1) {
            const uint8_t *S8 = reinterpret_cast<const uint8_t *>(S);
            if (!reps)
                zeros = hist_count<T, kH, unsigned long long, DIG>(S, base, len, sigma, reps, ktop, s_dyn, &s_nused,
                                                                   Cp1, bad);
            else if (sigma < 256)
                zeros = hist_count_u8<DIG, true>(S8, base, len, sigma, reps, ktop, s_dyn, bad);
            else
                zeros = hist_count_u8<DIG, false>(S8, base, len, sigma, reps, ktop, s_dyn, bad);
        } else {
            zeros = hist_count<T, kH, unsigned long long, DIG>(S, base, len, sigma, reps, ktop, s_dyn, &s_nused, Cp1,
                                                               bad);
        }
        if (cnt0) {
            if constexpr (DIG) {
                const uint64_t t = block_sum_u64(zeros, s_red);
                if (threadIdx.x == 0) reinterpret_cast<uint64_t *>(cnt0)[tile] = t;
            } else {
                const uint32_t t = block_sum_u32(zeros, reinterpret_cast<uint32_t *>(s_red));
                if (threadIdx.x == 0) reinterpret_cast<uint32_t *>(cnt0)[tile] = t;
            }
        }
    }
    if (__ballot(bad) && lane_id() == 0) atomicMax(status, kStatusSymbol);
    if (reps) hist_flush_replicas(s_dyn, reps, sigma, Cp1);
}


// Wide alphabets (sigma > 8192): block (chunk, slice) counts, over a chunk
// of whole level-0 tiles, the symbols of slice [slice*2^16, slice*2^16+2^16)
// in packed 16-bit LDS counters (128 KiB: one block per CU, 16 waves), then
// stores them as its row of `part` (chunk-major, sigma entries per row).  A
// counter that reaches 2^15 hands 2^15 to Cp1 (the thread whose add crossed
// the mark does it, so a half never carries into its neighbour).  Every
// slice of one chunk has the same blockIdx % 8 and so runs on one XCD:
// after the first of them fetched a tile, the others read it from that
// XCD's L2.  Slice 0 also checks the symbols and counts the zeros of the top
// bit per tile.
constexpr int kSliceThreads = 1024;
constexpr uint32_t kSliceBins = 1u << 16;
constexpr int kSliceUnroll = 4;  // tiles loaded before counting

template <typename T>
__global__ __launch_bounds__(kSliceThreads) void hist_slices(const T *__restrict__ S, uint64_t n, uint64_t sigma,
                                                             uint32_t nslices, uint64_t nchunks,
                                                             uint64_t tiles_per_chunk, uint32_t tile_shift,
                                                             uint32_t ktop, uint32_t *cnt0,
                                                             unsigned long long *Cp1, uint32_t *part,
                                                             uint32_t *status) {
    __shared__ uint32_t bins[kSliceBins / 2];
    __shared__ uint32_t red[2][kSliceUnroll][kSliceThreads / kWave];
    constexpr int V = 16 / sizeof(T);
    static_assert(kSliceThreads * 16 == 16384, "one 16-byte load per thread covers a level-0 tile");
    const uint32_t per = 8u * nslices;
    const uint64_t chunk = (uint64_t)(blockIdx.x / per) * 8u + blockIdx.x % 8u;
    const uint32_t slice = (blockIdx.x % per) / 8u;
    if (chunk >= nchunks) return;  // the grid is padded to whole groups of 8 chunks
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    for (int i = tid; i < (int)(kSliceBins / 2); i += kSliceThreads) bins[i] = 0;
    __syncthreads();
    const uint32_t lo = slice * kSliceBins;
    const bool lead = slice == 0;
    bool bad = false;
    auto count = [&](uint32_t x) -> uint32_t {
        bad |= x >= sigma;
        const uint32_t r = x - lo;  // below the slice: wraps past kSliceBins
        if (r < kSliceBins && x < sigma) {
            const uint32_t hi = r & 1u, inc = hi ? 0x10000u : 1u;
            const uint32_t old = atomicAdd(bins + (r >> 1), inc);
            if (((old >> (16 * hi)) & 0xFFFFu) == 0x7FFFu) {
                atomicSub(bins + (r >> 1), inc << 15);
                atomicAdd(Cp1 + x, 0x8000ull);
            }
        }
        return ((x >> ktop) & 1u) ^ 1u;
    };
    const uint64_t ntiles = cdiv(n, 1ull << tile_shift);
    const uint64_t t0 = chunk * tiles_per_chunk;
    const uint64_t t1 = min(ntiles, t0 + tiles_per_chunk);
    uint32_t buf = 0;
    for (uint64_t g = t0; g < t1; g += kSliceUnroll) {
        uint4 q[kSliceUnroll];
        uint32_t z[kSliceUnroll];
        if (g + kSliceUnroll <= t1 && ((g + kSliceUnroll) << tile_shift) <= n) {
            // all whole tiles: no branch between the loads, so they overlap
#pragma unroll
            for (int u = 0; u < kSliceUnroll; ++u) q[u] = reinterpret_cast<const uint4 *>(S + ((g + u) << tile_shift))[tid];
        } else {
#pragma unroll
            for (int u = 0; u < kSliceUnroll; ++u) {
                const uint64_t base = (g + u) << tile_shift;
                q[u] = make_uint4(0, 0, 0, 0);
                if (g + u < t1 && base + (1ull << tile_shift) <= n)
                    q[u] = reinterpret_cast<const uint4 *>(S + base)[tid];
            }
        }
#pragma unroll
        for (int u = 0; u < kSliceUnroll; ++u) {
            z[u] = 0;
            const uint64_t base = (g + u) << tile_shift;
            if (g + u >= t1) continue;
            if (base + (1ull << tile_shift) <= n) {
                union {
                    uint4 q;
                    T e[V];
                } v;
                v.q = q[u];
#pragma unroll
                for (int e = 0; e < V; ++e) z[u] += count((uint32_t)v.e[e]);
            } else {  // the last, partial tile of the input
                const uint32_t len = (uint32_t)(n - base);
                for (uint32_t e = tid; e < len; e += kSliceThreads) z[u] += count((uint32_t)S[base + e]);
            }
        }
        if (lead && cnt0) {
#pragma unroll
            for (int u = 0; u < kSliceUnroll; ++u) {
                const uint32_t w = (uint32_t)wave_sum_u64(z[u]);
                if (lane == 0) red[buf][u][wave] = w;
            }
            __syncthreads();
            if (tid < kSliceUnroll && g + tid < t1) {
                uint32_t t = 0;
#pragma unroll
                for (int w = 0; w < kSliceThreads / kWave; ++w) t += red[buf][tid][w];
                cnt0[g + tid] = t;
            }
            buf ^= 1u;  // the next group writes the other half: one barrier per group suffices
        }
    }
    if (__ballot(bad) && lane == 0) atomicMax(status, kStatusSymbol);
    __syncthreads();
    const uint64_t row = chunk * sigma + lo;
    const uint32_t nb = (uint32_t)min((uint64_t)kSliceBins, sigma - lo);
    for (uint32_t i = tid; i < nb; i += kSliceThreads) part[row + i] = (bins[i >> 1] >> (16 * (i & 1))) & 0xFFFFu;
}

// Cp1[c] += sum of the chunk rows of `part` at c.  Group blockIdx.y of
// gridDim.y sums its share of the rows and adds it atomically (Cp1 already
// holds the counters' overflow hand-overs), so many rows are summed by many
// threads at once.
__global__ __launch_bounds__(kBlock) void hist_reduce(const uint32_t *__restrict__ part, uint64_t nchunks,
                                                      uint64_t sigma, uint64_t *Cp1) {
    const uint64_t per = cdiv(nchunks, gridDim.y), k0 = blockIdx.y * per, k1 = min(nchunks, k0 + per);
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c < sigma; c += (uint64_t)gridDim.x * kBlock) {
        uint64_t t = 0;
        for (uint64_t k = k0; k < k1; ++k) t += part[k * sigma + c];
        if (t) atomicAdd((unsigned long long *)(Cp1 + c), (unsigned long long)t);
    }
}


// Exclusive prefix of per-tile zero counts (one block of 1024 threads, 16
// counts per thread; `cnt` and `pre` are 64-entry aligned).
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void tile_prefix_scan(const uint32_t *cnt, uint64_t *pre, uint64_t T) {
    __shared__ uint32_t s_w[kScanThreads / kWave];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    uint64_t carry = 0;
    for (uint64_t c0 = 0; c0 < T; c0 += (uint64_t)kScanThreads * 16) {
        const uint64_t base = c0 + (uint64_t)tid * 16;
        uint32_t v[16], own = 0;
        if (base + 16 <= T) {
            const uint4 *p4 = reinterpret_cast<const uint4 *>(cnt + base);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 x = p4[q];
                v[4 * q] = x.x;
                v[4 * q + 1] = x.y;
                v[4 * q + 2] = x.z;
                v[4 * q + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = base + j < T ? cnt[base + j] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) own += v[j];
        const uint32_t inc = wave_incl_scan_u32(own, lane);
        if (lane == kWave - 1) s_w[wave] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kScanThreads / kWave; ++w) {
            const uint32_t x = s_w[w];
            before += w < wave ? x : 0u;
            total += x;
        }
        uint64_t run = carry + before + inc - own;
        uint64_t o[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            o[j] = run;
            run += v[j];
        }
        if (base + 16 <= T) {
            ulonglong2 *q2 = reinterpret_cast<ulonglong2 *>(pre + base);
#pragma unroll
            for (int q = 0; q < 8; ++q) q2[q] = make_ulonglong2(o[2 * q], o[2 * q + 1]);
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (base + j < T) pre[base + j] = o[j];
        }
        carry += total;
        __syncthreads();
    }
}

// The same prefix over many tiles in one pass of several blocks: block b
// scans counts [4096 b, 4096 b + 4096) and takes the zeros before them from
// its predecessors' published totals (decoupled look-back with fallback;
// `state` holds one word per block and is zeroed with the counts).
constexpr int kTpItems = 16, kTpSpan = kBlock * kTpItems;  // tiles per block
__global__ __launch_bounds__(kBlock) void tile_prefix_multi(const uint32_t *cnt, uint64_t *pre, uint64_t T,
                                                            uint64_t *state, int spin_limit) {
    __shared__ uint32_t s_w[kWaves];
    __shared__ uint64_t s_excl;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint64_t blk = blockIdx.x, base = blk * kTpSpan + (uint64_t)tid * kTpItems;
    uint32_t v[kTpItems], own = 0;
    if (base + kTpItems <= T) {
        const uint4 *p4 = reinterpret_cast<const uint4 *>(cnt + base);
#pragma unroll
        for (int q = 0; q < kTpItems / 4; ++q) {
            const uint4 x = p4[q];
            v[4 * q] = x.x;
            v[4 * q + 1] = x.y;
            v[4 * q + 2] = x.z;
            v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kTpItems; ++j) v[j] = base + j < T ? cnt[base + j] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kTpItems; ++j) own += v[j];
    const uint32_t inc = wave_incl_scan_u32(own, lane);
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t x = s_w[w];
        before += w < wave ? x : 0u;
        total += x;
    }
    if (wave == 0) {
        auto agg_of = [&](uint64_t b) -> uint64_t {  // a predecessor's total, recounted
            uint64_t t = 0;
            for (uint64_t i = b * kTpSpan + lane; i < min((b + 1) * kTpSpan, T); i += kWave) t += cnt[i];
            return wave_sum_u64(t);
        };
        const uint64_t ex = lookback_exclusive<1>(state, blk, total, lane, spin_limit, agg_of);
        if (lane == 0) s_excl = ex;
    }
    __syncthreads();
    uint64_t run = s_excl + before + inc - own;
    uint64_t o[kTpItems];
#pragma unroll
    for (int j = 0; j < kTpItems; ++j) {
        o[j] = run;
        run += v[j];
    }
    if (base + kTpItems <= T) {
        ulonglong2 *q2 = reinterpret_cast<ulonglong2 *>(pre + base);
#pragma unroll
        for (int q = 0; q < kTpItems / 2; ++q) q2[q] = make_ulonglong2(o[2 * q], o[2 * q + 1]);
    } else {
#pragma unroll
        for (int j = 0; j < kTpItems; ++j)
            if (base + j < T) pre[base + j] = o[j];
    }
}

// Generic reduce-then-scan over values produced by a functor, cut into
// chunks of kScanChunk elements; exclusive sums restart at segment heads
// (the node tables use one segment per level).
//   F::value(g)            value of element g
//   F::store(g, excl)      consume the exclusive prefix of element g
//   F::seg_start(g)        first element of g's segment
//   F::chunk_seg_first(c)  first chunk of the segment that chunk c continues;
//                          a segment either starts inside a chunk (and then
//                          ends inside it too) or starts on a chunk boundary
template <typename F>
__global__ __launch_bounds__(kBlock) void scan_reduce(F f, uint64_t count, uint64_t *partials) {
    __shared__ BlockScanTmp tmp;
    const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kItems;
    uint64_t v[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) v[j] = base + j < count ? f.value(base + j) : 0;
    uint64_t total;
    block_excl_scan(v, tmp, total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

template <typename F>
__global__ __launch_bounds__(kBlock) void scan_final(F f, uint64_t count, const uint64_t *partials) {
    __shared__ BlockScanTmp tmp;
    __shared__ uint64_t s_ex[kScanChunk];
    const uint64_t chunk = blockIdx.x;
    const uint64_t cbase = chunk * kScanChunk;
    const uint64_t base = cbase + (uint64_t)threadIdx.x * kItems;
    uint64_t v[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) v[j] = base + j < count ? f.value(base + j) : 0;
    uint64_t total;
    block_excl_scan(v, tmp, total);
    // Exclusive prefix of the chunk inside its segment.
    uint64_t chunk_off = 0;
    if (partials) {
        uint64_t first = f.chunk_seg_first(chunk);
        chunk_off = partials[chunk] - partials[first];
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) s_ex[threadIdx.x * kItems + j] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        uint64_t g = base + j;
        if (g >= count) continue;
        uint64_t h = f.seg_start(g);
        uint64_t ex = h >= cbase ? v[j] - s_ex[h - cbase] : v[j] + chunk_off;
        f.store(g, ex);
    }
}

// C scan: values are counts held in Cp1[c] (= C[c+1]); stores inclusive sums.
struct CScanOp {
    uint64_t *Cp1;
    __device__ uint64_t value(uint64_t g) const { return Cp1[g]; }
    __device__ void store(uint64_t g, uint64_t ex) const { Cp1[g] = ex + Cp1[g]; }
    __device__ uint64_t seg_start(uint64_t) const { return 0; }
    __device__ uint64_t chunk_seg_first(uint64_t) const { return 0; }
};

// Exclusive scan of chunk partials restarting at chunk_seg_first; single block.
template <typename F>
__global__ __launch_bounds__(kBlock) void scan_partials_seg(F f, uint64_t nchunks, uint64_t *partials) {
    // Partials become "exclusive prefix from the first chunk of the whole
    // array"; scan_final subtracts partials[first chunk of the segment].
    __shared__ BlockScanTmp tmp;
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint64_t c0 = 0; c0 < nchunks; c0 += kScanChunk) {
        const uint64_t base = c0 + (uint64_t)threadIdx.x * kItems;
        uint64_t v[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) v[j] = base + j < nchunks ? partials[base + j] : 0;
        uint64_t total;
        block_excl_scan(v, tmp, total);
        uint64_t carry = s_carry;
#pragma unroll
        for (int j = 0; j < kItems; ++j)
            if (base + j < nchunks) partials[base + j] = carry + v[j];
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + total;
        __syncthreads();
    }
    (void)f;
}

// ---------------------------------------------------------------------------
// Level pass kernels: one block per tile of the level.
template <typename TIN, typename TOUT, bool SCATTER, bool DIRS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void level_pass(LevelArgs a) {
    __shared__ LdsLevel<TIN> s;
    level_tile<TIN, TOUT, SCATTER, DIRS>(a, blockIdx.x, s);
}

template <bool SCATTER, bool DIRS, bool PIECES = false, bool LASTBITS = false>
__global__ __launch_bounds__(kBlock) void level_pass_u8(LevelArgs a) {
    __shared__ LdsLevelU8 s;
    level_tile_u8<SCATTER, DIRS, PIECES, LASTBITS>(a, blockIdx.x, s);
}

constexpr int kDirsWaves = 4;  // tiles (one per wave) per block of level_dirs

__global__ __launch_bounds__(kDirsWaves * kWave) void level_dirs(LevelArgs a) {
    __shared__ uint64_t s_cl[kStatsMaxNodes + 1];
    for (uint32_t i = threadIdx.x; i < a.nodes; i += kDirsWaves * kWave) s_cl[i] = a.node_starts[i];
    __syncthreads();
    const uint64_t ntiles = cdiv(a.n, 16384);
    const uint64_t tile = (uint64_t)blockIdx.x * kDirsWaves + threadIdx.x / kWave;
    if (tile < ntiles) level_dirs_tile(a, tile, ntiles, s_cl);
}

template <bool SCATTER, bool DIRS>
__global__ __launch_bounds__(kBlock) void level_pass_u16(LevelArgs a) {
    __shared__ LdsLevelU16 s;
    level_tile_u16<SCATTER, DIRS>(a, blockIdx.x, s);
}

template <typename TOUT, bool SCATTER, bool DIRS>
__global__ __launch_bounds__(kBlock) void level_pass_u32(LevelArgs a) {
    __shared__ LdsLevelU32 s;
    level_tile_u32<TOUT, SCATTER, DIRS>(a, blockIdx.x, s);
}


// ---------------------------------------------------------------------------
// Fused tail levels (see fused_segment): the largest node of every level,
// the first fused level, and the fused pass itself (segments strided over a
// grid that exits at once when no level is fused).
constexpr int kFusedBytes = 16384;

__global__ __launch_bounds__(kBlock) void node_max_kernel(const uint64_t *C, uint64_t sigma, uint32_t L,
                                                          unsigned long long *maxnode) {
    __shared__ unsigned long long red[32];
    if (threadIdx.x < 32) red[threadIdx.x] = 0;
    __syncthreads();
    // Levels 0..L-2: fusion starts at L-2 at the latest.
    node_max_range(C, sigma, L, 1 + (uint64_t)blockIdx.x * kBlock, 1ull << (L - 1), (uint64_t)gridDim.x * kBlock,
                   red, maxnode);
}

__global__ void fuse_plan_kernel(const unsigned long long *maxnode, uint32_t L, uint64_t half, uint32_t most,
                                 uint32_t *l0) {
    if (threadIdx.x == 0) *l0 = fused_from(reinterpret_cast<const uint64_t *>(maxnode), L, half, most);
}

template <typename TIN0, typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void fused_pass(FusedArgs f, uint64_t nseg) {
    __shared__ LdsFused<T, kFusedBytes> s;
    if (*f.l0 >= f.L) return;  // the plan found no level to fuse
    for (uint64_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        fused_segment<TIN0, T, kFusedBytes>(f, seg, s);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Two levels per pass (byte alphabets, see pair_tile_u8).
constexpr uint64_t kPairTableBytes = 4 * 256 * 4;  // E_l of the pairs at l = 0, 2, 4, 6

template <bool SCATTER, bool NEXT_PAIR, bool DIRS>
__global__ __launch_bounds__(kBlock) void pair_pass(PairArgs a) {
    __shared__ LdsPair s;
    pair_tile_u8<SCATTER, NEXT_PAIR, DIRS>(a, blockIdx.x, s);
}

// E[4p+d] = C[(4p+d) << shift] - (symbols of digit d, bits [shift, shift+2),
// in the nodes before p) for the digit level j = blockIdx.x, shift = shift0 -
// 2j, 4^(j+1) entries at E + 256 j: the destinations of a split by two bits
// (pairs of binary levels from level 2j, or the levels of the 4-ary tree).
__global__ __launch_bounds__(kBlock) void digit_tables(const uint64_t *C, uint64_t sigma, uint32_t shift0,
                                                       uint32_t *E) {
    const uint32_t j = blockIdx.x, shift = shift0 - 2u * j;
    uint32_t *Ej = E + 256u * j;
    auto Cc = [&](uint64_t x) { return C[x < sigma ? x : sigma]; };
    for (uint32_t t = threadIdx.x; t < (4u << (2u * j)); t += kBlock) {
        const uint32_t p = t >> 2, d = t & 3u;
        uint64_t before = 0;
        for (uint32_t q = 0; q < p; ++q)
            before += Cc((uint64_t)(4u * q + d + 1u) << shift) - Cc((uint64_t)(4u * q + d) << shift);
        Ej[t] = (uint32_t)(Cc((uint64_t)t << shift) - before);
    }
}

// 4-ary tree: quad_pass runs quad_tile_u8 per block; quad_tails writes what
// only the level's totals decide (the last rank entry, the sample counts and
// the sample slots past them), the totals coming from C.
template <bool SCATTER>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void quad_pass(QuadArgs a) {
    __shared__ LdsQuad s;
    quad_tile_u8<SCATTER>(a, blockIdx.x, s);
}

__global__ __launch_bounds__(kBlock) void quad_tails(const uint64_t *C, uint64_t sigma, uint32_t Lq, uint64_t n,
                                                     uint64_t *rank4, uint64_t R, uint64_t *sel4, uint64_t cap,
                                                     uint64_t *counts4) {
    const uint32_t j = blockIdx.x, kq = 2u * (Lq - 1u - j);
    __shared__ unsigned long long tot[4];
    if (threadIdx.x < 4) tot[threadIdx.x] = 0;
    __syncthreads();
    auto Cc = [&](uint64_t x) { return C[x < sigma ? x : sigma]; };
    for (uint64_t t = threadIdx.x; t < (4ull << (2u * j)); t += kBlock) {
        const uint64_t c = Cc((t + 1) << kq) - Cc(t << kq);
        if (c) atomicAdd(&tot[t & 3u], (unsigned long long)c);
    }
    __syncthreads();
    constexpr uint64_t S = WT_SELECT_SAMPLE;
    uint64_t *rk = rank4 + (uint64_t)j * R * 4, *sl = sel4 + (uint64_t)j * 4 * cap;
    if (threadIdx.x < 4) {
        rk[(R - 1) * 4 + threadIdx.x] = tot[threadIdx.x];
        counts4[(uint64_t)j * 4 + threadIdx.x] = (tot[threadIdx.x] + S - 1) / S;
    }
    for (uint64_t i = threadIdx.x; i < 4 * cap; i += kBlock)
        if (i % cap >= (tot[i / cap] + S - 1) / S) sl[i] = n;
}

// Exclusive prefixes (G_0, G_1, G_2) of per-tile packed digit counts (one
// block of 1024 threads, 16 tiles per thread per round; n < 2^32).
__global__ __launch_bounds__(kScanThreads) void pair_prefix_scan(const uint64_t *cnt, uint4 *pre, uint64_t T) {
    __shared__ uint32_t s_w[3][kScanThreads / kWave];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    uint32_t carry[3] = {0, 0, 0};
    for (uint64_t c0 = 0; c0 < T; c0 += (uint64_t)kScanThreads * 16) {
        const uint64_t base = c0 + (uint64_t)tid * 16;
        uint64_t v[16];
        uint32_t own[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            v[j] = base + j < T ? cnt[base + j] : 0ull;
#pragma unroll
            for (int c = 0; c < 3; ++c) own[c] += (uint32_t)(v[j] >> (16 * c)) & 0xFFFFu;
        }
        uint32_t inc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            inc[c] = wave_incl_scan_u32(own[c], lane);
            if (lane == kWave - 1) s_w[c][wave] = inc[c];
        }
        __syncthreads();
        uint32_t run[3], total[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uint32_t before = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < kScanThreads / kWave; ++w) {
                const uint32_t x = s_w[c][w];
                before += w < wave ? x : 0u;
                tot += x;
            }
            run[c] = carry[c] + before + inc[c] - own[c];
            total[c] = tot;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (base + j < T) pre[base + j] = make_uint4(run[0], run[1], run[2], 0u);
#pragma unroll
            for (int c = 0; c < 3; ++c) run[c] += (uint32_t)(v[j] >> (16 * c)) & 0xFFFFu;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) carry[c] += total[c];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Wavelet matrix tables: every level is one node, so its table is {0 ones
// before the node, the level's zeros}.  A level's zeros are those of the
// tree's same level (the same bit of the same symbols): the last entry of
// the tree table D_l.
__global__ void matrix_tables(const uint64_t *D, uint32_t L, uint64_t *Dm, uint64_t *zeros) {
    const uint32_t l = threadIdx.x;
    if (l >= L) return;
    const uint64_t z = D[(2ull << l) - 2 + (2ull << l) - 1];
    Dm[2 * l] = 0;
    Dm[2 * l + 1] = z;
    zeros[l] = z;
}

// ---------------------------------------------------------------------------
// Directory tails of every level (grid.y = level).  The level totals come
// either from the node tables (zeros of a level = D_l's last entry) or from
// an array of per-level totals.
__global__ void dir_finish(const uint64_t *D, const uint64_t *zeros_tot, uint64_t n, uint32_t L,
                           uint64_t *rank, uint64_t rank_len, uint64_t *sel1, uint64_t *sel0, uint64_t cap,
                           uint64_t *sel_counts) {
    const uint32_t l = blockIdx.y;
    const uint64_t zeros = zeros_tot ? zeros_tot[l] : D[(1ull << (l + 2)) - 3];
    dir_tail(l, zeros, n, L, rank, rank_len, sel1, sel0, cap, sel_counts,
             (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x);
}


// ---------------------------------------------------------------------------
// Standalone directories from existing bits: one wave per tile of 64 words
// of one level (grid.y = level), zero-count look-back per level.
__global__ __launch_bounds__(kWave) void dir_tiles(const uint64_t *bits, uint64_t n, uint64_t W,
                                                   uint64_t *state, uint64_t T, uint64_t *zeros_tot,
                                                   uint64_t *rank, uint64_t rank_len, uint64_t *sel1,
                                                   uint64_t *sel0, uint64_t cap, int spin_limit) {
    const uint32_t l = blockIdx.y;
    const int lane = lane_id();
    const uint64_t tile = blockIdx.x;
    const uint64_t t0 = tile * kDirTile;
    const uint32_t len = (uint32_t)min((uint64_t)kDirTile, n - t0);
    const uint64_t wi = (t0 >> 6) + lane;
    const bool has = (uint32_t)lane * 64u < len;
    const uint64_t word = has ? bits[(uint64_t)l * W + wi] : 0ull;
    const uint32_t nb = clamp_count(len, (uint32_t)lane * 64u, 64u);
    const uint32_t zc = nb - (uint32_t)__popcll(word);
    uint32_t inc = wave_incl_scan_u32(zc, lane);
    uint32_t Zt = __shfl(inc, kWave - 1, kWave);
    auto zeros_of_tile = [&](uint64_t ft) -> uint64_t {
        const uint64_t f0 = ft * kDirTile;
        const uint32_t flen = (uint32_t)min((uint64_t)kDirTile, n - f0);
        const bool fh = (uint32_t)lane * 64u < flen;
        const uint32_t fnb = clamp_count(flen, (uint32_t)lane * 64u, 64u);
        const uint64_t fw = fh ? bits[(uint64_t)l * W + (f0 >> 6) + lane] : 0ull;
        return wave_sum_u64((uint64_t)(fnb - (uint32_t)__popcll(fw)));
    };
    uint64_t Z0 = lookback_exclusive<4>(state + (uint64_t)l * T, tile, Zt, lane, spin_limit, zeros_of_tile);
    const uint64_t wd[1] = {word};
    const uint32_t zp[1] = {inc - zc};
    emit_directories<1>(wd, zp, Z0, t0, len, Zt, n, rank + (uint64_t)l * rank_len, sel1 + (uint64_t)l * cap,
                        sel0 + (uint64_t)l * cap, lane);
    if (tile == T - 1 && lane == 0) zeros_tot[l] = Z0 + Zt;
}

// ---------------------------------------------------------------------------
// Host side.
struct Plan {
    uint64_t n, sigma;
    uint32_t L, in_bytes, mid_bytes;
    uint64_t W, T, rank_len, cap;
    uint64_t off_status, off_cnt, off_pre, off_D, off_part, off_E, off_M, off_S0, off_S1, total;
    uint64_t off_lbs, LB;             // look-back state of the tile-prefix pass, words per level
    uint64_t off_PZ, off_NZ, off_CL;  // byte alphabets: piece counts, node zeros, node starts (wt_stats.hpp)
    uint64_t PS;                      // piece counts per level
    bool sparse;                      // node tables over the nonempty nodes only (wt_sparse.hpp)
    uint64_t ucap;                    // sparse: most distinct symbols, min(n, sigma)
    uint64_t off_U, off_NID, off_NS, off_SP;  // sparse: distinct symbols, node ids, node starts, counters
    uint64_t n_part;
};

static uint32_t levels_of(uint64_t sigma) {
    uint32_t L = 0;
    while (L < 64 && (1ull << L) < sigma) ++L;
    return L;
}

static int make_plan(uint64_t n, uint64_t sigma, int sym_bytes, Plan &p) {
    if (sigma == 0 || (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4)) return WT_ERR_ARG;
    if (sigma > (1ull << (8 * sym_bytes))) return WT_ERR_ARG;
    if (n >= (1ull << 40)) return WT_ERR_RANGE;
    p.n = n;
    p.sigma = sigma;
    p.L = levels_of(sigma);
    p.in_bytes = (uint32_t)sym_bytes;
    // Dense node tables hold 2^(L+1) words; past 30 levels, or when they
    // would dwarf the sequence, only the nonempty nodes (at most min(n, sigma)
    // per level) get entries.
    p.ucap = std::min<uint64_t>(n, sigma);
    p.sparse = p.in_bytes == 4 && p.L > 16 && (p.L > 30 || (2ull << p.L) > 4 * p.ucap + 65536);
    p.mid_bytes = p.L <= 8 ? 1u : (p.L <= 16 ? 2u : 4u);  // width of S_l for l >= 1
    p.W = cdiv(n, 64);
    p.T = cdiv(n, kMinTile);
    p.rank_len = cdiv(n, WT_RANK_BLOCK_BITS) + 1;
    p.cap = cdiv(n, WT_SELECT_SAMPLE) + 1;
    const uint64_t table_elems = p.L && !p.sparse ? (1ull << p.L) : 0;  // node heap indices [0, 2^L)
    // 2^(l+1) entries per level, or 2 per nonempty node of one level at a time
    const uint64_t D_len = p.sparse ? 2 * p.ucap : (p.L ? (2ull << p.L) - 2 : 0);
    const uint64_t part_c = cdiv(sigma, kScanChunk);
    const uint64_t part_t = cdiv(table_elems, kScanChunk);
    p.n_part = std::max<uint64_t>(std::max<uint64_t>(part_c, part_t), 1);
    uint64_t o = 0;
    p.off_status = o;
    o += 256;
    p.T = align_up(p.T, 64);  // per-level stride of the tile arrays (keeps vector loads aligned)
    // Per-tile arrays for an even number of levels: passes over two levels
    // (and the 4-ary tree) keep 64-bit counts and 16-byte prefixes per tile
    // in the room of two levels.
    const uint64_t Lt = p.L + (p.L & 1u);
    p.off_cnt = o;  // zeros per tile, per level (count-ahead), zeroed each build
    o = align_up(o + 4ull * Lt * p.T, 256);
    p.LB = cdiv(p.T, kTpSpan) + 1;  // look-back words per level of the tile-prefix pass
    p.off_lbs = o;                  // zeroed with the counts (it lies before off_pre)
    o = align_up(o + 8ull * p.L * p.LB, 256);
    p.off_pre = o;  // exclusive zero prefix per tile, per level
    o = align_up(o + 8ull * Lt * p.T, 256);
    p.off_D = o;
    o = align_up(o + 8ull * D_len, 256);
    p.off_part = o;
    o = align_up(o + 8ull * p.n_part, 256);
    p.off_E = o;  // two-level pass tables (byte alphabets: at most 4 x 256 u32)
    o += p.L >= 2 && p.L <= 8 ? kPairTableBytes : 0;
    p.off_M = o;  // wavelet matrix: {0, zeros of level l} per level
    o = align_up(o + 16ull * p.L, 256);
    // Byte alphabets: the statistics that replace the histogram (every
    // level's piece counts, node zeros and node starts).
    const bool byte_stats = p.in_bytes == 1 && p.L >= 1 && p.L <= 8;
    p.PS = byte_stats ? piece_stride(cdiv(n, 16384), p.L) : 0;
    p.off_PZ = o;
    o = align_up(o + 4 * p.PS * p.L, 256);
    p.off_NZ = o;
    o = align_up(o + (byte_stats ? 8ull << p.L : 0), 256);
    p.off_CL = o;
    o = align_up(o + (byte_stats ? 8 * ((1ull << p.L) + p.L) : 0), 256);
    const uint64_t uc = p.sparse ? p.ucap : 0;
    p.off_U = o;
    o = align_up(o + 4 * uc, 256);
    p.off_NID = o;
    o = align_up(o + 4 * uc, 256);
    p.off_NS = o;
    o = align_up(o + (p.sparse ? 8 * (uc + 1) : 0), 256);
    p.off_SP = o;  // |U|, node count, zeros of every level
    o = align_up(o + (p.sparse ? 8ull * (2 + p.L) : 0), 256);
    p.off_S0 = o;
    const uint64_t sbytes = p.L >= 2 ? align_up(n * p.mid_bytes, 256) : 0;
    o += sbytes;
    p.off_S1 = o;
    o += p.L >= 3 ? sbytes : 0;
    p.total = o;
    return WT_OK;
}

// Settings of the wt_set_* calls.  Each host thread has its own copy, so a
// caller that changes one for a comparison does not change the builds of
// other threads.
static thread_local bool g_timing = false;
static thread_local uint32_t g_fuse = 1;  // wt_set_fused_levels
static thread_local bool g_slices = true;  // sliced LDS histogram for wide alphabets
static thread_local bool g_pairs = false;  // two levels per pass for byte alphabets (measured slower: see wt_set_level_pairs)
static thread_local int g_spin_limit = 8;

// Tile prefixes of level l from the counts its predecessor left: one block
// when they fit one, else the multi-block pass.
static void tile_prefixes(const Plan &p, unsigned char *sc, uint32_t l, uint64_t Tl, hipStream_t s) {
    const uint32_t *cnt = (const uint32_t *)(sc + p.off_cnt) + (uint64_t)l * p.T;
    uint64_t *pre = (uint64_t *)(sc + p.off_pre) + (uint64_t)l * p.T;
    if (Tl <= (uint64_t)kTpSpan) {
        tile_prefix_scan<<<1, kScanThreads, 0, s>>>(cnt, pre, Tl);
    } else {
        uint64_t *state = (uint64_t *)(sc + p.off_lbs) + (uint64_t)l * p.LB;
        tile_prefix_multi<<<(unsigned)cdiv(Tl, kTpSpan), kBlock, 0, s>>>(cnt, pre, Tl, state, g_spin_limit);
    }
}
constexpr uint64_t kOffMaxNode = 8;   // in the status block: largest node per level (u64 x 30)
constexpr uint64_t kOffFusedL0 = 248; // in the status block: first fused level (u32)


static std::mutex g_timing_mu;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;  // recorded, not yet collected
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_free;
// Timing mode: the next timed launch carries this start/stop pair in its own
// dispatch (hipExtLaunchKernel), so the events time the kernel itself and
// add no marker packets to the stream around it.
static thread_local const std::pair<hipEvent_t, hipEvent_t> *t_ev = nullptr;

template <typename A>
static void launch_k(void (*k)(A), dim3 g, dim3 b, hipStream_t s, const A &a) {
    if (t_ev) {
        hipExtLaunchKernelGGL(k, g, b, 0, s, t_ev->first, t_ev->second, 0, a);
        t_ev = nullptr;
    } else {
        hipLaunchKernelGGL(k, g, b, 0, s, a);
    }
}

static int timing_begin(hipStream_t s, std::pair<hipEvent_t, hipEvent_t> &ev) {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (!g_free.empty()) {
        ev = g_free.back();
        g_free.pop_back();
    } else {
        // Timing only: no system-scope fence (a cache writeback) at each record.
        if (hipEventCreateWithFlags(&ev.first, hipEventDisableSystemFence) != hipSuccess ||
            hipEventCreateWithFlags(&ev.second, hipEventDisableSystemFence) != hipSuccess)
            return WT_ERR_HIP;
    }
    t_ev = &ev;
    return WT_OK;
}

static int timing_end(hipStream_t, std::pair<hipEvent_t, hipEvent_t> &ev) {
    if (t_ev) {  // a launch path that does not take the events (a bug): no measurement
        t_ev = nullptr;
        std::lock_guard<std::mutex> lk(g_timing_mu);
        g_free.push_back(ev);
        return WT_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_events.push_back(ev);
    return WT_OK;
}

static int num_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

template <typename TIN, typename TOUT>
static void launch_level(bool scatter, bool dirs, hipStream_t s, const LevelArgs &a) {
    if (sizeof(TIN) == 1 && sizeof(TOUT) == 1 && a.n < (1ull << 32)) {
        dim3 g8((unsigned)cdiv(a.n, 16384)), b8(kBlock);
        if (scatter) {
            if (dirs) launch_k(level_pass_u8<true, true>, g8, b8, s, a);
            else launch_k(level_pass_u8<true, false>, g8, b8, s, a);
        } else {
            if (dirs) launch_k(level_pass_u8<false, true>, g8, b8, s, a);
            else launch_k(level_pass_u8<false, false>, g8, b8, s, a);
        }
        return;
    }
    if (sizeof(TIN) == 2 && sizeof(TOUT) == 2 && a.n < (1ull << 32)) {
        dim3 g16((unsigned)cdiv(a.n, LdsLevelU16::kTile)), b16(kBlock);
        if (scatter) {
            if (dirs) launch_k(level_pass_u16<true, true>, g16, b16, s, a);
            else launch_k(level_pass_u16<true, false>, g16, b16, s, a);
        } else {
            if (dirs) launch_k(level_pass_u16<false, true>, g16, b16, s, a);
            else launch_k(level_pass_u16<false, false>, g16, b16, s, a);
        }
        return;
    }
    if (sizeof(TIN) == 4 && a.n < (1ull << 32)) {
        dim3 g32((unsigned)cdiv(a.n, LdsLevelU32::kTile)), b32(kBlock);
        if (scatter) {
            if (dirs) launch_k(level_pass_u32<TOUT, true, true>, g32, b32, s, a);
            else launch_k(level_pass_u32<TOUT, true, false>, g32, b32, s, a);
        } else {
            if (dirs) launch_k(level_pass_u32<TOUT, false, true>, g32, b32, s, a);
            else launch_k(level_pass_u32<TOUT, false, false>, g32, b32, s, a);
        }
        return;
    }
    dim3 grid((unsigned)cdiv(a.n, TileCfg<TIN>::kTile)), block(kBlock);
    if (scatter) {
        if (dirs) launch_k(level_pass<TIN, TOUT, true, true>, grid, block, s, a);
        else launch_k(level_pass<TIN, TOUT, true, false>, grid, block, s, a);
    } else {
        if (dirs) launch_k(level_pass<TIN, TOUT, false, true>, grid, block, s, a);
        else launch_k(level_pass<TIN, TOUT, false, false>, grid, block, s, a);
    }
}

static void launch_level_any(uint32_t tin, uint32_t tout, bool scatter, bool dirs, hipStream_t s,
                             const LevelArgs &a) {
#define WT_LV(I, O)                                            \
    if (tin == sizeof(I) && tout == sizeof(O)) {               \
        launch_level<I, O>(scatter, dirs, s, a);               \
        return;                                                \
    }
    WT_LV(uint8_t, uint8_t)
    WT_LV(uint16_t, uint8_t)
    WT_LV(uint32_t, uint8_t)
    WT_LV(uint16_t, uint16_t)
    WT_LV(uint32_t, uint16_t)
    WT_LV(uint32_t, uint32_t)
#undef WT_LV
}


template <typename TIN0, typename T>
static void launch_fused_t(const FusedArgs &f, uint64_t n, hipStream_t s) {
    const uint64_t nseg = cdiv(n, FusedCfg<T, kFusedBytes>::kHalf);
    const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(nseg, (uint64_t)num_cus() * 4));
    fused_pass<TIN0, T><<<(unsigned)grid, kBlock, 0, s>>>(f, nseg);
}

static uint64_t fused_half(uint32_t mid) {
    return mid == 1 ? FusedCfg<uint8_t, kFusedBytes>::kHalf
                    : (mid == 2 ? FusedCfg<uint16_t, kFusedBytes>::kHalf : FusedCfg<uint32_t, kFusedBytes>::kHalf);
}

static void launch_fused(uint32_t in_w, uint32_t mid, const FusedArgs &f, uint64_t n, hipStream_t s) {
#define WT_FU(I, O)                                \
    if (in_w == sizeof(I) && mid == sizeof(O)) {   \
        launch_fused_t<I, O>(f, n, s);             \
        return;                                    \
    }
    WT_FU(uint8_t, uint8_t)
    WT_FU(uint16_t, uint8_t)
    WT_FU(uint32_t, uint8_t)
    WT_FU(uint16_t, uint16_t)
    WT_FU(uint32_t, uint16_t)
    WT_FU(uint32_t, uint32_t)
#undef WT_FU
}

// Wide alphabets: the sliced histogram when the S ping-pong (idle until
// level 0 scatters) holds one row of counts per chunk and the input is long
// enough to fill a chunk per slice; the LDS-hash histogram otherwise.
// Input chunks of the sliced histogram (one row of sigma counts each), or 0
// when it does not apply.
static uint64_t slice_chunks(const Plan &p, uint32_t in_bytes) {
    constexpr uint64_t kMinChunkTiles = 16;
    if (p.sigma <= 8192 || p.L < 2) return 0;
    const uint64_t ntiles = cdiv(p.n, 1ull << tile_shift_for(in_bytes));
    const uint32_t nslices = (uint32_t)cdiv(p.sigma, kSliceBins);
    const uint64_t row_room = align_up(p.n * p.mid_bytes, 256) / (4 * p.sigma);
    uint64_t nchunks = std::max<uint64_t>(1, (uint64_t)num_cus() / nslices);
    nchunks = std::min(nchunks, row_room);
    nchunks = std::min(nchunks, cdiv(ntiles, kMinChunkTiles));
    return nchunks;
}

template <typename T>
static bool launch_hist_slices(const void *seq, const Plan &p, uint64_t *Cp1, uint32_t *status, uint32_t *cnt0,
                               void *rows, hipStream_t s) {
    uint64_t nchunks = slice_chunks(p, sizeof(T));
    if (nchunks == 0) return false;
    const uint32_t shift = tile_shift_for(sizeof(T));
    const uint64_t ntiles = cdiv(p.n, 1ull << shift);
    const uint32_t nslices = (uint32_t)cdiv(p.sigma, kSliceBins);
    const uint64_t per_chunk = cdiv(ntiles, nchunks);
    nchunks = cdiv(ntiles, per_chunk);
    const uint64_t grid = cdiv(nchunks, 8) * 8 * nslices;
    hist_slices<T><<<(unsigned)grid, kSliceThreads, 0, s>>>((const T *)seq, p.n, p.sigma, nslices, nchunks, per_chunk,
                                                            shift, p.L - 1, cnt0, (unsigned long long *)Cp1,
                                                            (uint32_t *)rows, status);
    const uint64_t rblocks = std::min<uint64_t>(cdiv(p.sigma, kBlock), 4096);
    const dim3 rgrid((unsigned)rblocks, (unsigned)std::min<uint64_t>(nchunks, 16));
    hist_reduce<<<rgrid, kBlock, 0, s>>>((const uint32_t *)rows, nchunks, p.sigma, Cp1);
    return true;
}

// `digits`: the per-tile output is the packed digit counts of bits
// (dig_top, dig_top - 1), by default the top two (uint64 per tile), that a
// first pass over two levels reads.
template <typename T>
static void launch_hist(const void *seq, const Plan &p, uint64_t *Cp1, uint32_t *status, uint32_t *cnt0,
                        void *rows, bool digits, hipStream_t s, uint32_t dig_top = 0) {
    if (!digits && g_slices && launch_hist_slices<T>(seq, p, Cp1, status, cnt0, rows, s)) return;
    uint32_t reps = 0;  // LDS replicas (64 lanes share them), 0 = global atomics
    if (p.sigma <= 8192) reps = (uint32_t)std::min<uint64_t>(16, std::max<uint64_t>(1, 8192 / (p.sigma + 1)));
    const uint32_t shift = tile_shift_for(sizeof(T));
    const uint64_t ntiles = cdiv(p.n, 1ull << shift);
    uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>(ntiles, (uint64_t)num_cus() * 8));
    const size_t shm = reps ? (size_t)reps * (p.sigma + 1) * 4 : (size_t)HistHash<4096>::kWords * 4;
    if (digits)
        histogram<T, true><<<(unsigned)blocks, kBlock, shm, s>>>((const T *)seq, p.n, p.sigma,
                                                                 (unsigned long long *)Cp1, status, reps,
                                                                 dig_top ? dig_top : p.L - 1, cnt0, shift, ntiles);
    else
        histogram<T, false><<<(unsigned)blocks, kBlock, shm, s>>>((const T *)seq, p.n, p.sigma,
                                                                  (unsigned long long *)Cp1, status, reps,
                                                                  p.L ? p.L - 1 : 0u, p.L ? cnt0 : nullptr, shift,
                                                                  ntiles);
}

}  // namespace wt

using namespace wt;

extern "C" int wt_plan(uint64_t n, uint64_t sigma, int sym_bytes, wt_layout *out) {
    if (!out) return WT_ERR_ARG;
    Plan p;
    int rc = make_plan(n, sigma, sym_bytes, p);
    if (rc) return rc;
    out->n = n;
    out->sigma = sigma;
    out->L = p.L;
    out->sym_bytes = (uint32_t)sym_bytes;
    out->words_per_level = p.W;
    out->bits_words = (uint64_t)p.L * p.W;
    out->C_len = sigma + 1;
    out->rank_len = p.rank_len;
    out->sel_cap = p.cap;
    out->sel_counts_len = 2ull * p.L;
    out->scratch_bytes = p.total;
    out->rs_scratch_bytes = wt_rank_select_scratch_bytes(n, p.L);
    return WT_OK;
}

extern "C" uint64_t wt_rank_select_scratch_bytes(uint64_t n, uint32_t L) {
    uint64_t T = cdiv(n, kDirTile);
    // per-level zero totals, per-level look-back states
    return align_up(8ull * std::max<uint32_t>(L, 1u), 256) + align_up(8ull * L * T, 256);
}

// Which kernels a build runs, a function of the plan, the kind of build and
// this thread's settings.
struct PathChoice {
    bool fuse, pairs, two_phase, stats;
    uint32_t lmin, cbits, fine_blocks;
    int hist;  // WT_HIST_*
};

static PathChoice choose_path(const Plan &p, bool matrix, bool dirs) {
    PathChoice c{};
    const uint64_t n = p.n;
    // Fused tail levels need the directories (they write their entries) and
    // at least one split to save.  The 2^l nodes of level l share n symbols,
    // so its largest node holds at least ceil(n / 2^l): no level below
    // `lmin` can fuse, and when lmin > L-2 none can, which leaves the level
    // passes without the per-tile check of the fused level.
    c.lmin = 0;
    while (c.lmin < 63 && cdiv(n, 1ull << c.lmin) > fused_half(p.mid_bytes)) ++c.lmin;
    c.fuse = g_fuse != 0 && !matrix && !p.sparse && dirs && p.L >= 2 && n > 0 && c.lmin + 2 <= p.L;
    // Two levels per pass: byte symbols in and between levels, nothing fused
    // (inputs too small for that are the fused pass's), 32-bit positions.
    c.pairs = g_pairs && !matrix && !c.fuse && p.in_bytes == 1 && p.mid_bytes == 1 && p.L >= 2 && n > 0 &&
              n < (1ull << 32);
    // Wide alphabets (more than 16 levels): the two-phase histogram (see
    // hist_coarse / hist_fine) when its rows, overflow counts and tags fit
    // the idle ping-pong buffer at level c and no level before c can fuse.
    c.cbits = p.L > kFineBits ? p.L - kFineBits : 0u;
    c.fine_blocks = (uint32_t)std::min(num_cus(), 1024);
    const uint64_t fine_rows = (uint64_t)c.fine_blocks << kFineBits;  // u32 counts
    const uint64_t fine_bytes = 4 * fine_rows + 8 * align_up(p.sigma, 32) + 4 * 1024;
    c.two_phase = g_slices && !matrix && !c.pairs && !p.sparse && c.cbits >= 1 && c.cbits <= kCoarseMaxBits &&
                  p.in_bytes == 4 && p.mid_bytes == 4 && n >= (1ull << 20) && n < (1ull << 32) &&
                  fine_bytes <= align_up(n * p.mid_bytes, 256) && (!c.fuse || c.lmin >= c.cbits);
    // Byte alphabets with no fused or paired levels: no histogram pass (the
    // level passes count what the next level's tables need, wt_stats.hpp).
    c.stats = !matrix && !c.fuse && !c.pairs && p.in_bytes == 1 && p.L >= 1 && p.L <= 8 && n > 0 &&
              n < (1ull << 32);
    if (n == 0) c.hist = WT_HIST_NONE;
    else if (c.stats) c.hist = WT_HIST_LEVELS;
    else if (c.two_phase) c.hist = WT_HIST_TWO_PHASE;
    else if (!c.pairs && g_slices && slice_chunks(p, p.in_bytes)) c.hist = WT_HIST_SLICES;
    else if (p.sigma <= 8192) c.hist = WT_HIST_REPLICAS;
    else c.hist = WT_HIST_HASH;
    return c;
}

static void launch_pair(bool scatter, bool next_pair, bool dirs, uint32_t tiles, hipStream_t s, const PairArgs &a) {
#define WT_PAIR(SC, NP, DI) \
    if (scatter == SC && next_pair == NP && dirs == DI) return launch_k(pair_pass<SC, NP, DI>, dim3(tiles), dim3(kBlock), s, a);
    WT_PAIR(true, true, true)
    WT_PAIR(true, false, true)
    WT_PAIR(false, false, true)
    WT_PAIR(true, true, false)
    WT_PAIR(true, false, false)
    WT_PAIR(false, false, false)
#undef WT_PAIR
}

// The levels of a byte alphabet two at a time (a last odd level alone),
// after the histogram left the level-0 digit counts per tile.  Pair l reads
// S_l, writes B_l, B_{l+1}, their directory entries and S_{l+2}, and counts
// ahead for the next pass.
static int run_pairs(const void *d_seq, const Plan &p, const wt_outputs *out, unsigned char *sc, bool dirs,
                     hipStream_t s, bool timed) {
    const uint64_t n = p.n;
    uint32_t *status = (uint32_t *)(sc + p.off_status);
    uint32_t *cnt = (uint32_t *)(sc + p.off_cnt);
    uint64_t *pre = (uint64_t *)(sc + p.off_pre);
    uint64_t *D = (uint64_t *)(sc + p.off_D);
    uint32_t *E = (uint32_t *)(sc + p.off_E);
    digit_tables<<<p.L / 2, kBlock, 0, s>>>(out->C, p.sigma, p.L - 2, E);
    const uint32_t shift = tile_shift_for(1);
    const uint64_t Tl = cdiv(n, 1ull << shift);
    const void *cur = d_seq;
    int buf = 0;
    int rc;
    for (uint32_t l = 0; l < p.L; l += 2) {
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (l + 1 < p.L) {
            const bool scatter = l + 2 < p.L, next_pair = l + 3 < p.L;
            pair_prefix_scan<<<1, kScanThreads, 0, s>>>((const uint64_t *)(cnt + (uint64_t)l * p.T),
                                                        (uint4 *)(pre + (uint64_t)l * p.T), Tl);
            void *dst = buf == 0 ? (void *)(sc + p.off_S0) : (void *)(sc + p.off_S1);
            PairArgs a;
            a.in = (const uint8_t *)cur;
            a.out = scatter ? (uint8_t *)dst : nullptr;
            a.bits0 = out->bits + (uint64_t)l * p.W;
            a.bits1 = out->bits + (uint64_t)(l + 1) * p.W;
            a.C = out->C;
            a.sigma = p.sigma;
            a.D0 = D + ((2ull << l) - 2);
            a.D1 = D + ((4ull << l) - 2);
            a.E = E + 256u * (l / 2);
            a.pre = (const uint4 *)(pre + (uint64_t)l * p.T);
            a.next_cnt = scatter ? (void *)(cnt + (uint64_t)(l + 2) * p.T) : nullptr;
            a.next_shift = shift;
            a.status = status;
            a.rank0 = dirs ? out->rank + (uint64_t)l * p.rank_len : nullptr;
            a.sel10 = dirs ? out->sel1 + (uint64_t)l * p.cap : nullptr;
            a.sel00 = dirs ? out->sel0 + (uint64_t)l * p.cap : nullptr;
            a.rank1 = dirs ? out->rank + (uint64_t)(l + 1) * p.rank_len : nullptr;
            a.sel11 = dirs ? out->sel1 + (uint64_t)(l + 1) * p.cap : nullptr;
            a.sel01 = dirs ? out->sel0 + (uint64_t)(l + 1) * p.cap : nullptr;
            a.n = (uint32_t)n;
            a.k = p.L - 1 - l;
            a.level = l;
            if (timed && (rc = timing_begin(s, ev))) return rc;
            launch_pair(scatter, next_pair, dirs, (uint32_t)Tl, s, a);
            if (timed && (rc = timing_end(s, ev))) return rc;
            if (scatter) {
                cur = dst;
                buf ^= 1;
            }
        } else {
            tile_prefixes(p, sc, l, Tl, s);
            LevelArgs a;
            a.in = cur;
            a.out = nullptr;
            a.bits = out->bits + (uint64_t)l * p.W;
            a.D = D + ((2ull << l) - 2);
            a.nD = 2ull << l;
            a.tile_prefix = pre + (uint64_t)l * p.T;
            a.next_cnt = nullptr;
            a.next_shift = shift;
            a.status = status;
            a.rank = dirs ? out->rank + (uint64_t)l * p.rank_len : nullptr;
            a.sel1 = dirs ? out->sel1 + (uint64_t)l * p.cap : nullptr;
            a.sel0 = dirs ? out->sel0 + (uint64_t)l * p.cap : nullptr;
            a.n = n;
            a.k = 0;
            a.level = l;
            a.fused_l0 = nullptr;
            a.qmask = ~0u;
            if (timed && (rc = timing_begin(s, ev))) return rc;
            launch_level_any(1, 1, false, dirs, s, a);
            if (timed && (rc = timing_end(s, ev))) return rc;
        }
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
    }
    return WT_OK;
}

// Byte alphabets without a histogram pass (wt_stats.hpp): one read-only
// pass gives level 0's tile counts and the symbol check; then per level the
// statistics kernel (tile prefixes and the node table from the piece counts
// the level above left, the status word at level 0, C at the last level)
// and the byte level pass, which counts its next level's zeros per piece.
// Level L-2's pass writes the last level's bits itself (LASTBITS), so the
// last level reads only its bits, for its directories.
static int run_stats(const void *d_seq, const Plan &p, const wt_outputs *out, unsigned char *sc, bool dirs,
                     hipStream_t s, bool timed) {
    const uint64_t n = p.n;
    uint32_t *status = (uint32_t *)(sc + p.off_status);
    uint64_t *D = (uint64_t *)(sc + p.off_D);
    uint32_t *pz = (uint32_t *)(sc + p.off_PZ);
    uint64_t *NZ = (uint64_t *)(sc + p.off_NZ), *CL = (uint64_t *)(sc + p.off_CL);
    const uint32_t Tl = (uint32_t)cdiv(n, 16384);
    // Level 0's pieces are its tiles; everything after them is cleared.
    const uint64_t nclear = p.PS * p.L - Tl;
    const unsigned pg = (unsigned)cdiv(Tl, kPrepWaves), pb = kPrepWaves * kWave;
    if (p.sigma < 256)
        stats_prep_u8<true><<<pg, pb, 0, s>>>((const uint8_t *)d_seq, (uint32_t)n, p.L - 1, (uint32_t)p.sigma, pz,
                                              pz + Tl, nclear);
    else
        stats_prep_u8<false><<<pg, pb, 0, s>>>((const uint8_t *)d_seq, (uint32_t)n, p.L - 1, (uint32_t)p.sigma,
                                               pz, pz + Tl, nclear);
    const void *cur = d_seq;
    int rc;
    for (uint32_t l = 0; l < p.L; ++l) {
        const bool scatter = l + 1 < p.L;
        StatsArgs sa;
        sa.pieces = pz + (uint64_t)l * p.PS;
        sa.E = pz + (uint64_t)l * p.PS;  // in place: each thread rewrites only the counts it read
        sa.T = Tl;
        sa.tile_shift = tile_shift_for(1);
        sa.level = l;
        sa.L = p.L;
        sa.n = n;
        sa.sigma = p.sigma;
        sa.status = status;
        sa.NZ = NZ;
        sa.CL = CL;
        sa.D = D + ((2ull << l) - 2);
        sa.C = out->C;
        stats_scan<<<1, kStatsThreads, 0, s>>>(sa);
        void *dst = (l % 2 == 0) ? (void *)(sc + p.off_S0) : (void *)(sc + p.off_S1);
        LevelArgs a;
        a.in = cur;
        a.out = scatter ? dst : nullptr;
        a.bits = out->bits + (uint64_t)l * p.W;
        a.D = sa.D;
        a.nD = 2ull << l;
        a.tile_prefix = nullptr;
        a.piece_prefix = sa.E;
        a.node_starts = CL + (1ull << l) - 1 + l;  // CL_l (read by the last level's directory pass)
        a.nodes = (1u << l) + 1;
        a.next_cnt = scatter ? pz + (uint64_t)(l + 1) * p.PS : nullptr;
        a.next_shift = tile_shift_for(1);
        a.status = status;
        a.rank = dirs ? out->rank + (uint64_t)l * p.rank_len : nullptr;
        a.sel1 = dirs ? out->sel1 + (uint64_t)l * p.cap : nullptr;
        a.sel0 = dirs ? out->sel0 + (uint64_t)l * p.cap : nullptr;
        a.n = n;
        a.k = p.L - 1 - l;
        a.level = l;
        a.fused_l0 = nullptr;
        a.qmask = ~0u;
        a.tails = dirs ? 1u : 0u;
        a.L = p.L;
        a.sel_counts = out->sel_counts;
        a.rank_len = p.rank_len;
        a.cap = p.cap;
        const bool lastbits = l + 2 == p.L;  // this pass writes B_{L-1} too
        const bool dirs_only = l + 1 == p.L && p.L >= 2;
        if (lastbits) {
            a.out = nullptr;
            a.next_bits = out->bits + (uint64_t)(l + 1) * p.W;
        }
        if (dirs_only && !dirs) break;  // the last level's bits are in place
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (timed && (rc = timing_begin(s, ev))) return rc;
        const dim3 g(Tl), b(kBlock);
        if (dirs_only) {
            launch_k(level_dirs, dim3((unsigned)cdiv(Tl, kDirsWaves)), dim3(kDirsWaves * kWave), s, a);
        } else if (lastbits) {
            if (dirs) launch_k(level_pass_u8<true, true, true, true>, g, b, s, a);
            else launch_k(level_pass_u8<true, false, true, true>, g, b, s, a);
        } else if (scatter) {
            if (dirs) launch_k(level_pass_u8<true, true, true>, g, b, s, a);
            else launch_k(level_pass_u8<true, false, true>, g, b, s, a);
        } else {  // L = 1: the only level, its tile prefixes from its pieces (no tile_prefix array here)
            if (dirs) launch_k(level_pass_u8<false, true, true>, g, b, s, a);
            else launch_k(level_pass_u8<false, false, true>, g, b, s, a);
        }
        if (timed && (rc = timing_end(s, ev))) return rc;
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
        cur = dst;
    }
    return WT_OK;
}

// One device-wide scan over `count` values of the functor (see scan_final).
template <typename F>
static void run_scan(const F &f, uint64_t count, uint64_t *part, hipStream_t s) {
    const uint64_t chunks = cdiv(count, kScanChunk);
    if (chunks > 1) {
        scan_reduce<F><<<(unsigned)chunks, kBlock, 0, s>>>(f, count, part);
        scan_partials_seg<F><<<1, kBlock, 0, s>>>(f, chunks, part);
        scan_final<F><<<(unsigned)chunks, kBlock, 0, s>>>(f, count, part);
    } else if (count > 0) {
        scan_final<F><<<1, kBlock, 0, s>>>(f, count, nullptr);
    }
}

// The zeros of every level and their {0, zeros} tables for the wavelet
// matrix, from the symbols present.
__global__ void matrix_tables_from_zeros(const uint64_t *zeros_l, uint32_t L, uint64_t *Dm, uint64_t *zeros) {
    const uint32_t l = threadIdx.x;
    if (l >= L) return;
    Dm[2 * l] = 0;
    Dm[2 * l + 1] = zeros_l[l];
    if (zeros) zeros[l] = zeros_l[l];
}

struct SparseLevel {
    LevelArgs a;
    SparseArgs sp;
};

template <typename TIN, typename TOUT, bool SCATTER, bool DIRS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void level_pass_sparse(SparseLevel x) {
    __shared__ LdsSparse<TIN> s;
    level_tile_sparse<TIN, TOUT, SCATTER, DIRS>(x.a, x.sp, blockIdx.x, s);
}

// Sparse node tables (wt_sparse.hpp), after C: the distinct symbols, then
// per level its nonempty nodes, their table and the level's zeros.  For the
// tree, each level's pass follows its table; for the wavelet matrix only
// the zeros of every level are needed (its matrix passes run afterwards).
static int sparse_tables(const Plan &p, const wt_outputs *out, unsigned char *sc, uint32_t l, hipStream_t s) {
    uint32_t *U = (uint32_t *)(sc + p.off_U), *NID = (uint32_t *)(sc + p.off_NID);
    uint64_t *NS = (uint64_t *)(sc + p.off_NS), *SP = (uint64_t *)(sc + p.off_SP);
    uint64_t *D = (uint64_t *)(sc + p.off_D), *part = (uint64_t *)(sc + p.off_part);
    if (l == 0) run_scan(CompactOp{out->C, p.sigma, U, SP}, p.sigma, part, s);
    run_scan(NodeIdOp{U, SP, p.L - l, NID, SP + 1}, p.ucap, part, s);
    run_scan(SparseTableOp{out->C, p.sigma, p.n, NID, SP + 1, p.L - l, NS, D, SP + 2 + l}, p.ucap, part, s);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

template <typename TIN, typename TOUT>
static void launch_sparse_t(bool scatter, bool dirs, hipStream_t s, const SparseLevel &x) {
    const dim3 g((unsigned)cdiv(x.a.n, TileCfg<TIN>::kTile)), b(kBlock);
    if (scatter) {
        if (dirs) launch_k(level_pass_sparse<TIN, TOUT, true, true>, g, b, s, x);
        else launch_k(level_pass_sparse<TIN, TOUT, true, false>, g, b, s, x);
    } else {
        if (dirs) launch_k(level_pass_sparse<TIN, TOUT, false, true>, g, b, s, x);
        else launch_k(level_pass_sparse<TIN, TOUT, false, false>, g, b, s, x);
    }
}

static int run_sparse(const void *d_seq, const Plan &p, const wt_outputs *out, unsigned char *sc, bool dirs,
                      hipStream_t s, bool timed) {
    const uint64_t n = p.n;
    uint32_t *status = (uint32_t *)(sc + p.off_status);
    uint32_t *cnt = (uint32_t *)(sc + p.off_cnt);
    uint64_t *pre = (uint64_t *)(sc + p.off_pre);
    uint64_t *D = (uint64_t *)(sc + p.off_D), *SP = (uint64_t *)(sc + p.off_SP);
    const uint32_t shift = tile_shift_for(4);
    const uint64_t Tl = cdiv(n, 1ull << shift);
    const void *cur = d_seq;
    int rc;
    for (uint32_t l = 0; l < p.L; ++l) {
        if ((rc = sparse_tables(p, out, sc, l, s))) return rc;
        const bool scatter = l + 1 < p.L;
        void *dst = (l % 2 == 0) ? (void *)(sc + p.off_S0) : (void *)(sc + p.off_S1);
        tile_prefixes(p, sc, l, Tl, s);
        LevelArgs a;
        a.in = cur;
        a.out = scatter ? dst : nullptr;
        a.bits = out->bits + (uint64_t)l * p.W;
        a.D = D;
        a.nD = 2 * p.ucap;
        a.tile_prefix = pre + (uint64_t)l * p.T;
        a.next_cnt = scatter ? cnt + (uint64_t)(l + 1) * p.T : nullptr;
        a.next_shift = shift;
        a.status = status;
        a.rank = dirs ? out->rank + (uint64_t)l * p.rank_len : nullptr;
        a.sel1 = dirs ? out->sel1 + (uint64_t)l * p.cap : nullptr;
        a.sel0 = dirs ? out->sel0 + (uint64_t)l * p.cap : nullptr;
        a.n = n;
        a.k = p.L - 1 - l;
        a.level = l;
        a.fused_l0 = nullptr;
        a.qmask = ~0u;
        a.tails = dirs ? 1u : 0u;
        a.L = p.L;
        a.sel_counts = out->sel_counts;
        a.rank_len = p.rank_len;
        a.cap = p.cap;
        const SparseLevel x{a, SparseArgs{(const uint32_t *)(sc + p.off_NID), (const uint64_t *)(sc + p.off_NS),
                                          SP + 1, SP + 2 + l}};
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (timed && (rc = timing_begin(s, ev))) return rc;
        launch_sparse_t<uint32_t, uint32_t>(scatter, dirs, s, x);
        if (timed && (rc = timing_end(s, ev))) return rc;
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
        cur = dst;
    }
    return WT_OK;
}

// The wavelet tree (matrix = false) or the wavelet matrix (matrix = true:
// every level one node, split with D_l = {0, zeros of the level}; no fused
// or paired levels; the zero counts also go to d_zeros).
static int build_impl(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                      bool matrix, uint64_t *d_zeros, void *d_scratch, uint64_t scratch_bytes, void *stream,
                      bool timed) {
    Plan p;
    int rc = make_plan(n, sigma, sym_bytes, p);
    if (rc) return rc;
    if (!out || !out->C || !d_scratch || (n > 0 && !d_seq) || (p.L > 0 && n > 0 && !out->bits)) return WT_ERR_ARG;
    const bool dirs = out->rank != nullptr;
    if (dirs != (out->sel1 != nullptr) || dirs != (out->sel0 != nullptr) || dirs != (out->sel_counts != nullptr))
        return WT_ERR_ARG;
    if (((uintptr_t)d_seq & 15u) || ((uintptr_t)d_scratch & 255u)) return WT_ERR_ARG;
    if (scratch_bytes < p.total) return WT_ERR_SCRATCH;
    hipStream_t s = (hipStream_t)stream;
    unsigned char *sc = (unsigned char *)d_scratch;
    uint32_t *status = (uint32_t *)(sc + p.off_status);
    uint32_t *cnt = (uint32_t *)(sc + p.off_cnt);
    uint64_t *pre = (uint64_t *)(sc + p.off_pre);
    uint64_t *D = (uint64_t *)(sc + p.off_D);
    uint64_t *part = (uint64_t *)(sc + p.off_part);
    uint64_t *Dm = (uint64_t *)(sc + p.off_M);

    const PathChoice pc = choose_path(p, matrix, dirs);
    if (pc.stats) return run_stats(d_seq, p, out, sc, dirs, s, timed);
    const uint32_t lmin = pc.lmin, cbits = pc.cbits, fine_blocks = pc.fine_blocks;
    const bool fuse = pc.fuse, pairs = pc.pairs, two_phase = pc.two_phase;
    const uint64_t fine_rows = (uint64_t)fine_blocks << kFineBits;  // u32 counts

    // Zero: status + per-tile zero counts (one contiguous range), and C.
    {
        uint64_t na = p.off_pre / 8, nb = sigma + 1;
        uint64_t blocks = std::min<uint64_t>(cdiv(na + nb, kBlock), 4096);
        zero_fill<<<(unsigned)blocks, kBlock, 0, s>>>((uint64_t *)sc, na, out->C, nb);
    }
    if (n > 0 && two_phase) {
        // Coarse phase: group counts into the idle S1 (level 0 writes S0),
        // level-0 tile zeros, the symbol check; then C at the group starts.
        unsigned long long *cc = (unsigned long long *)(sc + p.off_S1);
        zero_fill<<<1, kBlock, 0, s>>>((uint64_t *)cc, 1ull << cbits, nullptr, 0);
        const uint32_t shift = tile_shift_for(4);
        const uint64_t ntiles = cdiv(n, 1ull << shift);
        const uint32_t reps = std::min<uint32_t>(16u, kCoarseTab / ((1u << cbits) + 1u));
        const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>(ntiles, (uint64_t)num_cus() * 8));
        hist_coarse<uint32_t><<<(unsigned)blocks, kBlock, 0, s>>>((const uint32_t *)d_seq, n, sigma, p.L, cbits, reps,
                                                                   shift, ntiles, cnt, cc, status);
        coarse_to_C<<<1, 1024, 0, s>>>(cc, cbits, p.L, sigma, out->C);
    } else if (n > 0) {
        void *rows = sc + p.off_S0;
        if (sym_bytes == 1) launch_hist<uint8_t>(d_seq, p, out->C + 1, status, cnt, rows, pairs, s);
        else if (sym_bytes == 2) launch_hist<uint16_t>(d_seq, p, out->C + 1, status, cnt, rows, false, s);
        else launch_hist<uint32_t>(d_seq, p, out->C + 1, status, cnt, rows, false, s);
        // C: prefix sums of the counts.
        CScanOp cop{out->C + 1};
        uint64_t chunks = cdiv(sigma, kScanChunk);
        if (chunks > 1) {
            scan_reduce<CScanOp><<<(unsigned)chunks, kBlock, 0, s>>>(cop, sigma, part);
            scan_partials_seg<CScanOp><<<1, kBlock, 0, s>>>(cop, chunks, part);
            scan_final<CScanOp><<<(unsigned)chunks, kBlock, 0, s>>>(cop, sigma, part);
        } else {
            scan_final<CScanOp><<<1, kBlock, 0, s>>>(cop, sigma, nullptr);
        }
    }
    // Node tables of the heap's first `count` entries (levels below
    // log2(count)), from C; with `tail`, the directory tails, the matrix
    // tables and the fusion plan, which need every level.
    uint32_t *fused_l0 = (uint32_t *)(sc + p.off_status + kOffFusedL0);
    auto tables = [&](uint64_t count, bool tail) {
        TableOp top{out->C, D, sigma, p.L};
        uint64_t chunks = cdiv(count, kScanChunk);
        if (chunks > 1) {
            scan_reduce<TableOp><<<(unsigned)chunks, kBlock, 0, s>>>(top, count, part);
            scan_partials_seg<TableOp><<<1, kBlock, 0, s>>>(top, chunks, part);
            scan_final<TableOp><<<(unsigned)chunks, kBlock, 0, s>>>(top, count, part);
        } else {
            scan_final<TableOp><<<1, kBlock, 0, s>>>(top, count, nullptr);
        }
        if (!tail) return;
        if (dirs) {
            dim3 g((unsigned)cdiv(p.cap, kBlock), p.L);
            dir_finish<<<g, kBlock, 0, s>>>(D, nullptr, n, p.L, out->rank, p.rank_len, out->sel1, out->sel0, p.cap,
                                            out->sel_counts);
        }
        if (matrix) matrix_tables<<<1, kWave, 0, s>>>(D, p.L, Dm, d_zeros);
        if (fuse) {
            unsigned long long *maxnode = (unsigned long long *)(sc + p.off_status + kOffMaxNode);
            const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>(cdiv(1ull << (p.L - 1), kBlock), 2048));
            node_max_kernel<<<(unsigned)blocks, kBlock, 0, s>>>(out->C, sigma, p.L, maxnode);
            fuse_plan_kernel<<<1, kWave, 0, s>>>(maxnode, p.L, fused_half(p.mid_bytes), g_fuse, fused_l0);
        }
    };
    auto c_scan = [&]() {
        CScanOp cop{out->C + 1};
        uint64_t chunks = cdiv(sigma, kScanChunk);
        if (chunks > 1) {
            scan_reduce<CScanOp><<<(unsigned)chunks, kBlock, 0, s>>>(cop, sigma, part);
            scan_partials_seg<CScanOp><<<1, kBlock, 0, s>>>(cop, chunks, part);
            scan_final<CScanOp><<<(unsigned)chunks, kBlock, 0, s>>>(cop, sigma, part);
        } else {
            scan_final<CScanOp><<<1, kBlock, 0, s>>>(cop, sigma, nullptr);
        }
    };
    if (p.sparse) {
        // Sparse node tables: the tree's passes follow them level by level;
        // the matrix needs only every level's zeros, then its own passes.
        uint64_t *SP = (uint64_t *)(sc + p.off_SP);
        if (n == 0) {
            zero_fill<<<1, kBlock, 0, s>>>(SP + 2, p.L, nullptr, 0);
        } else if (matrix) {
            for (uint32_t l = 0; l < p.L; ++l)
                if ((rc = sparse_tables(p, out, sc, l, s))) return rc;
        } else {
            return run_sparse(d_seq, p, out, sc, dirs, s, timed);
        }
        if (matrix) matrix_tables_from_zeros<<<1, kWave, 0, s>>>(SP + 2, p.L, Dm, d_zeros);
        if (dirs) {
            dim3 g((unsigned)cdiv(p.cap, kBlock), p.L);
            dir_finish<<<g, kBlock, 0, s>>>(nullptr, SP + 2, n, p.L, out->rank, p.rank_len, out->sel1, out->sel0,
                                            p.cap, out->sel_counts);
        }
    } else if (p.L > 0) {
        tables(two_phase ? (1ull << cbits) : (1ull << p.L), !two_phase);
    }
    if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
    if (n == 0 || p.L == 0) return WT_OK;
    if (pairs) return run_pairs(d_seq, p, out, sc, dirs, s, timed);

    const void *cur = d_seq;
    uint32_t cur_w = p.in_bytes;
    for (uint32_t l = 0; l < p.L; ++l) {
        if (two_phase && l == cbits) {
            // Fine phase over S_c (in `cur`), into the other buffer: the
            // rows, the overflow and later-segment counts, the tags; then
            // every count, C, and the tables of all levels.
            unsigned char *fb = (unsigned char *)((l % 2 == 0) ? (void *)(sc + p.off_S0) : (void *)(sc + p.off_S1));
            uint32_t *rows = (uint32_t *)fb;
            unsigned long long *extra = (unsigned long long *)(fb + 4 * fine_rows);
            uint32_t *tags = (uint32_t *)(fb + 4 * fine_rows + 8 * align_up(sigma, 32));
            zero_fill<<<(unsigned)std::min<uint64_t>(cdiv(sigma, kBlock), 4096), kBlock, 0, s>>>((uint64_t *)extra,
                                                                                                sigma, nullptr, 0);
            const uint64_t per = align_up(cdiv(n, fine_blocks), 4);
            hist_fine<<<fine_blocks, kFineThreads, 0, s>>>((const uint32_t *)cur, n, sigma, cbits, out->C, per, rows,
                                                           tags, extra, status);
            hist_fine_reduce<<<(unsigned)std::min<uint64_t>(cdiv(sigma, kBlock), 4096), kBlock, 0, s>>>(
                rows, tags, fine_blocks, extra, sigma, out->C + 1);
            c_scan();
            tables(1ull << p.L, true);
            if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
        }
        const bool scatter = l + 1 < p.L;
        void *dst = (l % 2 == 0) ? (void *)(sc + p.off_S0) : (void *)(sc + p.off_S1);
        // Tile prefixes of this level from the counts its predecessor left.
        const uint64_t Tl = cdiv(n, 1ull << tile_shift_for(cur_w));
        tile_prefixes(p, sc, l, Tl, s);
        LevelArgs a;
        a.in = cur;
        a.out = scatter ? dst : nullptr;
        a.bits = out->bits + (uint64_t)l * p.W;
        a.D = matrix ? Dm + 2ull * l : D + ((2ull << l) - 2);
        a.nD = matrix ? 2ull : 2ull << l;
        a.tile_prefix = pre + (uint64_t)l * p.T;
        a.next_cnt = scatter ? cnt + (uint64_t)(l + 1) * p.T : nullptr;
        a.next_shift = tile_shift_for(p.mid_bytes);
        a.status = status;
        a.rank = dirs ? out->rank + (uint64_t)l * p.rank_len : nullptr;
        a.sel1 = dirs ? out->sel1 + (uint64_t)l * p.cap : nullptr;
        a.sel0 = dirs ? out->sel0 + (uint64_t)l * p.cap : nullptr;
        a.n = n;
        a.k = p.L - 1 - l;
        a.level = l;
        a.fused_l0 = (fuse && l >= lmin) ? fused_l0 : nullptr;
        a.qmask = matrix ? 1u : ~0u;
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (timed && (rc = timing_begin(s, ev))) return rc;
        launch_level_any(cur_w, scatter ? p.mid_bytes : cur_w, scatter, dirs, s, a);
        if (timed && (rc = timing_end(s, ev))) return rc;
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
        cur = dst;
        cur_w = p.mid_bytes;
    }
    if (fuse) {
        FusedArgs f;
        f.in0 = d_seq;
        f.S0 = sc + p.off_S0;
        f.S1 = sc + p.off_S1;
        f.C = out->C;
        f.D = D;
        f.sigma = sigma;
        f.n = n;
        f.L = p.L;
        f.bits = out->bits;
        f.W = p.W;
        f.rank = out->rank;
        f.rank_len = p.rank_len;
        f.sel1 = out->sel1;
        f.sel0 = out->sel0;
        f.cap = p.cap;
        f.status = status;
        f.l0 = fused_l0;
        launch_fused(p.in_bytes, p.mid_bytes, f, n, s);
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
    }
    return WT_OK;
}

extern "C" int wt_build(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                        void *d_scratch, uint64_t scratch_bytes, void *stream) {
    return build_impl(d_seq, n, sigma, sym_bytes, out, false, nullptr, d_scratch, scratch_bytes, stream, g_timing);
}

extern "C" int wt_build_matrix(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                               uint64_t *d_zeros, void *d_scratch, uint64_t scratch_bytes, void *stream) {
    if (!d_zeros && levels_of(sigma) > 0) return WT_ERR_ARG;
    return build_impl(d_seq, n, sigma, sym_bytes, out, true, d_zeros, d_scratch, scratch_bytes, stream, g_timing);
}

extern "C" int wt_build_multiary(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes,
                                 const wt_multiary_outputs *out, void *d_scratch, uint64_t scratch_bytes,
                                 void *stream) {
    Plan p;
    int rc = make_plan(n, sigma, sym_bytes, p);
    if (rc) return rc;
    if (sym_bytes != 1 || n >= (1ull << 32)) return WT_ERR_RANGE;  // byte alphabets
    const uint32_t Lq = (p.L + 1) / 2;
    if (!out || !out->C || !d_scratch || (n > 0 && !d_seq)) return WT_ERR_ARG;
    if (Lq > 0 && (!out->rank4 || !out->sel4 || !out->counts4 || (n > 0 && !out->digits))) return WT_ERR_ARG;
    if (((uintptr_t)d_seq & 15u) || ((uintptr_t)d_scratch & 255u)) return WT_ERR_ARG;
    if (scratch_bytes < p.total) return WT_ERR_SCRATCH;
    hipStream_t s = (hipStream_t)stream;
    unsigned char *sc = (unsigned char *)d_scratch;
    uint32_t *status = (uint32_t *)(sc + p.off_status);
    uint32_t *cnt = (uint32_t *)(sc + p.off_cnt);
    uint64_t *pre = (uint64_t *)(sc + p.off_pre);
    uint64_t *part = (uint64_t *)(sc + p.off_part);
    uint32_t *E = (uint32_t *)(sc + p.off_E);
    {
        uint64_t na = p.off_pre / 8, nb = sigma + 1;
        uint64_t blocks = std::min<uint64_t>(cdiv(na + nb, kBlock), 4096);
        zero_fill<<<(unsigned)blocks, kBlock, 0, s>>>((uint64_t *)sc, na, out->C, nb);
    }
    if (n > 0) {
        // Digit counts of level 0 (bits 2Lq-1, 2Lq-2) per tile, and C.
        launch_hist<uint8_t>(d_seq, p, out->C + 1, status, cnt, sc + p.off_S0, Lq > 0, s, 2 * Lq - 1);
        CScanOp cop{out->C + 1};
        const uint64_t chunks = cdiv(sigma, kScanChunk);
        if (chunks > 1) {
            scan_reduce<CScanOp><<<(unsigned)chunks, kBlock, 0, s>>>(cop, sigma, part);
            scan_partials_seg<CScanOp><<<1, kBlock, 0, s>>>(cop, chunks, part);
            scan_final<CScanOp><<<(unsigned)chunks, kBlock, 0, s>>>(cop, sigma, part);
        } else {
            scan_final<CScanOp><<<1, kBlock, 0, s>>>(cop, sigma, nullptr);
        }
    }
    if (Lq == 0) return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
    const uint64_t W4 = cdiv(n, 32), R = cdiv(n, WT_RANK_BLOCK_BITS) + 1;
    digit_tables<<<Lq, kBlock, 0, s>>>(out->C, sigma, 2 * Lq - 2, E);
    quad_tails<<<Lq, kBlock, 0, s>>>(out->C, sigma, Lq, n, out->rank4, R, out->sel4, p.cap, out->counts4);
    if (n == 0) return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
    const uint32_t shift = tile_shift_for(1);
    const uint64_t Tl = cdiv(n, 1ull << shift);
    const void *cur = d_seq;
    for (uint32_t j = 0; j < Lq; ++j) {
        const bool scatter = j + 1 < Lq;
        void *dst = (j % 2 == 0) ? (void *)(sc + p.off_S0) : (void *)(sc + p.off_S1);
        pair_prefix_scan<<<1, kScanThreads, 0, s>>>((const uint64_t *)(cnt + 2ull * j * p.T),
                                                    (uint4 *)(pre + 2ull * j * p.T), Tl);
        QuadArgs a;
        a.in = (const uint8_t *)cur;
        a.out = scatter ? (uint8_t *)dst : nullptr;
        a.entries = (uint32_t *)(out->digits + (uint64_t)j * W4);
        a.nwords32 = 2 * W4;
        a.E = E + 256u * j;
        a.nkeys = 4u << (2u * j);
        a.pre = (const uint4 *)(pre + 2ull * j * p.T);
        a.next_cnt = scatter ? (uint64_t *)(cnt + 2ull * (j + 1) * p.T) : nullptr;
        a.next_shift = shift;
        a.status = status;
        a.rank4 = out->rank4 + (uint64_t)j * R * 4;
        a.sel4 = out->sel4 + (uint64_t)j * 4 * p.cap;
        a.cap = p.cap;
        a.n = (uint32_t)n;
        a.kq = 2 * (Lq - 1 - j);
        if (scatter) quad_pass<true><<<(unsigned)Tl, kBlock, 0, s>>>(a);
        else quad_pass<false><<<(unsigned)Tl, kBlock, 0, s>>>(a);
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
        cur = dst;
    }
    return WT_OK;
}

extern "C" int wt_build_rank_select(const uint64_t *d_bits, uint64_t n, uint32_t L, uint64_t *d_rank,
                                    uint64_t *d_sel1, uint64_t *d_sel0, uint64_t *d_sel_counts, void *d_scratch,
                                    uint64_t scratch_bytes, void *stream) {
    if (L == 0) return WT_OK;
    if (L > 30 || n >= (1ull << 40)) return WT_ERR_RANGE;
    if (!d_rank || !d_sel1 || !d_sel0 || !d_sel_counts || !d_scratch || (n > 0 && !d_bits)) return WT_ERR_ARG;
    if ((uintptr_t)d_scratch & 255u) return WT_ERR_ARG;
    if (scratch_bytes < wt_rank_select_scratch_bytes(n, L)) return WT_ERR_SCRATCH;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t W = cdiv(n, 64), T = cdiv(n, kDirTile), rank_len = cdiv(n, WT_RANK_BLOCK_BITS) + 1,
                   cap = cdiv(n, WT_SELECT_SAMPLE) + 1;
    unsigned char *sc = (unsigned char *)d_scratch;
    uint64_t *zeros_tot = (uint64_t *)sc;
    uint64_t *states = (uint64_t *)(sc + align_up(8ull * L, 256));
    uint64_t nz = wt_rank_select_scratch_bytes(n, L) / 8;
    zero_fill<<<(unsigned)std::min<uint64_t>(cdiv(nz, kBlock), 4096), kBlock, 0, s>>>((uint64_t *)sc, nz, nullptr,
                                                                                       0);
    if (T > 0) {
        dim3 g((unsigned)T, L);
        dir_tiles<<<g, kWave, 0, s>>>(d_bits, n, W, states, T, zeros_tot, d_rank, rank_len, d_sel1, d_sel0, cap,
                                      g_spin_limit);
    }
    dim3 g2((unsigned)cdiv(cap, kBlock), L);
    dir_finish<<<g2, kBlock, 0, s>>>(nullptr, zeros_tot, n, L, d_rank, rank_len, d_sel1, d_sel0, cap, d_sel_counts);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Huffman-shaped tree (byte alphabets): scratch = status block, per-tile
// zero counts and their prefixes for h_cap levels, two sequence buffers.
// The tables (HuffTab) are an output: the queries read them.
struct HuffPlan {
    uint64_t T, off_cnt, off_pre, off_S0, off_S1, total;
};

static uint32_t huff_height_bound(uint64_t n, uint64_t sigma) {
    if (n < 2 || sigma < 2) return 0;
    // a leaf at depth d needs F(d+2) symbols at least
    uint64_t f1 = 1, f2 = 1;  // F(d+1), F(d+2) for d = 0
    uint32_t d = 0;
    while (true) {
        const uint64_t f3 = f1 + f2;  // F(d+3)
        if (f3 > n) break;
        f1 = f2;
        f2 = f3;
        ++d;
    }
    return (uint32_t)std::min<uint64_t>(d, sigma - 1);
}

static HuffPlan huff_plan(uint64_t n, uint32_t h_cap) {
    HuffPlan p;
    p.T = align_up(std::max<uint64_t>(cdiv(n, 16384), 1), 64);
    uint64_t o = 256;
    p.off_cnt = o;
    o = align_up(o + 4ull * (h_cap + 1) * p.T, 256);
    p.off_pre = o;
    o = align_up(o + 8ull * (h_cap + 1) * p.T, 256);
    p.off_S0 = o;
    o = align_up(o + n, 256);
    p.off_S1 = o;
    o = align_up(o + n, 256);
    p.total = o;
    return p;
}

extern "C" int wt_huffman_plan(uint64_t n, uint64_t sigma, uint32_t h_cap, uint32_t *h_bound,
                               uint64_t *scratch_bytes, uint64_t *tables_bytes) {
    if (sigma == 0 || sigma > kHuffSyms || n >= (1ull << 32) || h_cap > (uint32_t)kHuffMaxLevels)
        return WT_ERR_RANGE;
    if (h_bound) *h_bound = huff_height_bound(n, sigma);
    if (scratch_bytes) *scratch_bytes = huff_plan(n, h_cap).total;
    if (tables_bytes) *tables_bytes = sizeof(HuffTab);
    return WT_OK;
}

extern "C" int wt_build_huffman(const void *d_seq, uint64_t n, uint64_t sigma, const wt_huffman_outputs *out,
                                uint32_t h_cap, uint32_t *h_out, void *d_scratch, uint64_t scratch_bytes,
                                void *stream) {
    if (sigma == 0 || sigma > kHuffSyms || n >= (1ull << 32) || h_cap > (uint32_t)kHuffMaxLevels)
        return WT_ERR_RANGE;
    if (!out || !out->C || !out->lens || !out->codes || !out->tables || !d_scratch || (n > 0 && !d_seq))
        return WT_ERR_ARG;
    if ((uintptr_t)out->tables & 15u) return WT_ERR_ARG;
    if (h_cap > 0 && (!out->bits || !out->rank || !out->sel1 || !out->sel0 || !out->sel_counts || !out->nd))
        return WT_ERR_ARG;
    if (((uintptr_t)d_seq & 15u) || ((uintptr_t)d_scratch & 255u)) return WT_ERR_ARG;
    Plan p;
    int rc = make_plan(n, sigma, 1, p);
    if (rc) return rc;
    const HuffPlan hp = huff_plan(n, h_cap);
    if (scratch_bytes < hp.total) return WT_ERR_SCRATCH;
    hipStream_t s = (hipStream_t)stream;
    unsigned char *sc = (unsigned char *)d_scratch;
    uint32_t *status = (uint32_t *)sc;
    HuffTab *tab = (HuffTab *)out->tables;
    uint32_t *cnt = (uint32_t *)(sc + hp.off_cnt);
    uint64_t *pre = (uint64_t *)(sc + hp.off_pre);
    // Zero: status and the per-tile counts; C.
    {
        const uint64_t na = hp.off_pre / 8, nb = sigma + 1;  // status and counts
        const uint64_t blocks = std::min<uint64_t>(cdiv(na + nb, kBlock), 4096);
        zero_fill<<<(unsigned)blocks, kBlock, 0, s>>>((uint64_t *)sc, na, out->C, nb);
    }
    if (n > 0) {
        launch_hist<uint8_t>(d_seq, p, out->C + 1, status, nullptr, sc + hp.off_S0, false, s);
        CScanOp cop{out->C + 1};  // sigma <= 256: one chunk
        scan_final<CScanOp><<<1, kBlock, 0, s>>>(cop, sigma, nullptr);
    }
    huff_codes<<<1, kHuffSyms, 0, s>>>(out->C, (uint32_t)sigma, tab);
    huff_levels<<<kHuffMaxLevels, kHuffSyms, 0, s>>>(tab);
    if (hipMemcpyAsync(out->lens, tab->lens, sizeof(tab->lens), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(out->codes, tab->codes, sizeof(tab->codes), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return WT_ERR_HIP;
    // The height and level sizes size the level passes: one wait.
    struct {
        uint32_t h, status;
        uint64_t nd[kHuffMaxLevels];
    } host{};
    if (hipMemcpyAsync(&host.h, &tab->h, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&host.status, status, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(host.nd, tab->nd, sizeof(host.nd), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return WT_ERR_HIP;
    const uint32_t h = host.h;
    if (h_out) *h_out = h;
    if (h > h_cap) return WT_ERR_RANGE;
    if (host.status || h == 0 || n == 0) return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
    if (hipMemcpyAsync(out->nd, tab->nd, sizeof(uint64_t) * h, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return WT_ERR_HIP;
    const uint64_t W = p.W;
    huff_count0<<<(unsigned)cdiv(n, 16384), kBlock, 0, s>>>((const uint8_t *)d_seq, n, tab, cnt);
    const uint8_t *cur = (const uint8_t *)d_seq;
    for (uint32_t d = 0; d < h; ++d) {
        const bool scatter = d + 1 < h;
        const uint64_t nd = host.nd[d];
        const uint64_t Tl = cdiv(nd, 16384);
        uint8_t *dst = (d % 2 == 0) ? sc + hp.off_S0 : sc + hp.off_S1;
        tile_prefix_scan<<<1, kScanThreads, 0, s>>>(cnt + (uint64_t)d * hp.T, pre + (uint64_t)d * hp.T, Tl);
        HuffArgs a;
        a.in = cur;
        a.out = scatter ? dst : nullptr;
        a.bits = out->bits + (uint64_t)d * W;
        a.lut = tab->lut[d];
        a.Dh = tab->Dh[d];
        a.tile_prefix = pre + (uint64_t)d * hp.T;
        a.next_cnt = scatter ? cnt + (uint64_t)(d + 1) * hp.T : nullptr;
        a.next_shift = 14;
        a.status = status;
        a.rank = out->rank + (uint64_t)d * p.rank_len;
        a.sel1 = out->sel1 + (uint64_t)d * p.cap;
        a.sel0 = out->sel0 + (uint64_t)d * p.cap;
        a.n = (uint32_t)nd;
        a.out_n = scatter ? (uint32_t)host.nd[d + 1] : 0u;
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (g_timing && (rc = timing_begin(s, ev))) return rc;
        if (scatter) launch_k(huff_level_pass<true, true>, dim3((unsigned)Tl), dim3(kBlock), s, a);
        else launch_k(huff_level_pass<false, true>, dim3((unsigned)Tl), dim3(kBlock), s, a);
        if (g_timing && (rc = timing_end(s, ev))) return rc;
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
        cur = dst;
    }
    {
        dim3 g((unsigned)std::max<uint64_t>(1, std::min<uint64_t>(cdiv(std::max(p.cap, W), kBlock), 1024)), h);
        huff_dir_finish<<<g, kBlock, 0, s>>>(tab, W, out->bits, out->rank, p.rank_len, out->sel1, out->sel0, p.cap,
                                             out->sel_counts);
    }
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

// ---------------------------------------------------------------------------
// sortWT (byte alphabets): scratch = status block, tile counts and starts per
// (level, key, tile), the L sorted copies of S, the directory builder's.
struct SortPlan {
    uint64_t T, off_cnt, off_base, off_S, off_rs, total;
};

static SortPlan sort_plan(uint64_t n, uint32_t L) {
    SortPlan p;
    p.T = std::max<uint64_t>(cdiv(n, kSortTile), 1);
    uint64_t o = 256;
    p.off_cnt = o;
    o = align_up(o + 4ull * L * kSortKeys * p.T, 256);
    p.off_base = o;
    o = align_up(o + 8ull * L * kSortKeys * p.T, 256);
    p.off_S = o;
    o = align_up(o + (uint64_t)L * align_up(n, 256), 256);
    p.off_rs = o;
    o = align_up(o + wt_rank_select_scratch_bytes(n, L), 256);
    p.total = o;
    return p;
}

extern "C" uint64_t wt_sort_scratch_bytes(uint64_t n, uint64_t sigma) {
    if (sigma == 0 || sigma > 256 || n >= (1ull << 32)) return 0;
    return sort_plan(n, levels_of(sigma)).total;
}

extern "C" int wt_build_sort(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                             void *d_scratch, uint64_t scratch_bytes, void *stream) {
    Plan p;
    int rc = make_plan(n, sigma, sym_bytes, p);
    if (rc) return rc;
    if (sym_bytes != 1 || n >= (1ull << 32)) return WT_ERR_RANGE;  // byte alphabets
    if (!out || !out->C || !d_scratch || (n > 0 && !d_seq)) return WT_ERR_ARG;
    if (p.L > 0 && (!out->rank || !out->sel1 || !out->sel0 || !out->sel_counts || (n > 0 && !out->bits)))
        return WT_ERR_ARG;
    if (((uintptr_t)d_seq & 15u) || ((uintptr_t)d_scratch & 255u)) return WT_ERR_ARG;
    const SortPlan sp = sort_plan(n, p.L);
    if (scratch_bytes < sp.total) return WT_ERR_SCRATCH;
    hipStream_t s = (hipStream_t)stream;
    unsigned char *sc = (unsigned char *)d_scratch;
    uint32_t *status = (uint32_t *)sc;
    {
        const uint64_t blocks = std::min<uint64_t>(cdiv(32 + sigma + 1, kBlock), 4096);
        zero_fill<<<(unsigned)blocks, kBlock, 0, s>>>((uint64_t *)sc, 32, out->C, sigma + 1);
    }
    if (n > 0) {
        launch_hist<uint8_t>(d_seq, p, out->C + 1, status, nullptr, sc + sp.off_S, false, s);
        CScanOp cop{out->C + 1};  // sigma <= 256: one chunk
        scan_final<CScanOp><<<1, kBlock, 0, s>>>(cop, sigma, nullptr);
    }
    if (p.L == 0) return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
    const uint64_t stride = align_up(n, 256);
    uint32_t *cnt = (uint32_t *)(sc + sp.off_cnt);
    uint64_t *base = (uint64_t *)(sc + sp.off_base);
    uint8_t *sorted = sc + sp.off_S;
    if (n > 0) {
        const dim3 gt((unsigned)sp.T, p.L), gk(kSortKeys, p.L);
        sort_count<<<gt, kBlock, 0, s>>>((const uint8_t *)d_seq, n, p.L, sp.T, cnt);
        sort_scan<<<gk, kBlock, 0, s>>>(cnt, out->C, sigma, p.L, sp.T, base);
        sort_scatter<<<gt, kBlock, 0, s>>>((const uint8_t *)d_seq, n, p.L, sp.T, base, sorted, stride);
        const dim3 gb((unsigned)cdiv(p.W, kBlock), p.L);
        sort_bits<<<gb, kBlock, 0, s>>>(sorted, n, p.L, stride, out->bits, p.W);
    }
    if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
    return wt_build_rank_select(out->bits, n, p.L, out->rank, out->sel1, out->sel0, out->sel_counts,
                                sc + sp.off_rs, sp.total - sp.off_rs, stream);
}

extern "C" int wt_histogram_path(uint64_t n, uint64_t sigma, int sym_bytes) {
    Plan p;
    const int rc = make_plan(n, sigma, sym_bytes, p);
    if (rc) return rc;
    return choose_path(p, false, true).hist;
}

extern "C" int wt_status_get(const void *d_scratch, void *stream) {
    if (!d_scratch) return WT_ERR_ARG;
    uint32_t st = 0;
    if (hipMemcpyAsync(&st, d_scratch, sizeof(st), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess)
        return WT_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return WT_ERR_HIP;
    return st == 0 ? WT_OK : (st == kStatusSymbol ? WT_ERR_SYMBOL : WT_ERR_HIP);
}

uint32_t wt::fused_levels_setting() { return g_fuse; }

extern "C" int wt_set_fused_levels(int levels) {
    if (levels < 0) return WT_ERR_ARG;
    g_fuse = (uint32_t)levels;
    return WT_OK;
}

extern "C" int wt_set_sliced_histogram(int enable) {
    g_slices = enable != 0;
    return WT_OK;
}

extern "C" int wt_set_level_pairs(int enable) {
    const int prev = g_pairs ? 1 : 0;
    g_pairs = enable != 0;
    return prev;
}

extern "C" int wt_set_lookback_spin_limit(int polls) {
    if (polls < 0) return WT_ERR_ARG;
    g_spin_limit = polls;
    return WT_OK;
}

extern "C" int wt_timing_enable(int enable) {
    g_timing = enable != 0;
    return WT_OK;
}

extern "C" int wt_timing_collect(float *ms, int cap) {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        evs.swap(g_events);
    }
    int count = (int)evs.size();
    int rc = count;
    for (int i = 0; i < count; ++i) {
        float t = 0.f;
        if (hipEventSynchronize(evs[i].second) != hipSuccess ||
            hipEventElapsedTime(&t, evs[i].first, evs[i].second) != hipSuccess)
            rc = WT_ERR_HIP;
        if (ms && i < cap) ms[i] = t;
    }
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_free.insert(g_free.end(), evs.begin(), evs.end());
    return rc;
}

// ---------------------------------------------------------------------------
// wt_build without allocation: the build's scratch is a file-scope device
// array, one copy per GPU for the life of the process.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): each device's address is looked up once with
// hipGetSymbolAddress, with that device current, and that address is what
// the kernels receive.
static __device__ __align__(256) unsigned char scratch[WT_NOALLOC_SCRATCH_BYTES];

namespace wt {

__global__ void status_to_code(const uint32_t *word, int32_t *code) {
    if (threadIdx.x == 0) *code = *word == 0 ? WT_OK : (*word == kStatusSymbol ? WT_ERR_SYMBOL : WT_ERR_HIP);
}

constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[kMaxDevices];  // device address of `scratch`, per device, once looked up

static int noalloc_scratch(void **ptr) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return WT_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return WT_ERR_RANGE;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p || ((uintptr_t)p & 255u))
            return WT_ERR_HIP;
        g_noalloc_ptr[dev] = p;
    }
    *ptr = g_noalloc_ptr[dev];
    return WT_OK;
}

}  // namespace wt

extern "C" int wt_build_noalloc(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                                int32_t *d_status, void *stream) {
    Plan p;
    int rc = make_plan(n, sigma, sym_bytes, p);
    if (rc) return rc;
    if (p.total > WT_NOALLOC_SCRATCH_BYTES) return WT_ERR_SCRATCH;
    void *sc = nullptr;
    if ((rc = noalloc_scratch(&sc))) return rc;
    // Untimed whatever this thread's timing switch says: timing creates events.
    rc = build_impl(d_seq, n, sigma, sym_bytes, out, false, nullptr, sc, WT_NOALLOC_SCRATCH_BYTES, stream, false);
    if (rc) return rc;
    if (d_status) {
        status_to_code<<<1, kWave, 0, (hipStream_t)stream>>>((const uint32_t *)sc, d_status);
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
    }
    return WT_OK;
}
