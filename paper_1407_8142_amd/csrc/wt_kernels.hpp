// Per-tile steps of levelWT (Fig. 1 of "Parallel Wavelet Tree Construction")
// on gfx950, shared by the single-sequence build (one kernel launch per step)
// and the batched build (one persistent kernel that runs the same steps as
// work items).  Every step here is a __device__ function run by one block of
// kBlock threads on one tile; its LDS is a struct the caller provides, so a
// kernel that runs several kinds of steps can overlay them in one union.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include "../../include/wt.h"
#include "wt_device.hpp"

namespace wt {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kWaves = kBlock / kWave;
constexpr int kScanChunk = kBlock * kItems;  // elements per block in the generic scans

constexpr uint32_t kStatusSymbol = 2u;

// Host switch of the fused tail levels (wt_set_fused_levels): 0 none, 1 from
// the first level whose nodes fit, m >= 2 at most the last m levels.
uint32_t fused_levels_setting();

__host__ __device__ inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline uint64_t align_up(uint64_t a, uint64_t b) { return cdiv(a, b) * b; }

// Positions per tile of a level whose sequence has `width`-byte symbols:
// a tile is 16 KiB whatever the width.
__host__ __device__ inline uint32_t tile_shift_for(uint32_t width) {
    return width == 1 ? 14u : (width == 2 ? 13u : 12u);
}

// Sum of one value per thread over the block (result valid in every thread).
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t *red) {
    const int lane = lane_id(), wave = (int)threadIdx.x / kWave;
    const uint32_t w = (uint32_t)wave_sum_u64(v);
    __syncthreads();
    if (lane == 0) red[wave] = w;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += red[i];
    return t;
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *red) {
    const int lane = lane_id(), wave = (int)threadIdx.x / kWave;
    const uint64_t w = wave_sum_u64(v);
    __syncthreads();
    if (lane == 0) red[wave] = w;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += red[i];
    return t;
}

// ---------------------------------------------------------------------------
// Histogram of one tile: the counts behind C (C[c] = #{S[i] < c}), the
// symbol check, and the zeros of the top bit in the tile (the count-ahead
// input of level 0).  Each thread reads 16 bytes at a time.
//   Small alphabets (reps > 0) count in LDS: `reps` replicas with a stride
//   of sigma+1 words (replicas of one symbol fall in different banks, the
//   lane picks its replica), one LDS atomic per symbol and no branches; a
//   symbol >= sigma is clamped into the pad word and raises the flag.
//   Large alphabets aggregate every kH/2 symbols in an LDS hash table of kH
//   slots (so skewed data does not hammer a few global counters) and flush
//   one global atomic per distinct symbol.
// LDS: `tab` holds reps*(sigma+1) words, or keys[kH] | vals[kH] | used[kH/2].
template <uint32_t kH>
struct HistHash {
    static constexpr uint32_t kChunk = kH / 2, kEmpty = 0xFFFFFFFFu;
    static constexpr uint32_t kWords = 2 * kH + kChunk;
};

template <uint32_t kH>
__device__ __forceinline__ void hist_init(uint32_t *tab, uint32_t *nused, uint32_t reps, uint64_t sigma) {
    const int tid = threadIdx.x;
    if (reps) {
        for (uint64_t i = tid; i < (sigma + 1) * reps; i += kBlock) tab[i] = 0;
    } else {
        for (uint32_t i = tid; i < kH; i += kBlock) {
            tab[i] = HistHash<kH>::kEmpty;
            tab[kH + i] = 0;
        }
        if (tid == 0) *nused = 0;
    }
    __syncthreads();
}

// Digit counts packed as (c0 | c1 << 16 | c2 << 32), digit = (x >> lo) & 3
// (bit lo+1 high, bit lo low); the fourth count is implied by the total.
// A tile holds at most 2^14 symbols, so per-tile sums never carry.
__device__ __forceinline__ uint64_t digit_inc(uint32_t x, uint32_t lo) {
    const uint32_t d = (x >> lo) & 3u;
    return d < 3u ? 1ull << (16u * d) : 0ull;
}

// Counts S[base, base+len) into the LDS table (hash path: flushed to
// `counts` every kH/2 symbols).  Returns this thread's zeros of bit ktop,
// or with DIG its packed counts of the digit (bit ktop, bit ktop-1).
template <typename T, uint32_t kH, typename CNT, bool DIG = false>
__device__ __forceinline__ std::conditional_t<DIG, uint64_t, uint32_t> hist_count(const T *__restrict__ S, uint64_t base, uint32_t len, uint64_t sigma,
                                               uint32_t reps, uint32_t ktop, uint32_t *tab, uint32_t *nused,
                                               CNT *counts, bool &bad) {
    using H = HistHash<kH>;
    const int tid = threadIdx.x, lane = lane_id();
    const bool lds = reps > 0;
    uint32_t *keys = tab, *vals = tab + kH, *used = tab + 2 * kH;
    uint32_t *s_hist = lds ? tab + (uint64_t)(lane % reps) * (sigma + 1) : nullptr;
    const uint32_t smax = (uint32_t)min(sigma, (uint64_t)0xFFFFFFFFu);
    const bool need_check = sigma < (1ull << (8 * sizeof(T)));
    constexpr int V = 16 / sizeof(T);
    // Replica path: `c` occurrences of symbol s at once.
    auto add_run = [&](uint32_t s, uint32_t c) {
        uint32_t bin = s;
        if (need_check) {
            bad |= s >= smax;
            bin = min(s, smax);
        }
        atomicAdd(s_hist + bin, c);
    };
    auto tally = [&](uint32_t x) -> std::conditional_t<DIG, uint64_t, uint32_t> {
        if constexpr (DIG) return digit_inc(x, ktop - 1u);
        else return ((x >> ktop) & 1u) ^ 1u;
    };
    auto visit = [&](uint32_t s) -> std::conditional_t<DIG, uint64_t, uint32_t> {
        if (lds) {
            add_run(s, 1u);
        } else if ((uint64_t)s >= sigma) {
            bad = true;
        } else if (s == H::kEmpty) {
            // 2^32 - 1 (sigma = 2^32) is the table's empty key: counted directly.
            atomicAdd(counts + s, (CNT)1);
        } else {
            uint32_t h = (s * 0x9E3779B1u) >> (32 - __builtin_ctz(kH));
            bool done = false;
#pragma unroll 1
            for (int probe = 0; probe < 8; ++probe) {
                const uint32_t old = atomicCAS(keys + h, H::kEmpty, s);
                if (old == H::kEmpty) used[atomicAdd(nused, 1u)] = h;
                if (old == H::kEmpty || old == s) {
                    atomicAdd(vals + h, 1u);
                    done = true;
                    break;
                }
                h = (h + 1) & (kH - 1);
            }
            if (!done) atomicAdd(counts + s, (CNT)1);
        }
        return tally(s);
    };
    std::conditional_t<DIG, uint64_t, uint32_t> zeros = 0;
    const uint32_t chunk = lds ? len : H::kChunk;  // hash path: at most kH/2 symbols per flush
    for (uint32_t c0 = 0; c0 < len; c0 += chunk) {
        const uint32_t clen = clamp_count(len, c0, chunk);
        if (clen % V == 0 && ((base + c0) % V) == 0) {
            // kU 16-byte loads per thread are issued before any is counted,
            // so that their HBM latencies overlap.
            constexpr int kU = 4;
            const uint32_t nvec = clen / V;
            for (uint32_t v0 = tid; v0 < nvec; v0 += kBlock * kU) {
                union {
                    uint4 q;
                    T e[V];
                } u[kU];
                const uint4 *src = reinterpret_cast<const uint4 *>(S + base + c0) + v0;
                if (v0 + (uint32_t)((kU - 1) * kBlock) < nvec) {  // all in range: no branch between the loads
#pragma unroll
                    for (int k = 0; k < kU; ++k) u[k].q = src[k * kBlock];
                } else {
#pragma unroll
                    for (int k = 0; k < kU; ++k)
                        u[k].q = v0 + (uint32_t)(k * kBlock) < nvec ? src[k * kBlock] : make_uint4(0, 0, 0, 0);
                }
#pragma unroll
                for (int k = 0; k < kU; ++k) {
                    if (v0 + (uint32_t)(k * kBlock) >= nvec) continue;
                    if (lds) {
                        // Runs of equal symbols in the group take one atomic
                        // each (text has many short runs).
                        uint32_t prev = (uint32_t)u[k].e[0], run = 1;
                        zeros += tally(prev);
#pragma unroll
                        for (int j = 1; j < V; ++j) {
                            const uint32_t x = (uint32_t)u[k].e[j];
                            zeros += tally(x);
                            if (x == prev) {
                                ++run;
                            } else {
                                add_run(prev, run);
                                prev = x;
                                run = 1;
                            }
                        }
                        add_run(prev, run);
                    } else {
#pragma unroll
                        for (int j = 0; j < V; ++j) zeros += visit((uint32_t)u[k].e[j]);
                    }
                }
            }
        } else {
            for (uint32_t e = tid; e < clen; e += kBlock) zeros += visit((uint32_t)S[base + c0 + e]);
        }
        if (!lds) {
            __syncthreads();
            const uint32_t nu = *nused;
            for (uint32_t i = tid; i < nu; i += kBlock) {
                const uint32_t h = used[i];
                atomicAdd(counts + keys[h], (CNT)vals[h]);
                keys[h] = H::kEmpty;
                vals[h] = 0;
            }
            __syncthreads();
            if (tid == 0) *nused = 0;
            __syncthreads();
        }
    }
    return zeros;
}

// Replica path: one global atomic per symbol present.
template <typename CNT>
__device__ __forceinline__ void hist_flush_replicas(const uint32_t *tab, uint32_t reps, uint64_t sigma,
                                                    CNT *counts) {
    __syncthreads();
    for (uint64_t c = threadIdx.x; c < sigma; c += kBlock) {
        uint32_t sum = 0;
        for (uint32_t r = 0; r < reps; ++r) sum += tab[(uint64_t)r * (sigma + 1) + c];
        if (sum) atomicAdd(counts + c, (CNT)sum);
    }
}

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of kItems values per thread (blocked layout).
struct BlockScanTmp {
    uint64_t wave_tot[kWaves];
};

template <int N = kItems>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t (&v)[N], BlockScanTmp &tmp, uint64_t &total) {
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    uint64_t own = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) own += v[j];
    uint64_t inc = wave_incl_scan_u64(own, lane);
    if (lane == kWave - 1) tmp.wave_tot[wave] = inc;
    __syncthreads();
    uint64_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        uint64_t t = tmp.wave_tot[w];
        if (w < wave) before += t;
        total += t;
    }
    __syncthreads();
    uint64_t run = before + inc - own;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        uint64_t x = v[j];
        v[j] = run;
        run += x;
    }
    return before + inc - own;
}

// One block scans `count` values, N per thread at a time:
// store(g, value(0) + ... + value(g-1)) for every g < count.  Returns the total.
template <int N, typename Val, typename Store>
__device__ __forceinline__ uint64_t block_scan_all(uint64_t count, BlockScanTmp &tmp, Val value, Store store) {
    uint64_t carry = 0;
    for (uint64_t c0 = 0; c0 < count; c0 += (uint64_t)kBlock * N) {
        const uint64_t base = c0 + (uint64_t)threadIdx.x * N;
        uint64_t v[N];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = base + j < count ? value(base + j) : 0;
        uint64_t total;
        block_excl_scan<N>(v, tmp, total);
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (base + j < count) store(base + j, carry + v[j]);
        carry += total;
    }
    return carry;
}

// ---------------------------------------------------------------------------
// Node tables.  Element g in [1, 2^L) is node p = g - 2^l of level l =
// floor(log2 g) (heap numbering from 1).  Its value is the ones of B_l
// inside node p = the symbols of its range whose bit k_l is 1 = C[end] -
// C[middle]; the exclusive scan of these values inside each level gives
//   D_l[2p]   = ones of B_l before node p,
//   D_l[2p+1] = zeros of B_l before node p+1,
// stored at D[2g-2] and D[2g-1] (level l occupies D[2^(l+1)-2, 2^(l+2)-2)).
struct TableOp {
    const uint64_t *C;
    uint64_t *D;
    uint64_t sigma;
    uint32_t L;
    __device__ static uint32_t level_of(uint64_t g) { return 63u - (uint32_t)__clzll((long long)g); }
    __device__ uint64_t Cc(uint64_t x) const { return C[x < sigma ? x : sigma]; }
    __device__ uint64_t value(uint64_t g) const {
        if (g == 0) return 0;
        uint32_t l = level_of(g), k = L - 1 - l;
        uint64_t p = g - (1ull << l);
        return Cc((p + 1) << (k + 1)) - Cc(((2 * p + 1) << k));
    }
    __device__ void store(uint64_t g, uint64_t ex) const {
        if (g == 0) return;
        uint32_t l = level_of(g), k = L - 1 - l;
        uint64_t p = g - (1ull << l);
        uint64_t ones = Cc((p + 1) << (k + 1)) - Cc(((2 * p + 1) << k));
        D[2 * g - 2] = ex;                                  // ones before node p
        D[2 * g - 1] = Cc((p + 1) << (k + 1)) - (ex + ones);  // zeros before node p+1
    }
    __device__ uint64_t seg_start(uint64_t g) const { return g == 0 ? 0 : (1ull << level_of(g)); }
    __device__ uint64_t chunk_seg_first(uint64_t c) const {
        // chunks >= 1 hold one level each; a level with several chunks
        // starts at chunk 2^(l-12) for 4096-element chunks.
        if (c == 0) return 0;
        return 1ull << (63u - (uint32_t)__clzll((long long)c));
    }
};

// Level l's node table (the values TableOp gives) for one job by one block,
// and the level's largest node.  Each node's C values are loaded once, a
// whole round's loads issued before any is used (the loads are the latency
// of this loop, not the arithmetic).  Returns the largest node in every
// thread.
template <int N>
__device__ __forceinline__ uint64_t table_level_block(const uint64_t *C, uint64_t sigma, uint32_t L, uint32_t l,
                                                      uint64_t *D, BlockScanTmp &tmp, unsigned long long *red) {
    const uint32_t k = L - 1 - l;
    const uint64_t P = 1ull << l;
    uint64_t *Dl = D + (2ull << l) - 2;  // D_l[2p] = ones before node p, D_l[2p+1] = zeros before node p+1
    auto Cc = [&](uint64_t x) { return C[x < sigma ? x : sigma]; };
    uint64_t carry = 0, big = 0;
    for (uint64_t c0 = 0; c0 < P; c0 += (uint64_t)kBlock * N) {
        const uint64_t base = c0 + (uint64_t)threadIdx.x * N;
        uint64_t ce[N], cm[N], v[N];
        const uint64_t cs = base < P ? Cc(base << (k + 1)) : 0;  // start of the thread's first node
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const uint64_t p = base + j < P ? base + j : P - 1;
            ce[j] = Cc((p + 1) << (k + 1));
            cm[j] = Cc((2 * p + 1) << k);
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            v[j] = base + j < P ? ce[j] - cm[j] : 0;  // ones of node p
            const uint64_t start = j == 0 ? cs : ce[j - 1];
            if (base + j < P) big = max(big, ce[j] - start);
        }
        uint64_t ones[N];
#pragma unroll
        for (int j = 0; j < N; ++j) ones[j] = v[j];
        uint64_t total;
        block_excl_scan<N>(v, tmp, total);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (base + j >= P) continue;
            const uint64_t p = base + j, ex = carry + v[j];
            Dl[2 * p] = ex;
            Dl[2 * p + 1] = ce[j] - (ex + ones[j]);
        }
        carry += total;
    }
    // largest node: wave maxima, then the block's
    for (int d = kWave / 2; d >= 1; d >>= 1) big = max(big, (uint64_t)__shfl_xor(big, d, kWave));
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x / kWave] = big;
    __syncthreads();
    uint64_t m = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) m = max(m, (uint64_t)red[w]);
    __syncthreads();
    return m;
}

// Directory tail of level l: rank[last] = ones of the level, the sample
// counts, and the sample entries at or past the counts set to n.  Thread t
// of `nthreads` handles sample entries t, t + nthreads, ...
__device__ __forceinline__ void dir_tail(uint32_t l, uint64_t zeros, uint64_t n, uint32_t L, uint64_t *rank,
                                         uint64_t rank_len, uint64_t *sel1, uint64_t *sel0, uint64_t cap,
                                         uint64_t *sel_counts, uint64_t t, uint64_t nthreads) {
    const uint64_t ones = n - zeros;
    const uint64_t c1 = cdiv(ones, WT_SELECT_SAMPLE), c0 = cdiv(zeros, WT_SELECT_SAMPLE);
    if (t == 0) {
        rank[(uint64_t)l * rank_len + rank_len - 1] = ones;
        sel_counts[l] = c1;
        sel_counts[L + l] = c0;
    }
    for (uint64_t e = min(c1, c0) + t; e < cap; e += nthreads) {
        if (e >= c1) sel1[(uint64_t)l * cap + e] = n;
        if (e >= c0) sel0[(uint64_t)l * cap + e] = n;
    }
}

// ---------------------------------------------------------------------------
// Level pass, one tile.
//
// A tile is 16 KiB of the level's sequence whatever the symbol width, so one
// block has enough bytes in flight to cover HBM latency.  The 256 threads
// hold the tile packed in 16 registers each (item r of thread t is position
// r*256 + t), which frees the LDS stage for the split.
template <typename T>
struct TileCfg {
    static constexpr int kBytes = 16384;
    static constexpr int kItems = kBytes / (kBlock * (int)sizeof(T));  // per thread
    static constexpr int kTile = kBlock * kItems;                       // positions
    static constexpr int kWords = kTile / 64;                           // level words
    static constexpr int kWPL = kWords / kWave;                         // words per lane of wave 0
    static constexpr int kPer = 4 / (int)sizeof(T);                     // symbols per packed register
    static constexpr int kRegs = kItems / kPer;
};
constexpr int kMinTile = TileCfg<uint32_t>::kTile;  // smallest tile: sizes the per-tile arrays
constexpr int kSmallD = 512;                        // node tables up to this size are cached in LDS

struct LevelArgs {
    const void *in;          // S_l (TIN), 16-byte aligned
    void *out;               // S_{l+1} (TOUT)
    uint64_t *bits;          // B_l
    uint64_t *next_bits = nullptr;  // B_{l+1}, written by the pass of level L-2 (LASTBITS)
    // Byte passes with PIECES: zeros of B_l before each piece of the level
    // (tile + node; see wt_stats.hpp) instead of tile_prefix: a tile's own
    // prefix is the one of its first piece, found from its first symbol.
    const uint32_t *piece_prefix = nullptr;
    const uint64_t *node_starts = nullptr;  // the last level's directory pass: its node starts
    uint32_t nodes = 0;                     // (2^(L-1) + 1 of them)
    const uint64_t *D;       // D_l: 2^(l+1) entries
    uint64_t nD;             // 2^(l+1)
    const uint64_t *tile_prefix;  // zeros of B_l before each tile of this level
    uint32_t *next_cnt;      // zeros of B_{l+1} per tile of the next level (accumulated here)
    uint32_t next_shift;     // log2(positions per tile of the next level)
    const uint32_t *status;  // non-zero: input rejected, do nothing
    uint64_t *rank, *sel1, *sel0;  // directory rows of level l
    uint64_t n;
    uint32_t k;              // bit examined at this level: L-1-l
    uint32_t level;          // l
    const uint32_t *fused_l0;  // levels >= *fused_l0 are done by the fused pass (NULL: none)
    uint32_t qmask;          // node index = (symbol >> k) & qmask: ~0 for the tree (node and bit),
                             // 1 for the wavelet matrix (one node per level, D = {0, zeros})
    // tails != 0: the blocks also write level l's directory tail (last rank
    // entry, sample counts, sample entries past the counts), from the level's
    // zeros = D[nD - 1]; sel_counts is the whole [2L] array.
    uint32_t tails = 0, L = 0;
    uint64_t *sel_counts = nullptr;
    uint64_t rank_len = 0, cap = 0;
};

// Count-ahead: while level l scatters S_{l+1}, it also counts, for every tile
// of level l+1, the zeros that tile will hold (bit k-1 of the symbols that
// land in it).  A scan of those counts gives each tile of level l+1 its
// exclusive zero prefix before level l+1 starts, so no tile ever waits for
// another.  Each lane keeps a running count for the destination tile it is
// filling and hands it to a small LDS table keyed by destination tile when
// that tile changes (a block's runs touch few tiles); the table reaches HBM
// as one atomic add per touched tile when the block ends, and a table that
// is full falls back to a direct atomic.
constexpr int kCountSlots = 64;
constexpr uint32_t kNoTile = 0xFFFFFFFFu;
// LOG2: log2 of the slot count (the byte pass, whose blocks touch only a
// few destination tiles, takes 32 slots to fit one more block per CU).
template <int LOG2>
struct CountTableN {
    static constexpr int kSlots = 1 << LOG2;
    uint32_t key[kSlots];
    uint32_t cnt[kSlots];
};
using CountTable = CountTableN<6>;
static_assert(CountTable::kSlots == kCountSlots, "pair tables share the slot count");

template <int LOG2>
__device__ __forceinline__ void count_init(CountTableN<LOG2> &t, int tid) {
    if (tid < CountTableN<LOG2>::kSlots) {
        t.key[tid] = kNoTile;
        t.cnt[tid] = 0;
    }
}

template <int LOG2>
__device__ __forceinline__ void count_add(CountTableN<LOG2> &t, uint32_t *next_cnt, uint32_t ntile, uint32_t c) {
    // Hashed slot with a short linear probe: the tiles one block touches are
    // few but can be far apart by large powers of two (a run of zeros and a
    // run of ones half a level apart), so the low bits alone would collide.
    uint32_t slot = (ntile * 0x9E3779B9u) >> (32 - LOG2);
#pragma unroll 1
    for (int probe = 0; probe < 8; ++probe) {
        const uint32_t old = atomicCAS(&t.key[slot], kNoTile, ntile);
        if (old == kNoTile || old == ntile) {
            atomicAdd(&t.cnt[slot], c);
            return;
        }
        slot = (slot + 1) & (CountTableN<LOG2>::kSlots - 1);
    }
    atomicAdd(next_cnt + ntile, c);
}

template <int LOG2>
__device__ __forceinline__ void count_flush(CountTableN<LOG2> &t, uint32_t *next_cnt, int tid) {
    if (tid < CountTableN<LOG2>::kSlots && t.key[tid] != kNoTile && t.cnt[tid])
        atomicAdd(next_cnt + t.key[tid], t.cnt[tid]);
}

// Hands every lane's (tile, c) with `want` set to the table with one update
// per distinct tile of the wave: the lanes of a wave mostly fill the same
// destination tile, and 64 lanes updating one LDS slot would serialize.
// Called by all lanes of the wave.
template <int LOG2>
__device__ __forceinline__ void count_add_wave(CountTableN<LOG2> &t, uint32_t *next_cnt, bool want, uint32_t tile,
                                               uint32_t c, int lane) {
    uint64_t pend = __ballot(want);
    while (pend) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const uint32_t kt = (uint32_t)__builtin_amdgcn_readlane((int)tile, leader);
        const bool mine = want && tile == kt;
        const uint32_t tot = wave_sum_u32(mine ? c : 0u);
        if (lane == leader) count_add(t, next_cnt, kt, tot);
        pend &= ~__ballot(mine);
    }
}

// Per-lane running count for one destination tile.
struct LaneCount {
    uint32_t tile = kNoTile, cnt = 0;
    template <int LOG2>
    __device__ __forceinline__ void add(CountTableN<LOG2> &t, uint32_t *next_cnt, uint32_t ntile, uint32_t c) {
        if (ntile != tile) {
            if (cnt) count_add(t, next_cnt, tile, cnt);
            tile = ntile;
            cnt = 0;
        }
        cnt += c;
    }
    // As add, but a finished tile's count is returned in (ftile, fcnt) for a
    // wave-wide hand-over instead of going to the table.
    __device__ __forceinline__ void step(uint32_t ntile, uint32_t c, uint32_t &ftile, uint32_t &fcnt) {
        if (ntile != tile) {
            ftile = tile;
            fcnt = cnt;
            tile = ntile;
            cnt = 0;
        }
        cnt += c;
    }
    template <int LOG2>
    __device__ __forceinline__ void flush(CountTableN<LOG2> &t, uint32_t *next_cnt) {
        if (cnt) count_add(t, next_cnt, tile, cnt);
        cnt = 0;
    }
    // flush by all lanes of the wave
    template <int LOG2>
    __device__ __forceinline__ void flush_wave(CountTableN<LOG2> &t, uint32_t *next_cnt, int lane) {
        count_add_wave(t, next_cnt, cnt != 0, tile, cnt, lane);
        cnt = 0;
    }
};

template <typename TIN>
struct LdsLevel {
    __align__(16) unsigned char stage[TileCfg<TIN>::kBytes];
    uint64_t words[TileCfg<TIN>::kWords];
    uint32_t zpre[TileCfg<TIN>::kWords];
    uint64_t D[kSmallD];
    uint64_t Z0;
    uint32_t Zt;
    CountTable ct;
};

// Generic widths (TIN, TOUT in {1, 2, 4} bytes).  The caller synchronises
// the block before reusing `s`.
template <typename TIN, typename TOUT, bool SCATTER, bool DIRS>
__device__ __forceinline__ void level_tile(const LevelArgs &a, uint64_t tile, LdsLevel<TIN> &s) {
    using Cfg = TileCfg<TIN>;
    constexpr int kTile = Cfg::kTile, kIt = Cfg::kItems, kWPL = Cfg::kWPL;
    constexpr int V = 16 / sizeof(TIN);

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint64_t t0 = tile * kTile;
    const uint32_t len = (uint32_t)min((uint64_t)kTile, a.n - t0);
    const uint32_t k = a.k;
    const bool d_lds = SCATTER && a.nD <= (uint64_t)kSmallD;

    // 1. Coalesced 16-byte loads of the tile into LDS (a whole tile's loads
    //    back to back, the node table after them, so the latencies overlap).
    TIN *stage_in = reinterpret_cast<TIN *>(s.stage);
    const TIN *in = reinterpret_cast<const TIN *>(a.in) + t0;
    if (len == (uint32_t)kTile) {
        // The node table's two loads (indices clamped into the table; LDS
        // entries past nD are unused) go out first and land in LDS only after
        // the tile's loads are issued: one wait covers all six.
        // No branch around them (s.D is read only when the table is cached).
        static_assert(kSmallD == 2 * kBlock, "node table fill is two steps");
        uint64_t d0 = 0, d1 = 0;
        if (SCATTER) {
            const uint64_t last = a.nD - 1;
            d0 = a.D[min((uint64_t)tid, last)];
            d1 = a.D[min((uint64_t)(tid + kBlock), last)];
        }
        uint4 q[kIt / V];
#pragma unroll
        for (int r = 0; r < kIt / V; ++r) q[r] = *reinterpret_cast<const uint4 *>(in + (r * kBlock + tid) * V);
        if (SCATTER) {
            s.D[tid] = d0;
            s.D[tid + kBlock] = d1;
        }
#pragma unroll
        for (int r = 0; r < kIt / V; ++r) *reinterpret_cast<uint4 *>(stage_in + (r * kBlock + tid) * V) = q[r];
    } else {
        for (uint32_t e = tid; e < len; e += kBlock) stage_in[e] = in[e];
        if (d_lds)
            for (int i = tid; i < (int)a.nD; i += kBlock) s.D[i] = a.D[i];
    }
    if (SCATTER) count_init(s.ct, tid);
    // Flags uniform across the grid, tested once the tile's loads are in
    // flight (nothing has been written to global memory yet): the input was
    // rejected, or this level is left to the fused pass.
    if (*a.status) return;
    if (a.fused_l0 && a.level >= *a.fused_l0) return;
    __syncthreads();

    // 2. Striped view: item r of wave w, lane j is position r*256 + 64w + j,
    //    so each ballot is one position-ordered word of B_l (word 4r + w).
    uint32_t pk[Cfg::kRegs];
#pragma unroll
    for (int i = 0; i < Cfg::kRegs; ++i) pk[i] = 0;
#pragma unroll
    for (int r = 0; r < kIt; ++r) {
        uint32_t e = (uint32_t)(r * kBlock + tid);
        bool valid = e < len;
        uint32_t sym = valid ? (uint32_t)stage_in[e] : 0u;
        pk[r / Cfg::kPer] |= sym << (8 * sizeof(TIN) * (r % Cfg::kPer));
        bool bit = valid && ((sym >> k) & 1u);
        uint64_t vm = __ballot(valid);
        uint64_t w = __ballot(bit);
        if (lane == 0) {
            s.words[r * kWaves + wave] = w;
            s.zpre[r * kWaves + wave] = (uint32_t)(__popcll(vm) - __popcll(w));
        }
    }
    __syncthreads();

    // 3. Wave 0: scan of the word zero-counts, bit words to HBM, directory
    //    entries.
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
        uint32_t inc = wave_incl_scan_u32(own, lane);
        uint32_t Zt = __shfl(inc, kWave - 1, kWave);
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
            uint32_t w = (uint32_t)lane * kWPL + m;
            if (w * 64u < len) a.bits[(t0 >> 6) + w] = wd[m];
        }
        if (DIRS) emit_directories<kWPL>(wd, zp, Z0, t0, len, Zt, a.n, a.rank, a.sel1, a.sel0, lane);
    }
    if (!SCATTER) return;
    __syncthreads();
    const uint64_t Z0 = s.Z0;
    const uint32_t Zt = s.Zt;

    // 4. Stable split of the tile by the level bit into LDS: zeros keep their
    //    order at [0, Zt), ones at [Zt, len).  Inside each region the
    //    elements stay grouped by node, and each node's group lands on
    //    consecutive positions of S_{l+1}.
    TOUT *stage_out = reinterpret_cast<TOUT *>(s.stage);
    const uint64_t lt = lanemask_lt(lane);
#pragma unroll
    for (int r = 0; r < kIt; ++r) {
        uint32_t e = (uint32_t)(r * kBlock + tid);
        if (e < len) {
            uint64_t w = s.words[r * kWaves + wave];
            uint32_t zl = s.zpre[r * kWaves + wave] + (uint32_t)__popcll(~w & lt);
            uint32_t slot = ((w >> lane) & 1ull) ? Zt + (e - zl) : zl;
            uint32_t sym = (pk[r / Cfg::kPer] >> (8 * sizeof(TIN) * (r % Cfg::kPer))) &
                           (uint32_t)((1ull << (8 * sizeof(TIN))) - 1ull);
            stage_out[slot] = (TOUT)sym;
        }
    }
    __syncthreads();

    // 5. Scatter.  Position s of the split tile holds a zero of node p iff
    //    s < Zt; its destination is D[2p] + (zeros before it on the level)
    //    for a zero and D[2p+1] + (ones before it) for a one -- Fig. 1's
    //    start + X[i] and start + X_s + i - X[i] with the node-relative
    //    counts rebased to level-wide counts through the tables.
    TOUT *out = reinterpret_cast<TOUT *>(a.out);
    const uint64_t O0 = t0 - Z0;
    const uint32_t kn = k - 1;  // bit of the next level
    LaneCount lc;
#pragma unroll 4
    for (int r = 0; r < kIt; ++r) {
        uint32_t sp = (uint32_t)(r * kBlock + tid);
        if (sp < len) {
            TOUT v = stage_out[sp];
            uint64_t q = (uint64_t)(((uint32_t)v >> k) & a.qmask);
            if (q < a.nD) {
                uint64_t base = d_lds ? s.D[q] : a.D[q];
                uint64_t dest = base + (sp < Zt ? Z0 + sp : O0 + (sp - Zt));
                if (dest < a.n) {
                    out[dest] = v;
                    lc.add(s.ct, a.next_cnt, (uint32_t)(dest >> a.next_shift), (((uint32_t)v >> kn) & 1u) ^ 1u);
                }
            }
        }
    }
    lc.flush_wave(s.ct, a.next_cnt, lane);
    __syncthreads();
    count_flush(s.ct, a.next_cnt, tid);
}

// ---------------------------------------------------------------------------
// Level pass for byte symbols (n < 2^32): the same steps as level_tile with
// SWAR arithmetic, since at HBM rate a byte symbol leaves only about ten
// lane operations per level.  A tile is 4 rows of 4096 bytes; thread t owns
// bytes [16t, 16t+16) of every row as four dwords.
//   bits:  a 4x4 byte transpose (v_perm) lines bit k of the 16 bytes up so
//          that a few shifts and ORs give them as a 16-bit mask in position
//          order; four lanes' masks are one word of B_l, so the LDS array of
//          masks read as 64-bit words *is* the tile's slice of B_l.
//   scan:  two rows per 32-bit value (16-bit fields), one wave scan each.
//   split: bytes go to their LDS slot one at a time.
//   scatter: sixteen slots per lane; inside one run (same node, same bit)
//          they have consecutive destinations and leave as one (possibly
//          unaligned) 16-byte store.
typedef uint32_t u128_unaligned __attribute__((ext_vector_type(4), aligned(1)));

// A + 2^(s mod 32): v_lshl_add_u32 reads its shift amount mod 32, so a split
// cursor can advance by an unmasked selector (no AND per byte).
__device__ __forceinline__ uint32_t add_pow2_mod32(uint32_t A, uint32_t s) {
    uint32_t r;
    asm("v_lshl_add_u32 %0, 1, %1, %2" : "=v"(r) : "v"(s), "v"(A));
    return r;
}

// x >> 8 that the compiler cannot fold into later shifts: bytes 1 and 3 of
// x then leave from its low byte and from bits 16..23 (a d16_hi LDS write),
// with one shift for both.
__device__ __forceinline__ uint32_t shr8_opaque(uint32_t x) {
    uint32_t r;
    asm("v_lshrrev_b32 %0, 8, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ uint32_t mask16_bit(uint4 d, uint32_t k) {
    // Transpose so that byte B of t_i is byte 4B+i of the chunk ...
    const uint32_t a0 = __builtin_amdgcn_perm(d.y, d.x, 0x05010400u);
    const uint32_t a1 = __builtin_amdgcn_perm(d.y, d.x, 0x07030602u);
    const uint32_t a2 = __builtin_amdgcn_perm(d.w, d.z, 0x05010400u);
    const uint32_t a3 = __builtin_amdgcn_perm(d.w, d.z, 0x07030602u);
    const uint32_t t0 = __builtin_amdgcn_perm(a2, a0, 0x05040100u);
    const uint32_t t1 = __builtin_amdgcn_perm(a2, a0, 0x07060302u);
    const uint32_t t2 = __builtin_amdgcn_perm(a3, a1, 0x05040100u);
    const uint32_t t3 = __builtin_amdgcn_perm(a3, a1, 0x07060302u);
    // ... then byte B of u holds bit k of chunk bytes 4B..4B+3 at bits 0..3:
    // a rotation right by k - i (mod 32) takes bit k of every byte of t_i to
    // bit i of that byte (k < 8, so no bit crosses into the wrong byte).
    const uint32_t M = 0x01010101u;
    uint32_t u = __builtin_amdgcn_alignbit(t0, t0, k & 31u) & M;
    u |= __builtin_amdgcn_alignbit(t1, t1, (k - 1u) & 31u) & (M << 1);
    u |= __builtin_amdgcn_alignbit(t2, t2, (k - 2u) & 31u) & (M << 2);
    u |= __builtin_amdgcn_alignbit(t3, t3, (k - 3u) & 31u) & (M << 3);
    // Bytes 0 and 2 of u | u >> 4 hold positions 0..7 and 8..15.
    u |= u >> 4;
    return __builtin_amdgcn_perm(u, u, 0x0C0C0200u);
}

__device__ __forceinline__ uint32_t byte_of(const uint4 &d, int b) {
    const uint32_t w = b < 4 ? d.x : (b < 8 ? d.y : (b < 12 ? d.z : d.w));
    return (w >> (8 * (b & 3))) & 0xFFu;
}

struct LdsLevelU8 {
    static constexpr int kTile = 16384, kRows = 4, kRowBytes = 4096;
    __align__(16) uint8_t stage[kTile];
    __align__(16) uint16_t m16[kTile / 16];  // 256 words of B_l
    uint32_t wz[kRows][kWaves];
    uint16_t zpre[kTile / 64];  // at most kTile
    uint32_t D[256];
    CountTableN<5> ct;  // with the 16-bit zpre: 8 blocks per CU fit in LDS
    uint32_t z0;        // PIECES: the tile's zero prefix, looked up by thread 0
};

// Bits [lo, hi) of a word, 0 <= lo <= hi <= 64.
__device__ __forceinline__ uint64_t bit_range(uint32_t lo, uint32_t hi) {
    const uint64_t h = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    return h & ~((1ull << lo) - 1ull);
}

// Bits of slots [s0, s0 + 64) of a split tile's bit array (256 words, slot
// i = bit i % 64 of word i / 64); slots outside the tile read as 0.
__device__ __forceinline__ uint64_t slot_bits64(const uint64_t *SB, int32_t s0) {
    const int32_t wi = s0 >> 6, sh = s0 & 63;
    const uint64_t lo = wi >= 0 && wi < 256 ? SB[wi] : 0ull;
    const uint64_t hi = wi + 1 >= 0 && wi + 1 < 256 ? SB[wi + 1] : 0ull;
    return sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
}

// PIECES: the count-ahead counts per piece of the next level, the part of
// a next-level tile inside one next-level node, at index tile + node (see
// wt_stats.hpp), instead of per tile.
// LASTBITS (level L-2): the next level is the last, which splits nothing,
// so this pass writes B_{L-1} itself instead of S_{L-1}.  In the split tile
// each run of one node and bit (a "group") lands on consecutive positions of
// level L-1, and its symbols' bit 0 are the bits there: the words of the
// group's destination range are funnel shifts of the tile's slot-order bit
// array, stored whole inside the range and merged into the two words it
// shares with other groups by atomics on disjoint masks (the analog of the
// paper's CAS on words shared by nodes).  Level L-1 is then left with its
// directories (level_dirs_tile).
template <bool SCATTER, bool DIRS, bool PIECES = false, bool LASTBITS = false>
__device__ __forceinline__ void level_tile_u8(const LevelArgs &a, uint32_t tile, LdsLevelU8 &s) {
    constexpr int kTile = LdsLevelU8::kTile, kRows = LdsLevelU8::kRows, kRowBytes = LdsLevelU8::kRowBytes;

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t t0 = tile * (uint32_t)kTile;
    const uint32_t len = (uint32_t)min((uint64_t)kTile, a.n - t0);
    const uint32_t k = a.k;
    // Zeros of the level before this tile: from the tile prefixes, or (PIECES)
    // the prefix of the tile's first piece, whose node is its first symbol's
    // top l bits (looked up by thread 0, read by all after the first barrier).
    uint32_t Z0 = PIECES ? 0u : (uint32_t)a.tile_prefix[tile];
    const uint8_t *in = reinterpret_cast<const uint8_t *>(a.in) + t0;
    const uint32_t first = PIECES && tid == 0 ? (uint32_t)in[0] : 0u;

    // Load: thread t, row r holds positions r*4096 + 16t .. +15.  A whole
    // tile's four loads are issued back to back (no branch between them),
    // so their latencies overlap; the node table follows them.  Positions
    // past the end of a short tile read as 0xFF (see the split).
    uint4 d[kRows];
    uint32_t m[kRows], z[kRows];
    if (len == (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) d[r] = *reinterpret_cast<const uint4 *>(in + r * kRowBytes + 16 * tid);
    } else {
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid);
            if (p + 16 <= len) {
                d[r] = *reinterpret_cast<const uint4 *>(in + p);
            } else {
                const uint32_t nv = clamp_count(len, p, 16u);
                uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    w[j >> 2] |= ((uint32_t)j < nv ? (uint32_t)in[p + j] : 0xFFu) << (8 * (j & 3));
                d[r] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    if (SCATTER) {  // byte symbols: at most 256 nodes' entries, one per thread
        if ((uint64_t)tid < a.nD) s.D[tid] = (uint32_t)a.D[tid];
        count_init(s.ct, tid);
    }
    // Grid-uniform flags, tested with the loads in flight and before any
    // global write: the input was rejected, or the fused pass owns this level.
    if (*a.status) return;
    if (a.fused_l0 && a.level >= *a.fused_l0) return;
    if (DIRS && a.tails)
        dir_tail(0, a.D[a.nD - 1], a.n, a.L, a.rank, a.rank_len, a.sel1, a.sel0, a.cap, a.sel_counts + a.level,
                 (uint64_t)tile * kBlock + tid, (uint64_t)gridDim.x * kBlock);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid);
        const uint32_t nv = clamp_count(len, p, 16u);
        m[r] = mask16_bit(d[r], k) & ((1u << nv) - 1u);
        z[r] = nv - (uint32_t)__popc(m[r]);
        s.m16[r * kBlock + tid] = (uint16_t)m[r];
    }

    // Zero-count scan in position order (rows outer, threads inner).
    const uint32_t v01 = z[0] | (z[1] << 16), v23 = z[2] | (z[3] << 16);
    const uint32_t i01 = wave_incl_scan_u32(v01, lane), i23 = wave_incl_scan_u32(v23, lane);
    if (lane == kWave - 1) {
        s.wz[0][wave] = i01 & 0xFFFFu;
        s.wz[1][wave] = i01 >> 16;
        s.wz[2][wave] = i23 & 0xFFFFu;
        s.wz[3][wave] = i23 >> 16;
    }
    if (PIECES && tid == 0) s.z0 = a.piece_prefix[tile + (first >> (k + 1))];
    __syncthreads();
    if (PIECES) Z0 = s.z0;
    const uint32_t e01 = i01 - v01, e23 = i23 - v23;
    const uint32_t we[kRows] = {e01 & 0xFFFFu, e01 >> 16, e23 & 0xFFFFu, e23 >> 16};
    uint32_t zl[kRows], acc = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t x = s.wz[r][w];
            before += w < wave ? x : 0u;
            tot += x;
        }
        zl[r] = acc + before + we[r];
        acc += tot;
    }
    const uint32_t Zt = acc;
    if ((tid & 3) == 0)
#pragma unroll
        for (int r = 0; r < kRows; ++r) s.zpre[r * (kBlock / 4) + tid / 4] = zl[r];
    __syncthreads();

    // Bit words of the tile (word tid = m16[4 tid .. 4 tid + 3]).
    const uint64_t *s_w64 = reinterpret_cast<const uint64_t *>(s.m16);
    if ((uint32_t)tid * 64u < len) a.bits[(t0 >> 6) + tid] = s_w64[tid];

    // Directory entries: wave w covers row w, i.e. words 64w .. 64w+63.
    if (DIRS) {
        const uint32_t wbase = (uint32_t)wave * kRowBytes;
        if (wbase < len) {
            const uint32_t zb = s.zpre[wave * kWave];  // zeros of the tile before this row
            const uint32_t ze = wave + 1 < kWaves ? s.zpre[(wave + 1) * kWave] : Zt;
            const uint64_t wd[1] = {s_w64[tid]};
            const uint32_t zp[1] = {s.zpre[tid] - zb};
            emit_directories<1>(wd, zp, (uint64_t)Z0 + zb, (uint64_t)t0 + wbase, clamp_count(len, wbase, (uint32_t)kRowBytes),
                                ze - zb, a.n, a.rank, a.sel1, a.sel0, lane);
        }
    }
    if (!SCATTER) return;

    if (LASTBITS && tid == 0) s.wz[0][0] = 0;  // group count (wz is read only before the last barrier)

    // Stable split into LDS (zeros at [0, Zt), ones at [Zt, len)).  The
    // zeros' and ones' cursors of a lane share one word (low and high 16
    // bits); 16 times a byte's level bit selects the half, as the offset of
    // the read and the shift of the increment, so a byte costs an extract
    // and an add, with no branch.  The 0xFF bytes past the end of a short
    // tile are ones after every zero of the tile, so position e >= len goes
    // to slot Zt + (e - Zt) = e: slots [len, kTile), which nothing reads.
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t e0 = (uint32_t)(r * kRowBytes + 16 * tid);
        uint32_t A = zl[r] | ((Zt + e0 - zl[r]) << 16);
        const uint32_t dw[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // Bit 8i+4 of T is bit k of byte i (a rotation right by k-4 mod 32).
            // The field offset of v_bfe_u32 and the amount of a shift are the
            // low five bits of their operands, so T >> 8i serves unmasked:
            // its bits 0..4 are 16 times bit k of byte i.
            const uint32_t T = __builtin_amdgcn_alignbit(dw[j], dw[j], (k + 28u) & 31u) & 0x10101010u;
            const uint32_t h = shr8_opaque(dw[j]);  // bytes 1 and 3 in the low bytes of its halves
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t sh = T >> (8 * i);
                const uint32_t src = (i & 1) ? h : dw[j];
                s.stage[__builtin_amdgcn_ubfe(A, sh, 16u)] = (uint8_t)(src >> (16 * (i >> 1)));
                A = add_pow2_mod32(A, sh);
            }
        }
    }
    __syncthreads();

    // Scatter (see level_tile for the destination formula), sixteen slots
    // per lane: inside one run (same node, same bit) the sixteen bytes have
    // consecutive destinations and leave as one unaligned 16-byte store.
    const uint32_t O0 = t0 - Z0;
    const uint32_t kn = k - 1;  // bit of the next level
    const uint32_t Mn = 0x01010101u << kn;
    const uint32_t n16 = a.n > 15 ? (uint32_t)(a.n - 15) : 0u;  // dest < n16 <=> dest + 15 < n
    uint8_t *out = reinterpret_cast<uint8_t *>(a.out);
    // Wave w walks chunks [256w, 256w + 256) of the split tile, 64 at a time,
    // so a lane's chunks mostly stay in one run and one destination tile:
    // its running count changes tile rarely, and the counts of a wave reach
    // the table together (count_add_wave).
    const uint4 *s_st128 = reinterpret_cast<const uint4 *>(s.stage);
    constexpr int kChunksPerWave = kTile / 16 / kWaves;
    if constexpr (LASTBITS) {
        // Slot-order bits of the next level (over m16, dead since the
        // directories), group starts (over zpre: at most 2^(l+1) <= 128
        // groups for byte symbols), and the count-ahead.
        uint16_t *SB16 = s.m16, *gstart = s.zpre;
        uint32_t &ng = s.wz[0][0];
        LaneCount lc;
        auto qof = [&](uint32_t b) { return (b >> k) & a.qmask; };
        auto record = [&](uint32_t slot) {
            const uint32_t g = atomicAdd(&ng, 1u);
            if (g < kTile / 64) gstart[g] = (uint16_t)slot;
        };
#pragma unroll
        for (int i = 0; i < kChunksPerWave / kWave; ++i) {
            const uint32_t j = (uint32_t)(wave * kChunksPerWave + i * kWave + lane), sl = 16u * j;
            uint32_t ftile = kNoTile, fcnt = 0;
            if (sl < len) {
                const uint4 v = s_st128[j];
                SB16[j] = (uint16_t)mask16_bit(v, kn);
                const uint32_t q0 = qof(v.x & 0xFFu), q15 = qof(v.w >> 24);
                const uint32_t qp = sl ? qof(s.stage[sl - 1]) : ~0u;
                if (sl + 15 < len && q0 == q15) {
                    if (q0 != qp) record(sl);
                    const uint32_t dest = s.D[q0] + ((q0 & 1u) ? O0 + sl - Zt : Z0 + sl);
                    if (dest < n16) {
                        const uint32_t nt = dest >> a.next_shift;
                        if (((dest + 15) >> a.next_shift) == nt) {
                            const uint32_t ones = (uint32_t)(__popc(v.x & Mn) + __popc(v.y & Mn) +
                                                             __popc(v.z & Mn) + __popc(v.w & Mn));
                            lc.step(PIECES ? nt + q0 : nt, 16u - ones, ftile, fcnt);
                        } else {
                            for (uint32_t c = 0; c < 16; ++c)
                                if (!((byte_of(v, (int)c) >> kn) & 1u))
                                    count_add(s.ct, a.next_cnt, ((dest + c) >> a.next_shift) + (PIECES ? q0 : 0u),
                                              1u);
                        }
                    }
                } else {
                    const uint32_t nc = clamp_count(len, sl, 16u);
                    uint32_t qprev = qp;
                    for (uint32_t c = 0; c < nc; ++c) {
                        const uint32_t bc = byte_of(v, (int)c), qc = qof(bc), sc = sl + c;
                        if (qc != qprev) record(sc);
                        qprev = qc;
                        const uint32_t dest = s.D[qc] + ((qc & 1u) ? O0 + sc - Zt : Z0 + sc);
                        if (dest < a.n && !((bc >> kn) & 1u))
                            count_add(s.ct, a.next_cnt, (dest >> a.next_shift) + (PIECES ? qc : 0u), 1u);
                    }
                }
            }
            count_add_wave(s.ct, a.next_cnt, fcnt != 0, ftile, fcnt, lane);
        }
        lc.flush_wave(s.ct, a.next_cnt, lane);
        __syncthreads();
        count_flush(s.ct, a.next_cnt, tid);
        // Group starts in slot order (ranked in place; few groups).
        const uint32_t G = min(ng, (uint32_t)(kTile / 64));
        const uint32_t mine = (uint32_t)tid < G ? gstart[tid] : 0u;
        uint32_t rank = 0;
        if ((uint32_t)tid < G)
            for (uint32_t u = 0; u < G; ++u) rank += gstart[u] < mine ? 1u : 0u;
        __syncthreads();
        if ((uint32_t)tid < G) gstart[rank] = (uint16_t)mine;
        __syncthreads();
        // Each wave takes groups g = wave, wave + 4, ...; its lanes the
        // destination words of the group.
        const uint64_t *SB = reinterpret_cast<const uint64_t *>(s.m16);
        uint64_t *B = a.next_bits;
        for (uint32_t g = (uint32_t)wave; g < G; g += kWaves) {
            const uint32_t sa = gstart[g], se = g + 1 < G ? gstart[g + 1] : len;
            const uint32_t q = qof(s.stage[sa]);
            const uint32_t off = s.D[q] + ((q & 1u) ? O0 - Zt : Z0);  // destination of slot x: off + x
            const uint32_t da = off + sa, de = off + se;             // [da, de)
            for (uint32_t w = (da >> 6) + (uint32_t)lane; w <= (de - 1) >> 6; w += kWave) {
                const uint32_t lo = max(da, 64u * w) - 64u * w;
                const uint32_t hi = min(de, 64u * w + 64u) - 64u * w;
                const uint64_t own = bit_range(lo, hi);
                // the group holding position n-1 also clears the padding bits
                const uint64_t pad = (de == a.n && hi < 64u) ? bit_range(hi, 64u) : 0ull;
                const uint64_t val = slot_bits64(SB, (int32_t)(64u * w) - (int32_t)off) & own;
                if ((own | pad) == ~0ull) {
                    B[w] = val;
                } else {
                    atomicAnd((unsigned long long *)(B + w), (unsigned long long)~(own | pad));
                    if (val) atomicOr((unsigned long long *)(B + w), (unsigned long long)val);
                }
            }
        }
        return;
    }
    LaneCount lc;
#pragma unroll
    for (int i = 0; i < kChunksPerWave / kWave; ++i) {
        const uint32_t j = (uint32_t)(wave * kChunksPerWave + i * kWave + lane), sl = 16u * j;
        uint32_t ftile = kNoTile, fcnt = 0;  // a tile this lane has finished counting
        if (sl < len) {
            const uint4 v = s_st128[j];
            const uint32_t q0 = ((v.x & 0xFFu) >> k) & a.qmask, q15 = ((v.w >> 24) >> k) & a.qmask;
            if (sl + 15 < len && q0 == q15) {
                // One run: the bit is the low bit of q, so the region is uniform too.
                const uint32_t dest = s.D[q0] + ((q0 & 1u) ? O0 + sl - Zt : Z0 + sl);
                if (dest < n16) {
                    *reinterpret_cast<u128_unaligned *>(out + dest) = u128_unaligned{v.x, v.y, v.z, v.w};
                    const uint32_t nt = dest >> a.next_shift;
                    if (((dest + 15) >> a.next_shift) == nt) {
                        const uint32_t ones = (uint32_t)(__popc(v.x & Mn) + __popc(v.y & Mn) + __popc(v.z & Mn) +
                                                         __popc(v.w & Mn));
                        lc.step(PIECES ? nt + q0 : nt, 16u - ones, ftile, fcnt);
                    } else {
                        for (uint32_t c = 0; c < 16; ++c)
                            if (!((byte_of(v, (int)c) >> kn) & 1u))
                                count_add(s.ct, a.next_cnt, ((dest + c) >> a.next_shift) + (PIECES ? q0 : 0u), 1u);
                    }
                }
            } else {
                // Several runs meet here (or the tile ends): byte by byte.
                const uint32_t nc = clamp_count(len, sl, 16u);
                for (uint32_t c = 0; c < nc; ++c) {
                    const uint32_t bc = byte_of(v, (int)c), qc = (bc >> k) & a.qmask, sc = sl + c;
                    const uint32_t dest = s.D[qc] + ((qc & 1u) ? O0 + sc - Zt : Z0 + sc);
                    if (dest < a.n) {
                        out[dest] = (uint8_t)bc;
                        if (!((bc >> kn) & 1u))
                            count_add(s.ct, a.next_cnt, (dest >> a.next_shift) + (PIECES ? qc : 0u), 1u);
                    }
                }
            }
        }
        count_add_wave(s.ct, a.next_cnt, fcnt != 0, ftile, fcnt, lane);
    }
    lc.flush_wave(s.ct, a.next_cnt, lane);
    __syncthreads();
    count_flush(s.ct, a.next_cnt, tid);
}

// ---------------------------------------------------------------------------
// Directories of a level whose bits are already in place (the last level,
// written by the LASTBITS pass of level L-2): one wave per tile of 2^14
// positions, lane j holding words 4j .. 4j+3 (position order), their zeros,
// a wave scan, and the entries (emit_directories); with a.tails the level's
// directory tail too.  a.tile_prefix holds the zeros before each tile (from
// the count-ahead of level L-2).
// s_cl: the level's node starts (a.nodes of them, the last = n) in LDS.
__device__ __forceinline__ void level_dirs_tile(const LevelArgs &a, uint64_t tile, uint64_t ntiles,
                                                const uint64_t *s_cl) {
    constexpr uint32_t kTile = 16384, kWPL = 4;
    const int lane = lane_id();
    const uint64_t t0 = tile * kTile;
    const uint32_t len = (uint32_t)min((uint64_t)kTile, a.n - t0);
    if (*a.status) return;
    if (a.tails)
        dir_tail(0, a.D[a.nD - 1], a.n, a.L, a.rank, a.rank_len, a.sel1, a.sel0, a.cap, a.sel_counts + a.level,
                 tile * kWave + lane, ntiles * kWave);
    // The tile's prefix: its first piece's, whose node is the last one
    // starting at or before t0.
    uint32_t lo = 0, hi = a.nodes - 1;  // s_cl[lo] <= t0 < s_cl[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (s_cl[mid] <= t0) lo = mid;
        else hi = mid;
    }
    const uint64_t Z0 = a.piece_prefix[tile + lo];
    uint64_t wd[kWPL];
    uint32_t zp[kWPL], own = 0;
    const uint64_t *B = a.bits + (t0 >> 6);
    // (a level's words start 8-byte aligned only: W need not be even)
#pragma unroll
    for (int m = 0; m < kWPL; ++m) wd[m] = (uint32_t)(lane * kWPL + m) * 64u < len ? B[lane * kWPL + m] : 0ull;
#pragma unroll
    for (int m = 0; m < kWPL; ++m) {
        zp[m] = own;
        own += clamp_count(len, (uint32_t)(lane * kWPL + m) * 64u, 64u) - (uint32_t)__popcll(wd[m]);
    }
    const uint32_t inc = wave_incl_scan_u32(own, lane);
    const uint32_t Zt = __shfl(inc, kWave - 1, kWave), ex = inc - own;
#pragma unroll
    for (int m = 0; m < kWPL; ++m) zp[m] += ex;
    emit_directories<kWPL>(wd, zp, Z0, t0, len, Zt, a.n, a.rank, a.sel1, a.sel0, lane);
}

// ---------------------------------------------------------------------------
// Fused tail levels: levels l0..L-1 of one node-aligned segment in LDS.
//
// Once every node of level l0 holds at most kHalf positions, the positions
// from the first node boundary of level l0 at or after s*kHalf to the first
// one at or after (s+1)*kHalf form segment s: at most 2*kHalf positions
// (consecutive boundaries are at most kHalf apart) and no node of level l0
// crosses it.  Deeper nodes refine those of level l0, so the segment stays
// whole at every later level, and each block finds its own bounds by a
// binary search over C (or takes them from a table).  One block loads its
// segment once and runs every remaining level on it: the bits and
// directory entries of each level go to HBM, and no sequence traffic is
// left for those levels.  Destinations are those of the global pass (the
// node tables), rebased to the segment; the zeros of a level before the
// segment are the zeros before its first node, a table entry.  A bit word
// shared with the neighbouring segment is cleared and set over this
// segment's bit range only, with atomics (the two ranges are disjoint, so
// the order of the two segments does not matter).
//
// The segment lives in registers between levels, in a frame of kCap
// positions aligned to its first bit word (frame position a63 + j holds
// position a + j): item r of thread t is frame position r*256 + t, so the
// ballot of item r in wave w is the segment's bit word 4r + w, as in the
// level pass's tile.  The split goes through one LDS stage and back.
template <typename T, int kBytes>
struct FusedCfg {
    static constexpr int kCap = kBytes / (int)sizeof(T);  // frame positions
    static constexpr int kHalf = kCap / 2 - 32;           // segment stride: a segment and its offset fit the frame
    static constexpr int kVWords = kCap / 64;             // bit words of the frame
    static constexpr int kItems = kCap / kBlock;          // frame positions per thread
    static constexpr int kPer = 4 / (int)sizeof(T);       // items per packed register
    static constexpr int kRegs = kItems / kPer;
};

constexpr int kFusedDCache = 512;  // node-table entries of a segment's key range kept in LDS

template <typename T, int kBytes>
struct LdsFused {
    T stage[FusedCfg<T, kBytes>::kCap];
    uint64_t words[FusedCfg<T, kBytes>::kVWords];
    uint32_t zpre[FusedCfg<T, kBytes>::kVWords];  // zeros of the segment before each word
    uint64_t dcache[kFusedDCache];                // D_l[qlo + i]
    uint32_t red[kWaves];
};

struct FusedArgs {
    const void *in0;        // S (level-0 input, TIN0)
    const void *S0, *S1;    // sequences written by even / odd level passes (T)
    const uint64_t *C;      // C[0..sigma]
    const uint64_t *D;      // node tables of every level
    uint64_t sigma, n;
    uint32_t L;
    uint64_t *bits, W;
    uint64_t *rank, rank_len;
    uint64_t *sel1, *sel0, cap;
    const uint32_t *status;
    const uint32_t *l0;     // first fused level (>= L: no fusion)
    const uint32_t *segb = nullptr;  // segment starts (and n), when known; else found by search
};


// First fused level from the largest node of each level: the first level
// whose nodes all fit in kHalf positions, if it leaves a split to do
// (l0 <= L-2); L otherwise.
__device__ __forceinline__ uint32_t fused_from(const uint64_t *maxnode, uint32_t L, uint64_t half,
                                               uint32_t most = 1) {
    for (uint32_t l = 0; l + 2 <= L; ++l)
        if (maxnode[l] <= half) {
            // at most the last `most` levels when most >= 2
            const uint32_t from = most >= 2 && most < L && l < L - most ? L - most : l;
            return from + 2 <= L ? from : L;
        }
    return L;
}

// Largest node of levels [0, L) over heap elements g in [g0, g1) (g in
// [2^l, 2^(l+1)) is node g - 2^l of level l): block maxima per level into
// `red` (L entries, LDS, zeroed), then, when maxnode is not NULL, one
// atomicMax per level into it.
__device__ __forceinline__ void node_max_range(const uint64_t *C, uint64_t sigma, uint32_t L, uint64_t g0,
                                               uint64_t g1, uint64_t gstride, unsigned long long *red,
                                               unsigned long long *maxnode) {
    auto Cc = [&](uint64_t x) { return C[x < sigma ? x : sigma]; };
    for (uint64_t g = g0 + threadIdx.x; g < g1; g += gstride) {
        const uint32_t l = 63u - (uint32_t)__clzll((long long)g);
        const uint64_t p = g - (1ull << l);
        const uint64_t sz = Cc((p + 1) << (L - l)) - Cc(p << (L - l));
        if (sz) atomicMax(red + l, (unsigned long long)sz);
    }
    __syncthreads();
    if (maxnode && threadIdx.x < L && red[threadIdx.x]) atomicMax(maxnode + threadIdx.x, red[threadIdx.x]);
}

template <typename TIN0, typename T, int kBytes>
__device__ __forceinline__ void fused_segment(const FusedArgs &f, uint64_t seg, LdsFused<T, kBytes> &s) {
    using Cfg = FusedCfg<T, kBytes>;
    constexpr int kIt = Cfg::kItems, kPer = Cfg::kPer, kRegs = Cfg::kRegs;
    constexpr uint32_t kBitsPer = 8 * sizeof(T), kMask = (uint32_t)(((uint64_t)1 << kBitsPer) - 1);
    if (*f.status) return;
    const uint32_t L = f.L, l0 = *f.l0;
    if (l0 >= L) return;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint64_t n = f.n, sigma = f.sigma;
    auto Cc = [&](uint64_t x) { return f.C[x < sigma ? x : sigma]; };
    const uint32_t shift = L - l0;  // node p of level l0 covers symbols [p << shift, (p+1) << shift)
    // First node boundary of level l0 at or after `target`: a 64-way search
    // by each wave (one probe per lane and round, so about three dependent
    // loads instead of one per halving).
    auto boundary = [&](uint64_t target) -> uint64_t {
        if (target >= n) return n;
        uint64_t lo = 0, hi = 1ull << l0;  // the answer is a node index in [lo, hi]; C at node 2^l0 is n
        while (hi - lo > 1) {
            const uint64_t step = (hi - lo + kWave - 1) / kWave;
            const uint64_t p = min(lo + (uint64_t)(lane + 1) * step, hi);
            const uint64_t ge = __ballot(Cc(p << shift) >= target);  // lane 63 probes hi: always set
            const int fi = __ffsll((unsigned long long)ge) - 1;
            hi = min(lo + (uint64_t)(fi + 1) * step, hi);
            lo = fi == 0 ? lo : lo + (uint64_t)fi * step;
            if (fi == 0 && Cc(lo << shift) >= target) hi = lo;
        }
        return Cc(lo << shift) >= target ? Cc(lo << shift) : Cc(hi << shift);
    };
    const uint64_t a = f.segb ? f.segb[seg] : boundary(seg * Cfg::kHalf);
    const uint64_t e = f.segb ? f.segb[seg + 1] : boundary((seg + 1) * Cfg::kHalf);
    const uint32_t a63 = (uint32_t)(a & 63);
    if (a >= e || e - a + a63 > (uint64_t)Cfg::kCap) return;  // empty (or tables inconsistent with the input)
    const uint32_t m = (uint32_t)(e - a);
    // The segment into the stage at frame offset a63: the 16-byte vectors
    // that cover [a, e), four per thread in flight at a time (the sequences
    // are 16-byte aligned; a vector that runs past the sequence's end is
    // read symbol by symbol).
    auto load_segment = [&](auto src_tag) {
        using TS = decltype(src_tag);
        constexpr int V = 16 / (int)sizeof(TS), kG = 4;
        const TS *src = l0 == 0 ? reinterpret_cast<const TS *>(f.in0)
                                : reinterpret_cast<const TS *>((l0 - 1) % 2 == 0 ? f.S0 : f.S1);
        const uint64_t va = a / V;
        const uint32_t nv = (uint32_t)(cdiv(e, (uint64_t)V) - va);
        for (uint32_t g0 = 0; g0 < nv; g0 += kBlock * kG) {
            union {
                uint4 q;
                TS x[V];
            } u[kG];
#pragma unroll
            for (int r = 0; r < kG; ++r) {
                const uint32_t vi = g0 + r * kBlock + tid;
                if (vi < nv) {
                    if ((va + vi + 1) * V <= n) {
                        u[r].q = reinterpret_cast<const uint4 *>(src)[va + vi];
                    } else {
#pragma unroll
                        for (int x = 0; x < V; ++x) {
                            const uint64_t pos = (va + vi) * V + x;
                            u[r].x[x] = pos < n ? src[pos] : TS{};
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < kG; ++r) {
                const uint32_t vi = g0 + r * kBlock + tid;
                if (vi < nv)
#pragma unroll
                    for (int x = 0; x < V; ++x) {
                        const uint64_t pos = (va + vi) * V + x;
                        if (pos >= a && pos < e) s.stage[pos - a + a63] = (T)u[r].x[x];
                    }
            }
        }
    };
    if (l0 == 0) load_segment(TIN0{});
    else load_segment(T{});
    __syncthreads();
    // Registers: item r of this thread (frame position r*256 + tid), kPer
    // items per register.  valid(r): the position is in the segment.
    uint32_t pk[kRegs];
    auto valid = [&](int r) { return (uint32_t)(r * kBlock + tid) - a63 < m; };
    auto item = [&](int r) { return kPer == 1 ? pk[r] : (pk[r / kPer] >> (kBitsPer * (r % kPer))) & kMask; };
    auto reload = [&]() {
#pragma unroll
        for (int g = 0; g < kRegs; ++g) {
            uint32_t w = 0;
#pragma unroll
            for (int x = 0; x < kPer; ++x) {
                const int r = g * kPer + x;
                const uint32_t v = valid(r) ? (uint32_t)s.stage[r * kBlock + tid] : 0u;
                w |= v << (kBitsPer * x);
            }
            pk[g] = w;
        }
    };
    reload();
    const uint32_t nvw = (a63 + m + 63) / 64;
    const uint64_t gw0 = a >> 6;
    // Positions of word vw inside the segment; the segment that ends the
    // level also owns the padding bits of its last word (written as 0).
    auto vmask_of = [&](uint32_t vw) {
        const uint32_t lo = vw == 0 ? a63 : 0u;
        const int32_t hi = (int32_t)(a63 + m) - (int32_t)(64 * vw);
        return bit_range(lo, (uint32_t)min(max(hi, 0), 64));
    };
    auto wmask_of = [&](uint32_t vw) {
        const uint32_t lo = vw == 0 ? a63 : 0u;
        const int32_t hi = (int32_t)(a63 + m) - (int32_t)(64 * vw);
        return bit_range(lo, e == n && hi > 0 ? 64u : (uint32_t)min(max(hi, 0), 64));
    };
    // Node-table state of the current level: Za (zeros of the level before
    // the segment) and the cached window D_l[qlo, qlo + nq) of the keys
    // q = symbol >> k the split looks up.  Level l0's is loaded here; each
    // later level's is loaded while the level before it runs: the segment's
    // nodes at level l+1 are the children of its nodes [pa, pz] at level l,
    // so its keys lie in [4 pa, 4 pz + 3] and the zeros before it are
    // D_{l+1}[4 pa - 1] (the first child may be empty: the zeros before an
    // empty node equal those before the next).
    constexpr int kPf = kFusedDCache / kBlock;  // window entries per thread
    uint64_t pa = (uint64_t)((uint32_t)s.stage[a63] >> shift);  // nodes of level l0 the segment spans
    uint64_t pz = (uint64_t)((uint32_t)s.stage[a63 + m - 1] >> shift);
    uint64_t Za = 0, qlo = 0, nq = 0;
    {
        const uint64_t *Dl = f.D + ((2ull << l0) - 2);
        Za = pa ? Dl[2 * pa - 1] : 0;
        if (l0 + 1 < L) {
            qlo = 2 * pa;
            nq = min(2 * (pz - pa) + 2, (uint64_t)kFusedDCache);
            for (uint32_t i = tid; i < nq; i += kBlock) s.dcache[i] = Dl[qlo + i];
        }
    }
    const uint64_t lt = lanemask_lt(lane);
    for (uint32_t l = l0; l < L; ++l) {
        const uint32_t k = L - 1 - l;
        const uint64_t *Dl = f.D + ((2ull << l) - 2);
        // Next level's table entries, in flight while this level runs.
        uint64_t ZaN = 0, qloN = 0, nqN = 0, pf[kPf];
        if (l + 1 < L) {
            const uint64_t *Dn = f.D + ((2ull << (l + 1)) - 2);
            ZaN = pa ? Dn[4 * pa - 1] : 0;
            if (l + 2 < L) {
                qloN = 4 * pa;
                nqN = min(4 * (pz - pa) + 4, (uint64_t)kFusedDCache);
#pragma unroll
                for (int r = 0; r < kPf; ++r) {
                    const uint64_t i = (uint64_t)r * kBlock + tid;
                    pf[r] = i < nqN ? Dn[qloN + i] : 0;
                }
            }
        }
        // 1. Bit words straight from the registers: the ballot of item r in
        //    wave w is word 4r + w; zeros per word.
#pragma unroll
        for (int r = 0; r < kIt; ++r) {
            const bool ok = valid(r);
            const uint64_t wb = __ballot(ok && ((item(r) >> k) & 1u));
            const uint64_t vb = __ballot(ok);
            if (lane == 0) {
                s.words[r * kWaves + wave] = wb;
                s.zpre[r * kWaves + wave] = (uint32_t)(__popcll(vb) - __popcll(wb));
            }
        }
        __syncthreads();
        // 2. Exclusive scan of the zero counts of the segment's words.
        {
            constexpr int kWPT = (Cfg::kVWords + kBlock - 1) / kBlock;  // words per thread
            uint32_t c[kWPT], own = 0;
#pragma unroll
            for (int x = 0; x < kWPT; ++x) {
                const uint32_t w = kWPT * tid + x;
                c[x] = w < nvw ? s.zpre[w] : 0u;
                own += c[x];
            }
            const uint32_t inc = wave_incl_scan_u32(own, lane);
            if (lane == kWave - 1) s.red[wave] = inc;
            __syncthreads();
            uint32_t ex = inc - own;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) ex += w < wave ? s.red[w] : 0u;
#pragma unroll
            for (int x = 0; x < kWPT; ++x) {
                const uint32_t w = kWPT * tid + x;
                if (w < nvw) s.zpre[w] = ex;
                ex += c[x];
            }
            __syncthreads();
        }
        const uint32_t Zseg = s.red[0] + s.red[1] + s.red[2] + s.red[3];
        const uint64_t Oa = a - Za;
        uint64_t *B = f.bits + (uint64_t)l * f.W;
        uint64_t *R = f.rank + (uint64_t)l * f.rank_len;
        uint64_t *S1 = f.sel1 + (uint64_t)l * f.cap, *S0 = f.sel0 + (uint64_t)l * f.cap;
        // 3. Bit words to HBM and rank entries (positions 512 j inside the segment).
        for (uint32_t vw = tid; vw < nvw; vw += kBlock) {
            const uint64_t gw = gw0 + vw, word = s.words[vw], wm = wmask_of(vw);
            if (wm == ~0ull) {
                B[gw] = word;
            } else {
                atomicAnd((unsigned long long *)(B + gw), (unsigned long long)~wm);
                atomicOr((unsigned long long *)(B + gw), (unsigned long long)word);
            }
            if ((gw & 7) == 0 && (vmask_of(vw) & 1ull)) R[gw >> 3] = 64 * gw - (Za + s.zpre[vw]);
        }
        // 4. Select samples whose ordinal falls in the segment (targets
        //    counted by their offset r inside the segment, so the loops run
        //    at most m/4096 + 1 times whatever Za holds).
        constexpr uint64_t SS = WT_SELECT_SAMPLE;
        const uint64_t Oseg = m - Zseg;
        for (uint64_t r = (SS - Oa % SS) % SS; r < Oseg; r += SS) {
            const uint64_t t = (Oa + r) / SS;
            for (uint32_t vw = tid; vw < nvw; vw += kBlock) {
                const uint64_t word = s.words[vw];
                const uint64_t ob = (vw == 0 ? 0 : 64 * vw - a63) - s.zpre[vw];
                if (t < f.cap && ob <= r && r < ob + (uint64_t)__popcll(word))
                    S1[t] = 64 * (gw0 + vw) + select_in_word(word, (uint32_t)(r - ob));
            }
        }
        for (uint64_t r = (SS - Za % SS) % SS; r < Zseg; r += SS) {
            const uint64_t t = (Za + r) / SS;
            for (uint32_t vw = tid; vw < nvw; vw += kBlock) {
                const uint64_t zword = ~s.words[vw] & vmask_of(vw);
                const uint64_t zb = s.zpre[vw];
                if (t < f.cap && zb <= r && r < zb + (uint64_t)__popcll(zword))
                    S0[t] = 64 * (gw0 + vw) + select_in_word(zword, (uint32_t)(r - zb));
            }
        }
        if (l + 1 == L) break;
        // 5. Stable split into the stage (free: the level is in registers),
        //    at the global pass's destinations minus the segment start.
        //    Destinations are below m < 2^32, so 32-bit wrapping arithmetic
        //    gives them exactly: a zero goes to D[q] + Za + z - a, a one to
        //    D[q] + j - Za - z (z: zeros of the segment before it).
        const uint32_t add0 = (uint32_t)(Za - a), add1 = (uint32_t)(0 - Za);
#pragma unroll
        for (int r = 0; r < kIt; ++r) {
            const bool ok = valid(r);
            const uint32_t v = item(r), vw = (uint32_t)(r * kWaves + wave);
            const uint64_t vb = __ballot(ok), word = s.words[vw];
            const uint32_t z = s.zpre[vw] + (uint32_t)__popcll(~word & vb & lt);
            const uint32_t j = (uint32_t)(r * kBlock + tid) - a63;
            const uint64_t q = (uint64_t)(v >> k);
            if (ok) {
                const uint64_t d = q - qlo < nq ? s.dcache[q - qlo] : (q < (2ull << l) ? Dl[q] : ~0ull);
                const uint32_t dest = (q & 1u) ? (uint32_t)d + j + add1 - z : (uint32_t)d + z + add0;
                if (dest < m) s.stage[a63 + dest] = (T)v;
            }
        }
        __syncthreads();
        reload();
        // The next level's state: its window into the cache (the next
        // level's first barrier orders these writes before its split).
        if (l + 2 < L)
#pragma unroll
            for (int r = 0; r < kPf; ++r) {
                const uint64_t i = (uint64_t)r * kBlock + tid;
                if (i < nqN) s.dcache[i] = pf[r];
            }
        Za = ZaN;
        qlo = qloN;
        nq = nqN;
        pa = (uint64_t)((uint32_t)s.stage[a63] >> k);  // nodes of level l+1 (node = symbol >> k_{l+1} + 1 = symbol >> k)
        pz = (uint64_t)((uint32_t)s.stage[a63 + m - 1] >> k);
    }
}

// Exclusive prefix of per-tile zero counts by one block: pre[t] =
// cnt[0] + ... + cnt[t-1] for t < T.  The counts were summed by atomics of
// other blocks, so they are read with agent-scope atomic loads.
__device__ __forceinline__ void tile_prefix_block(const uint32_t *cnt, uint64_t *pre, uint64_t T, BlockScanTmp &tmp) {
    block_scan_all<4>(
        T, tmp,
        [&](uint64_t g) -> uint64_t { return __hip_atomic_load(cnt + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); },
        [&](uint64_t g, uint64_t ex) { pre[g] = ex; });
}

}  // namespace wt
