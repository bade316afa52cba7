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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/wt.h"
#include "wt_device.hpp"

namespace wt {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kDirTile = 4096;               // bits per tile of the standalone directory builder
constexpr int kWaves = kBlock / kWave;
constexpr int kScanChunk = kBlock * kItems;  // elements per block in the generic scans

constexpr uint32_t kStatusSymbol = 2u;

__host__ __device__ inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline uint64_t align_up(uint64_t a, uint64_t b) { return cdiv(a, b) * b; }

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
// histogram: counts into Cp1[c] = C[c+1] (zeroed).  Each thread reads 16
// bytes at a time and merges runs of equal symbols before counting, which
// keeps atomics off the hot symbol of skewed text.  Small alphabets count in
// LDS (kRep replicas indexed by lane to spread same-address atomics).
template <typename T>
__global__ __launch_bounds__(kBlock) void histogram(const T *__restrict__ S, uint64_t n, uint64_t sigma,
                                                    uint64_t *Cp1, uint32_t *status, uint32_t reps, uint32_t ktop,
                                                    uint32_t *cnt0, uint32_t tile_shift, uint64_t ntiles) {
    // Blocks take whole tiles of level 0, so the zeros of the top bit in each
    // tile (the count-ahead input of level 0) come out of the same read.
    // Small alphabets (reps > 0) count in LDS: `reps` replicas with a stride
    // of sigma+1 words (replicas of one symbol fall in different banks), one
    // LDS atomic per symbol and no branches; a symbol >= sigma is clamped
    // into the pad word and raises the status flag.  Large alphabets
    // aggregate every 2048 symbols in an LDS hash table (so skewed data does
    // not hammer a few global counters) and flush one global atomic per
    // distinct symbol.
    extern __shared__ uint32_t s_dyn[];
    __shared__ uint32_t s_red[kWaves];
    __shared__ uint32_t s_nused;
    constexpr uint32_t kH = 4096, kChunk = 2048, kEmpty = 0xFFFFFFFFu;
    const bool lds = reps > 0;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint64_t stride = sigma + 1;
    uint32_t *keys = s_dyn, *vals = s_dyn + kH, *used = s_dyn + 2 * kH;  // hash path
    if (lds) {
        for (uint64_t i = tid; i < stride * reps; i += kBlock) s_dyn[i] = 0;
    } else {
        for (uint32_t i = tid; i < kH; i += kBlock) {
            keys[i] = kEmpty;
            vals[i] = 0;
        }
        if (tid == 0) s_nused = 0;
    }
    __syncthreads();
    uint32_t *s_hist = lds ? s_dyn + (uint64_t)(lane % reps) * stride : nullptr;
    const uint32_t smax = (uint32_t)min(sigma, (uint64_t)0xFFFFFFFFu);
    const bool need_check = sigma < (1ull << (8 * sizeof(T)));
    constexpr int V = 16 / sizeof(T);
    const uint32_t tile_elems = 1u << tile_shift;
    bool bad = false;
    auto visit = [&](uint32_t s) -> uint32_t {
        if (lds) {
            uint32_t bin = s;
            if (need_check) {
                bad |= s >= smax;
                bin = min(s, smax);
            }
            atomicAdd(s_hist + bin, 1u);
        } else if ((uint64_t)s >= sigma) {
            bad = true;
        } else {
            uint32_t h = (s * 0x9E3779B1u) >> 20;  // 12 bits
            bool done = false;
#pragma unroll 1
            for (int probe = 0; probe < 8 && !done; ++probe) {
                const uint32_t old = atomicCAS(keys + h, kEmpty, s);
                if (old == kEmpty) used[atomicAdd(&s_nused, 1u)] = h;
                if (old == kEmpty || old == s) {
                    atomicAdd(vals + h, 1u);
                    done = true;
                }
                h = (h + 1) & (kH - 1);
            }
            if (!done) atomicAdd((unsigned long long *)(Cp1 + s), 1ull);
        }
        return ((s >> ktop) & 1u) ^ 1u;
    };
    auto flush = [&]() {
        __syncthreads();
        const uint32_t nu = s_nused;
        for (uint32_t i = tid; i < nu; i += kBlock) {
            const uint32_t h = used[i];
            atomicAdd((unsigned long long *)(Cp1 + keys[h]), (unsigned long long)vals[h]);
            keys[h] = kEmpty;
            vals[h] = 0;
        }
        __syncthreads();
        if (tid == 0) s_nused = 0;
        __syncthreads();
    };
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t base = tile << tile_shift;
        const uint32_t len = (uint32_t)min((uint64_t)tile_elems, n - base);
        uint32_t zeros = 0;
        for (uint32_t c0 = 0; c0 < len; c0 += kChunk) {  // hash path: at most kChunk symbols per flush
            const uint32_t clen = min(kChunk, len - c0);
            if (clen == kChunk) {
                for (uint32_t v = tid; v < kChunk / V; v += kBlock) {
                    union {
                        uint4 q;
                        T e[V];
                    } u;
                    u.q = *reinterpret_cast<const uint4 *>(S + base + c0 + (uint64_t)v * V);
#pragma unroll
                    for (int j = 0; j < V; ++j) zeros += visit((uint32_t)u.e[j]);
                }
            } else {
                for (uint32_t e = tid; e < clen; e += kBlock) zeros += visit((uint32_t)S[base + c0 + e]);
            }
            if (!lds) flush();
        }
        if (cnt0) {
            uint32_t w = (uint32_t)wave_sum_u64(zeros);
            if (lane == 0) s_red[wave] = w;
            __syncthreads();
            if (tid == 0) {
                uint32_t t = 0;
                for (int i = 0; i < kWaves; ++i) t += s_red[i];
                cnt0[tile] = t;
            }
            __syncthreads();
        }
    }
    if (__ballot(bad) && lane == 0) atomicMax(status, kStatusSymbol);
    if (lds) {
        __syncthreads();
        for (uint64_t c = tid; c < sigma; c += kBlock) {
            uint32_t sum = 0;
            for (uint32_t r = 0; r < reps; ++r) sum += s_dyn[(uint64_t)r * stride + c];
            if (sum) atomicAdd((unsigned long long *)(Cp1 + c), (unsigned long long)sum);
        }
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

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of kItems values per thread (blocked layout).
struct BlockScanTmp {
    uint64_t wave_tot[kWaves];
};

__device__ __forceinline__ uint64_t block_excl_scan(uint64_t (&v)[kItems], BlockScanTmp &tmp, uint64_t &total) {
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    uint64_t own = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) own += v[j];
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
    for (int j = 0; j < kItems; ++j) {
        uint64_t x = v[j];
        v[j] = run;
        run += x;
    }
    return before + inc - own;
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

// Node tables.  Element g in [1, 2^L) is node p = g - 2^l of level l =
// floor(log2 g) (heap numbering from 1).  value = ones of B_l inside node p
// = symbols of its range whose bit k_l is 1 = C[end] - C[middle].
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
// Level pass.
//
// A tile is 16 KiB of the level's sequence whatever the symbol width, so one
// block has enough bytes in flight to cover HBM latency and a level has few
// enough tiles for the look-back to stay short.  The 256 threads hold the
// tile packed in 16 registers each (item r of thread t is position
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
constexpr int kMinTile = TileCfg<uint32_t>::kTile;  // smallest tile: sizes the look-back state arrays
constexpr int kSmallD = 512;                        // node tables up to this size are cached in LDS

struct LevelArgs {
    const void *in;          // S_l (TIN), 16-byte aligned
    void *out;               // S_{l+1} (TOUT)
    uint64_t *bits;          // B_l
    const uint64_t *D;       // D_l: 2^(l+1) entries
    uint64_t nD;             // 2^(l+1)
    const uint64_t *tile_prefix;  // zeros of B_l before each tile of this level
    uint32_t *next_cnt;      // zeros of B_{l+1} per tile of the next level (accumulated here)
    uint32_t next_shift;     // log2(positions per tile of the next level)
    const uint32_t *status;  // non-zero: input rejected, do nothing
    uint64_t *rank, *sel1, *sel0;  // directory rows of level l
    uint64_t n;
    uint32_t k;              // bit examined at this level: L-1-l
};

// Count-ahead: while level l scatters S_{l+1}, it also counts, for every tile
// of level l+1, the zeros that tile will hold (bit k-1 of the symbols that
// land in it).  A scan of those counts gives each tile of level l+1 its
// exclusive zero prefix before level l+1 starts, so no tile ever waits for
// another.  Each lane keeps a running count for the destination tile it is
// filling and hands it to a small LDS table keyed by destination tile when
// that tile changes (a block's runs touch few tiles); the table reaches HBM
// as one atomic add per touched tile when the block ends, and a slot
// collision falls back to a direct atomic.
constexpr int kCountSlots = 64;
constexpr uint32_t kNoTile = 0xFFFFFFFFu;
struct CountTable {
    uint32_t key[kCountSlots];
    uint32_t cnt[kCountSlots];
};

__device__ __forceinline__ void count_init(CountTable &t, int tid) {
    if (tid < kCountSlots) {
        t.key[tid] = kNoTile;
        t.cnt[tid] = 0;
    }
}

__device__ __forceinline__ void count_add(CountTable &t, uint32_t *next_cnt, uint32_t ntile, uint32_t c) {
    // Hashed slot with a short linear probe: the tiles one block touches are
    // few but can be far apart by large powers of two (a run of zeros and a
    // run of ones half a level apart), so the low bits alone would collide.
    uint32_t slot = (ntile * 0x9E3779B9u) >> 26;
#pragma unroll 1
    for (int probe = 0; probe < 8; ++probe) {
        const uint32_t old = atomicCAS(&t.key[slot], kNoTile, ntile);
        if (old == kNoTile || old == ntile) {
            atomicAdd(&t.cnt[slot], c);
            return;
        }
        slot = (slot + 1) & (kCountSlots - 1);
    }
    atomicAdd(next_cnt + ntile, c);
}

__device__ __forceinline__ void count_flush(CountTable &t, uint32_t *next_cnt, int tid) {
    if (tid < kCountSlots && t.key[tid] != kNoTile && t.cnt[tid]) atomicAdd(next_cnt + t.key[tid], t.cnt[tid]);
}

// Per-lane running count for one destination tile.
struct LaneCount {
    uint32_t tile = kNoTile, cnt = 0;
    __device__ __forceinline__ void add(CountTable &t, uint32_t *next_cnt, uint32_t ntile, uint32_t c) {
        if (ntile != tile) {
            if (cnt) count_add(t, next_cnt, tile, cnt);
            tile = ntile;
            cnt = 0;
        }
        cnt += c;
    }
    __device__ __forceinline__ void flush(CountTable &t, uint32_t *next_cnt) {
        if (cnt) count_add(t, next_cnt, tile, cnt);
        cnt = 0;
    }
};

template <typename T>
__device__ __forceinline__ uint32_t zero_bits(const uint4 &q, uint32_t k) {
    union {
        uint4 v;
        T e[16 / sizeof(T)];
    } u;
    u.v = q;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < (int)(16 / sizeof(T)); ++j) c += (((uint32_t)u.e[j] >> k) & 1u) ^ 1u;
    return c;
}

template <typename TIN, typename TOUT, bool SCATTER, bool DIRS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void level_pass(LevelArgs a) {
    using Cfg = TileCfg<TIN>;
    constexpr int kTile = Cfg::kTile, kItems = Cfg::kItems, kWPL = Cfg::kWPL;
    constexpr int V = 16 / sizeof(TIN);
    __shared__ __align__(16) unsigned char s_stage[Cfg::kBytes];
    __shared__ uint64_t s_words[Cfg::kWords];
    __shared__ uint32_t s_zpre[Cfg::kWords];
    __shared__ uint64_t s_D[SCATTER ? kSmallD : 1];
    __shared__ uint64_t s_Z0;
    __shared__ uint32_t s_Zt;
    __shared__ CountTable s_ct;

    if (*a.status) return;  // uniform across the grid: the input was rejected
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint64_t tile = blockIdx.x;
    const uint64_t t0 = tile * kTile;
    const uint32_t len = (uint32_t)min((uint64_t)kTile, a.n - t0);
    const uint32_t k = a.k;
    const bool d_lds = SCATTER && a.nD <= (uint64_t)kSmallD;
    if (d_lds)
        for (int i = tid; i < (int)a.nD; i += kBlock) s_D[i] = a.D[i];
    if (SCATTER) count_init(s_ct, tid);

    // 1. Coalesced 16-byte loads of the tile into LDS.
    TIN *stage_in = reinterpret_cast<TIN *>(s_stage);
    const TIN *in = reinterpret_cast<const TIN *>(a.in) + t0;
    if (len == (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kItems / V; ++r) {
            int e = (r * kBlock + tid) * V;
            *reinterpret_cast<uint4 *>(stage_in + e) = *reinterpret_cast<const uint4 *>(in + e);
        }
    } else {
        for (uint32_t e = tid; e < len; e += kBlock) stage_in[e] = in[e];
    }
    __syncthreads();

    // 2. Striped view: item r of wave w, lane j is position r*256 + 64w + j,
    //    so each ballot is one position-ordered word of B_l (word 4r + w).
    uint32_t pk[Cfg::kRegs];
#pragma unroll
    for (int i = 0; i < Cfg::kRegs; ++i) pk[i] = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        uint32_t e = (uint32_t)(r * kBlock + tid);
        bool valid = e < len;
        uint32_t sym = valid ? (uint32_t)stage_in[e] : 0u;
        pk[r / Cfg::kPer] |= sym << (8 * sizeof(TIN) * (r % Cfg::kPer));
        bool bit = valid && ((sym >> k) & 1u);
        uint64_t vm = __ballot(valid);
        uint64_t w = __ballot(bit);
        if (lane == 0) {
            s_words[r * kWaves + wave] = w;
            s_zpre[r * kWaves + wave] = (uint32_t)(__popcll(vm) - __popcll(w));
        }
    }
    __syncthreads();

    // 3. Wave 0: scan of the word zero-counts, look-back across tiles, bit
    //    words to HBM, directory entries.
    if (wave == 0) {
        uint32_t zp[kWPL];
        uint64_t wd[kWPL];
        uint32_t own = 0;
#pragma unroll
        for (int m = 0; m < kWPL; ++m) {
            zp[m] = own;
            own += s_zpre[lane * kWPL + m];
            wd[m] = s_words[lane * kWPL + m];
        }
        uint32_t inc = wave_incl_scan_u32(own, lane);
        uint32_t Zt = __shfl(inc, kWave - 1, kWave);
        const uint64_t Z0 = a.tile_prefix[tile];
        const uint32_t ex = inc - own;
#pragma unroll
        for (int m = 0; m < kWPL; ++m) {
            zp[m] += ex;
            s_zpre[lane * kWPL + m] = zp[m];
        }
        if (lane == 0) {
            s_Z0 = Z0;
            s_Zt = Zt;
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
    const uint64_t Z0 = s_Z0;
    const uint32_t Zt = s_Zt;

    // 4. Stable split of the tile by the level bit into LDS: zeros keep their
    //    order at [0, Zt), ones at [Zt, len).  Inside each region the
    //    elements stay grouped by node, and each node's group lands on
    //    consecutive positions of S_{l+1}.
    TOUT *stage_out = reinterpret_cast<TOUT *>(s_stage);
    const uint64_t lt = lanemask_lt(lane);
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        uint32_t e = (uint32_t)(r * kBlock + tid);
        if (e < len) {
            uint64_t w = s_words[r * kWaves + wave];
            uint32_t zl = s_zpre[r * kWaves + wave] + (uint32_t)__popcll(~w & lt);
            uint32_t slot = ((w >> lane) & 1ull) ? Zt + (e - zl) : zl;
            uint32_t sym = (pk[r / Cfg::kPer] >> (8 * sizeof(TIN) * (r % Cfg::kPer))) &
                           (sizeof(TIN) == 4 ? 0xFFFFFFFFu : ((1u << (8 * sizeof(TIN))) - 1u));
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
    for (int r = 0; r < kItems; ++r) {
        uint32_t s = (uint32_t)(r * kBlock + tid);
        if (s < len) {
            TOUT v = stage_out[s];
            uint64_t q = (uint64_t)((uint32_t)v >> k);
            if (q < a.nD) {
                uint64_t base = d_lds ? s_D[q] : a.D[q];
                uint64_t dest = base + (s < Zt ? Z0 + s : O0 + (s - Zt));
                if (dest < a.n) {
                    out[dest] = v;
                    lc.add(s_ct, a.next_cnt, (uint32_t)(dest >> a.next_shift), (((uint32_t)v >> kn) & 1u) ^ 1u);
                }
            }
        }
    }
    lc.flush(s_ct, a.next_cnt);
    __syncthreads();
    count_flush(s_ct, a.next_cnt, tid);
}

// ---------------------------------------------------------------------------
// Level pass for byte symbols (n < 2^32): the same steps as level_pass with
// SWAR arithmetic, since at HBM rate a byte symbol leaves only about ten
// lane operations per level.  A tile is 4 rows of 4096 bytes; thread t owns
// bytes [16t, 16t+16) of every row as four dwords.
//   bits:  a 4x4 byte transpose (v_perm) lines bit k of the 16 bytes up so
//          that a few shifts and ORs give them as a 16-bit mask in position
//          order; four lanes' masks are one word of B_l, so the LDS array of
//          masks read as 64-bit words *is* the tile's slice of B_l.
//   scan:  two rows per 32-bit value (16-bit fields), one wave scan each.
//   split: bytes go to their LDS slot while wave 0 runs the look-back.
//   scatter: sixteen slots per lane; inside one run (same node, same bit)
//          they have consecutive destinations and leave as one (possibly
//          unaligned) 16-byte store.
typedef uint32_t u128_unaligned __attribute__((ext_vector_type(4), aligned(1)));

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
    // ... then byte B of u holds bit k of chunk bytes 4B..4B+3 at bits 0..3.
    const uint32_t M = 0x01010101u;
    uint32_t u = ((t0 >> k) & M) | (((t1 >> k) & M) << 1) | (((t2 >> k) & M) << 2) | (((t3 >> k) & M) << 3);
    u |= u >> 4;
    return (u & 0xFFu) | ((u >> 8) & 0xFF00u);
}

__device__ __forceinline__ uint32_t byte_of(const uint4 &d, int b) {
    const uint32_t w = b < 4 ? d.x : (b < 8 ? d.y : (b < 12 ? d.z : d.w));
    return (w >> (8 * (b & 3))) & 0xFFu;
}

template <bool SCATTER, bool DIRS>
__global__ __launch_bounds__(kBlock) void level_pass_u8(LevelArgs a) {
    constexpr int kTile = 16384, kRows = 4, kRowBytes = 4096;
    __shared__ __align__(16) uint8_t s_stage[kTile];
    __shared__ __align__(16) uint16_t s_m16[kTile / 16];  // 256 words of B_l
    __shared__ uint32_t s_wz[kRows][kWaves];
    __shared__ uint32_t s_zpre[kTile / 64];
    __shared__ uint32_t s_D[SCATTER ? 256 : 1];
    __shared__ CountTable s_ct;

    if (*a.status) return;  // uniform across the grid: the input was rejected
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t tile = blockIdx.x;
    const uint32_t t0 = tile * (uint32_t)kTile;
    const uint32_t len = (uint32_t)min((uint64_t)kTile, a.n - t0);
    const uint32_t k = a.k;
    const uint32_t Z0 = (uint32_t)a.tile_prefix[tile];  // zeros of the level before this tile
    if (SCATTER) {
        for (int i = tid; i < (int)a.nD; i += kBlock) s_D[i] = (uint32_t)a.D[i];
        count_init(s_ct, tid);
    }

    // Load: thread t, row r holds positions r*4096 + 16t .. +15.
    const uint8_t *in = reinterpret_cast<const uint8_t *>(a.in) + t0;
    uint4 d[kRows];
    uint32_t m[kRows], z[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid);
        if (p + 16 <= len) {
            d[r] = *reinterpret_cast<const uint4 *>(in + p);
        } else {
            uint32_t w[4] = {0, 0, 0, 0};
            for (uint32_t j = 0; j < 16 && p + j < len; ++j) w[j >> 2] |= (uint32_t)in[p + j] << (8 * (j & 3));
            d[r] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid);
        const uint32_t nv = p >= len ? 0u : min(16u, len - p);
        m[r] = mask16_bit(d[r], k) & ((1u << nv) - 1u);
        z[r] = nv - (uint32_t)__popc(m[r]);
        s_m16[r * kBlock + tid] = (uint16_t)m[r];
    }

    // Zero-count scan in position order (rows outer, threads inner).
    const uint32_t v01 = z[0] | (z[1] << 16), v23 = z[2] | (z[3] << 16);
    const uint32_t i01 = wave_incl_scan_u32(v01, lane), i23 = wave_incl_scan_u32(v23, lane);
    if (lane == kWave - 1) {
        s_wz[0][wave] = i01 & 0xFFFFu;
        s_wz[1][wave] = i01 >> 16;
        s_wz[2][wave] = i23 & 0xFFFFu;
        s_wz[3][wave] = i23 >> 16;
    }
    __syncthreads();
    const uint32_t e01 = i01 - v01, e23 = i23 - v23;
    const uint32_t we[kRows] = {e01 & 0xFFFFu, e01 >> 16, e23 & 0xFFFFu, e23 >> 16};
    uint32_t zl[kRows], acc = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t x = s_wz[r][w];
            before += w < wave ? x : 0u;
            tot += x;
        }
        zl[r] = acc + before + we[r];
        acc += tot;
    }
    const uint32_t Zt = acc;
    if ((tid & 3) == 0)
#pragma unroll
        for (int r = 0; r < kRows; ++r) s_zpre[r * (kBlock / 4) + tid / 4] = zl[r];
    __syncthreads();

    // Bit words of the tile (word tid = s_m16[4 tid .. 4 tid + 3]).
    const uint64_t *s_w64 = reinterpret_cast<const uint64_t *>(s_m16);
    if ((uint32_t)tid * 64u < len) a.bits[(t0 >> 6) + tid] = s_w64[tid];

    // Directory entries: wave w covers row w, i.e. words 64w .. 64w+63.
    if (DIRS) {
        const uint32_t wbase = (uint32_t)wave * kRowBytes;
        if (wbase < len) {
            const uint32_t zb = s_zpre[wave * kWave];  // zeros of the tile before this row
            const uint32_t ze = wave + 1 < kWaves ? s_zpre[(wave + 1) * kWave] : Zt;
            const uint64_t wd[1] = {s_w64[tid]};
            const uint32_t zp[1] = {s_zpre[tid] - zb};
            emit_directories<1>(wd, zp, (uint64_t)Z0 + zb, (uint64_t)t0 + wbase, min(len - wbase, (uint32_t)kRowBytes),
                                ze - zb, a.n, a.rank, a.sel1, a.sel0, lane);
        }
    }
    if (!SCATTER) return;

    // Stable split into LDS (zeros at [0, Zt), ones at [Zt, len)).
    if (len == (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const uint32_t e0 = (uint32_t)(r * kRowBytes + 16 * tid);
            uint32_t zc = zl[r], oc = Zt + e0 - zl[r];
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                const uint32_t bit = (m[r] >> b) & 1u;
                s_stage[bit ? oc : zc] = (uint8_t)byte_of(d[r], b);
                zc += bit ^ 1u;
                oc += bit;
            }
        }
    } else {
        for (int r = 0; r < kRows; ++r) {
            const uint32_t e0 = (uint32_t)(r * kRowBytes + 16 * tid);
            uint32_t zc = zl[r], oc = Zt + e0 - zl[r];
            for (int b = 0; b < 16 && e0 + b < len; ++b) {
                const uint32_t bit = (m[r] >> b) & 1u;
                s_stage[bit ? oc : zc] = (uint8_t)byte_of(d[r], b);
                zc += bit ^ 1u;
                oc += bit;
            }
        }
    }
    __syncthreads();

    // Scatter (see level_pass for the destination formula), sixteen slots
    // per lane: inside one run (same node, same bit) the sixteen bytes have
    // consecutive destinations and leave as one unaligned 16-byte store.
    const uint32_t O0 = t0 - Z0;
    const uint32_t kn = k - 1;  // bit of the next level
    const uint32_t Mn = 0x01010101u << kn;
    const uint32_t n16 = a.n > 15 ? (uint32_t)(a.n - 15) : 0u;  // dest < n16 <=> dest + 15 < n
    uint8_t *out = reinterpret_cast<uint8_t *>(a.out);
    const uint4 *s_st128 = reinterpret_cast<const uint4 *>(s_stage);
    LaneCount lc;
#pragma unroll
    for (int i = 0; i < kTile / (16 * kBlock); ++i) {
        const uint32_t j = (uint32_t)(tid + i * kBlock), sl = 16u * j;
        if (sl >= len) continue;
        const uint4 v = s_st128[j];
        const uint32_t q0 = (v.x & 0xFFu) >> k, q15 = (v.w >> 24) >> k;
        if (sl + 15 < len && q0 == q15) {
            // One run: the bit is the low bit of q, so the region is uniform too.
            const uint32_t dest = s_D[q0] + ((q0 & 1u) ? O0 + sl - Zt : Z0 + sl);
            if (dest < n16) {
                *reinterpret_cast<u128_unaligned *>(out + dest) = u128_unaligned{v.x, v.y, v.z, v.w};
                const uint32_t nt = dest >> a.next_shift;
                if (((dest + 15) >> a.next_shift) == nt) {
                    const uint32_t ones = (uint32_t)(__popc(v.x & Mn) + __popc(v.y & Mn) + __popc(v.z & Mn) +
                                                     __popc(v.w & Mn));
                    lc.add(s_ct, a.next_cnt, nt, 16u - ones);
                } else {
                    for (uint32_t c = 0; c < 16; ++c)
                        if (!((byte_of(v, (int)c) >> kn) & 1u))
                            count_add(s_ct, a.next_cnt, (dest + c) >> a.next_shift, 1u);
                }
            }
        } else {
            // Several runs meet here (or the tile ends): byte by byte.
            for (uint32_t c = 0; c < 16 && sl + c < len; ++c) {
                const uint32_t bc = byte_of(v, (int)c), qc = bc >> k, sc = sl + c;
                const uint32_t dest = s_D[qc] + ((qc & 1u) ? O0 + sc - Zt : Z0 + sc);
                if (dest < a.n) {
                    out[dest] = (uint8_t)bc;
                    if (!((bc >> kn) & 1u)) count_add(s_ct, a.next_cnt, dest >> a.next_shift, 1u);
                }
            }
        }
    }
    lc.flush(s_ct, a.next_cnt);
    __syncthreads();
    count_flush(s_ct, a.next_cnt, tid);
}

// ---------------------------------------------------------------------------
// Directory tails: for every level, rank[l][last] = ones of the level, the
// sample counts, and sample entries past the counts set to n.  The level
// totals come either from the node tables (zeros of a level = D_l's last
// entry) or from an array of per-level totals.
__global__ void dir_finish(const uint64_t *D, const uint64_t *zeros_tot, uint64_t n, uint32_t L,
                           uint64_t *rank, uint64_t rank_len, uint64_t *sel1, uint64_t *sel0, uint64_t cap,
                           uint64_t *sel_counts) {
    const uint32_t l = blockIdx.y;
    uint64_t zeros = zeros_tot ? zeros_tot[l] : D[(1ull << (l + 2)) - 3];
    uint64_t ones = n - zeros;
    uint64_t c1 = cdiv(ones, WT_SELECT_SAMPLE), c0 = cdiv(zeros, WT_SELECT_SAMPLE);
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        rank[(uint64_t)l * rank_len + rank_len - 1] = ones;
        sel_counts[l] = c1;
        sel_counts[L + l] = c0;
    }
    if (t < cap) {
        if (t >= c1) sel1[(uint64_t)l * cap + t] = n;
        if (t >= c0) sel0[(uint64_t)l * cap + t] = n;
    }
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
    const uint32_t nb = has ? min(64u, len - (uint32_t)lane * 64u) : 0u;
    const uint32_t zc = nb - (uint32_t)__popcll(word);
    uint32_t inc = wave_incl_scan_u32(zc, lane);
    uint32_t Zt = __shfl(inc, kWave - 1, kWave);
    auto zeros_of_tile = [&](uint64_t ft) -> uint64_t {
        const uint64_t f0 = ft * kDirTile;
        const uint32_t flen = (uint32_t)min((uint64_t)kDirTile, n - f0);
        const bool fh = (uint32_t)lane * 64u < flen;
        const uint32_t fnb = fh ? min(64u, flen - (uint32_t)lane * 64u) : 0u;
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
    uint64_t off_status, off_cnt, off_pre, off_D, off_part, off_S0, off_S1, total;
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
    if (p.L > 30) return WT_ERR_RANGE;  // dense node tables: 2^(L+1) words
    p.in_bytes = (uint32_t)sym_bytes;
    p.mid_bytes = p.L <= 8 ? 1u : (p.L <= 16 ? 2u : 4u);  // width of S_l for l >= 1
    p.W = cdiv(n, 64);
    p.T = cdiv(n, kMinTile);
    p.rank_len = cdiv(n, WT_RANK_BLOCK_BITS) + 1;
    p.cap = cdiv(n, WT_SELECT_SAMPLE) + 1;
    const uint64_t table_elems = p.L ? (1ull << p.L) : 0;        // node heap indices [0, 2^L)
    const uint64_t D_len = p.L ? (2ull << p.L) - 2 : 0;          // 2^(l+1) entries per level
    const uint64_t part_c = cdiv(sigma, kScanChunk);
    const uint64_t part_t = cdiv(table_elems, kScanChunk);
    p.n_part = std::max<uint64_t>(std::max<uint64_t>(part_c, part_t), 1);
    uint64_t o = 0;
    p.off_status = o;
    o += 256;
    p.T = align_up(p.T, 64);  // per-level stride of the tile arrays (keeps vector loads aligned)
    p.off_cnt = o;  // zeros per tile, per level (count-ahead), zeroed each build
    o = align_up(o + 4ull * p.L * p.T, 256);
    p.off_pre = o;  // exclusive zero prefix per tile, per level
    o = align_up(o + 8ull * p.L * p.T, 256);
    p.off_D = o;
    o = align_up(o + 8ull * D_len, 256);
    p.off_part = o;
    o = align_up(o + 8ull * p.n_part, 256);
    p.off_S0 = o;
    const uint64_t sbytes = p.L >= 2 ? align_up(n * p.mid_bytes, 256) : 0;
    o += sbytes;
    p.off_S1 = o;
    o += p.L >= 3 ? sbytes : 0;
    p.total = o;
    return WT_OK;
}

static bool g_timing = false;
static int g_spin_limit = 8;
static std::mutex g_timing_mu;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;  // recorded, not yet collected
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_free;

static int timing_begin(hipStream_t s, std::pair<hipEvent_t, hipEvent_t> &ev) {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (!g_free.empty()) {
        ev = g_free.back();
        g_free.pop_back();
    } else {
        if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) return WT_ERR_HIP;
    }
    return hipEventRecord(ev.first, s) == hipSuccess ? WT_OK : WT_ERR_HIP;
}

static int timing_end(hipStream_t s, std::pair<hipEvent_t, hipEvent_t> &ev) {
    if (hipEventRecord(ev.second, s) != hipSuccess) return WT_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_events.push_back(ev);
    return WT_OK;
}

template <typename TIN, typename TOUT>
static void launch_level(bool scatter, bool dirs, hipStream_t s, const LevelArgs &a) {
    if (sizeof(TIN) == 1 && sizeof(TOUT) == 1 && a.n < (1ull << 32)) {
        dim3 g8((unsigned)cdiv(a.n, 16384)), b8(kBlock);
        if (scatter) {
            if (dirs) level_pass_u8<true, true><<<g8, b8, 0, s>>>(a);
            else level_pass_u8<true, false><<<g8, b8, 0, s>>>(a);
        } else {
            if (dirs) level_pass_u8<false, true><<<g8, b8, 0, s>>>(a);
            else level_pass_u8<false, false><<<g8, b8, 0, s>>>(a);
        }
        return;
    }
    dim3 grid((unsigned)cdiv(a.n, TileCfg<TIN>::kTile)), block(kBlock);
    if (scatter) {
        if (dirs) level_pass<TIN, TOUT, true, true><<<grid, block, 0, s>>>(a);
        else level_pass<TIN, TOUT, true, false><<<grid, block, 0, s>>>(a);
    } else {
        if (dirs) level_pass<TIN, TOUT, false, true><<<grid, block, 0, s>>>(a);
        else level_pass<TIN, TOUT, false, false><<<grid, block, 0, s>>>(a);
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

// Positions per tile of a level whose sequence has `width`-byte symbols.
static uint32_t tile_shift_for(uint32_t width) { return width == 1 ? 14u : (width == 2 ? 13u : 12u); }

template <typename T>
static void launch_hist(const void *seq, const Plan &p, uint64_t *Cp1, uint32_t *status, uint32_t *cnt0,
                        hipStream_t s) {
    uint32_t reps = 0;  // LDS replicas (64 lanes share them), 0 = global atomics
    if (p.sigma <= 8192) reps = (uint32_t)std::min<uint64_t>(16, std::max<uint64_t>(1, 8192 / (p.sigma + 1)));
    const uint32_t shift = tile_shift_for(sizeof(T));
    const uint64_t ntiles = cdiv(p.n, 1ull << shift);
    uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>(ntiles, (uint64_t)num_cus() * 8));
    size_t shm = reps ? (size_t)reps * (p.sigma + 1) * 4 : (size_t)(2 * 4096 + 2048) * 4;  // replicas, or hash table + used list
    histogram<T><<<(unsigned)blocks, kBlock, shm, s>>>((const T *)seq, p.n, p.sigma, Cp1, status, reps,
                                                       p.L ? p.L - 1 : 0u, p.L ? cnt0 : nullptr, shift, ntiles);
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

extern "C" int wt_build(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                        void *d_scratch, uint64_t scratch_bytes, void *stream) {
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

    // Zero: status + per-tile zero counts (one contiguous range), and C.
    {
        uint64_t na = p.off_pre / 8, nb = sigma + 1;
        uint64_t blocks = std::min<uint64_t>(cdiv(na + nb, kBlock), 4096);
        zero_fill<<<(unsigned)blocks, kBlock, 0, s>>>((uint64_t *)sc, na, out->C, nb);
    }
    if (n > 0) {
        if (sym_bytes == 1) launch_hist<uint8_t>(d_seq, p, out->C + 1, status, cnt, s);
        else if (sym_bytes == 2) launch_hist<uint16_t>(d_seq, p, out->C + 1, status, cnt, s);
        else launch_hist<uint32_t>(d_seq, p, out->C + 1, status, cnt, s);
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
    if (p.L > 0) {
        // Node tables for every level.
        TableOp top{out->C, D, sigma, p.L};
        uint64_t count = 1ull << p.L;
        uint64_t chunks = cdiv(count, kScanChunk);
        if (chunks > 1) {
            scan_reduce<TableOp><<<(unsigned)chunks, kBlock, 0, s>>>(top, count, part);
            scan_partials_seg<TableOp><<<1, kBlock, 0, s>>>(top, chunks, part);
            scan_final<TableOp><<<(unsigned)chunks, kBlock, 0, s>>>(top, count, part);
        } else {
            scan_final<TableOp><<<1, kBlock, 0, s>>>(top, count, nullptr);
        }
        if (dirs) {
            dim3 g((unsigned)cdiv(p.cap, kBlock), p.L);
            dir_finish<<<g, kBlock, 0, s>>>(D, nullptr, n, p.L, out->rank, p.rank_len, out->sel1, out->sel0, p.cap,
                                            out->sel_counts);
        }
    }
    if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
    if (n == 0 || p.L == 0) return WT_OK;

    const void *cur = d_seq;
    uint32_t cur_w = p.in_bytes;
    for (uint32_t l = 0; l < p.L; ++l) {
        const bool scatter = l + 1 < p.L;
        void *dst = (l % 2 == 0) ? (void *)(sc + p.off_S0) : (void *)(sc + p.off_S1);
        // Tile prefixes of this level from the counts its predecessor left.
        const uint64_t Tl = cdiv(n, 1ull << tile_shift_for(cur_w));
        tile_prefix_scan<<<1, kScanThreads, 0, s>>>(cnt + (uint64_t)l * p.T, pre + (uint64_t)l * p.T, Tl);
        LevelArgs a;
        a.in = cur;
        a.out = scatter ? dst : nullptr;
        a.bits = out->bits + (uint64_t)l * p.W;
        a.D = D + ((2ull << l) - 2);
        a.nD = 2ull << l;
        a.tile_prefix = pre + (uint64_t)l * p.T;
        a.next_cnt = scatter ? cnt + (uint64_t)(l + 1) * p.T : nullptr;
        a.next_shift = tile_shift_for(p.mid_bytes);
        a.status = status;
        a.rank = dirs ? out->rank + (uint64_t)l * p.rank_len : nullptr;
        a.sel1 = dirs ? out->sel1 + (uint64_t)l * p.cap : nullptr;
        a.sel0 = dirs ? out->sel0 + (uint64_t)l * p.cap : nullptr;
        a.n = n;
        a.k = p.L - 1 - l;
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (g_timing && (rc = timing_begin(s, ev))) return rc;
        launch_level_any(cur_w, scatter ? p.mid_bytes : cur_w, scatter, dirs, s, a);
        if (g_timing && (rc = timing_end(s, ev))) return rc;
        if (hipGetLastError() != hipSuccess) return WT_ERR_HIP;
        cur = dst;
        cur_w = p.mid_bytes;
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

extern "C" int wt_status_get(const void *d_scratch, void *stream) {
    if (!d_scratch) return WT_ERR_ARG;
    uint32_t st = 0;
    if (hipMemcpyAsync(&st, d_scratch, sizeof(st), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess)
        return WT_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return WT_ERR_HIP;
    return st == 0 ? WT_OK : (st == kStatusSymbol ? WT_ERR_SYMBOL : WT_ERR_HIP);
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
