// Batched construction: many sequences of uneven length and alphabet built
// together from a list of work items (levelWT, Fig. 1 of "Parallel Wavelet
// Tree Construction", applied to every sequence).
//
// Work items, in queue order (phase-major, so that the items one item waits
// for were all handed out long before it):
//   histogram tile (job, t)   counts of one tile of S into the job's symbol
//                             counts (LDS replicas or hash, global atomics),
//                             the symbol check, the zeros of the top bit
//   job histogram (job)       a whole job with 8192 < sigma <= 2^16 in one
//                             block: packed 16-bit LDS counters, C written
//                             by the block itself
//   tables (job)              C (unless its histogram wrote it), the node
//                             tables D_l, the directory tails, the tile
//                             prefixes of level 0, the first fused level and
//                             the fused segments' starts
//   level tile (job, l, t)    one tile of the level pass (bits, directories,
//                             stable split and scatter, count-ahead of l+1);
//                             byte-symbol and wider tiles are separate phases
//   fused segment (job, s)    the job's tail levels on chip on one
//                             node-aligned segment, once every node fits
//
// Two launch forms, same items and outputs:
//  * one launch per phase (the default): a kernel built for that phase's
//    kind only (and, for a level phase whose tiles take one variant, for that
//    variant only).  The tables phase lists the live items of level 0 and of
//    the fused phase, and a set-up launch before each level l >= 1 scans the
//    count-ahead totals into the level's tile prefixes and lists its live
//    tiles; level and fused launches take their items from those lists.
//    Kernel boundaries order the phases, so no wait ever spins and no
//    cross-XCD write-back is needed between items;
//  * one persistent launch over the whole queue: blocks take chunks of items
//    from a global head counter and wait, with release/acquire fences, for
//    the items their own depends on (the block that finishes the last tile
//    of a level scans the count-ahead totals into the next level's tile
//    prefixes and marks that level ready).  A block only waits on items that
//    precede its own in the queue, and items are handed out in queue order to
//    blocks that are running, so every wait ends whatever the residency
//    (induction on queue position).  A wait is still bounded: after
//    `spin_limit` polls it raises the batch's abort flag and the job's
//    timeout status and goes on (outputs are then unspecified); later waits
//    return at once once the flag is up.
// Either form is a fixed sequence of kernel launches with no host work in
// between, so it can be captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/wt.h"
#include "wt_device.hpp"
#include "wt_kernels.hpp"
#include "wt_u16.hpp"
#include "wt_u32.hpp"

namespace wt {
namespace batch {

constexpr uint32_t kStatusTimeout = 4u;
constexpr uint32_t kHistH = 2048;                         // hash slots of the batched histogram
constexpr uint32_t kHistWords = HistHash<kHistH>::kWords;  // LDS words of its table (replicas or hash)
constexpr uint32_t kKindHist = 0, kKindPrep = 1, kKindLevel = 2;  // level l is kind 2 + l
constexpr uint32_t kKindFused = 64;                                 // a segment of the fused tail levels
constexpr uint32_t kKindJobHist = 65;                               // a whole job's histogram
constexpr int kFusedBytes = 16384;                                  // per LDS buffer of a fused segment
constexpr uint32_t kJobHistMaxSigma = 65536;  // packed 16-bit LDS bins of one block (128 KiB)

// Item kinds a kernel is built for: each phase of the per-phase launch gets
// a kernel with only its own kind (its own LDS and registers; the whole-job
// histograms, bit 2, have a kernel of their own, job_hist_kernel); the
// persistent launch gets one with every kind.
constexpr uint32_t kHasTileHist = 1, kHasPrep = 4, kHasLevel8 = 8, kHasLevelWide = 16, kHasFused = 32,
                   kHasAll = 63;
constexpr uint32_t kHasLevel = kHasLevel8 | kHasLevelWide;

// Tile variants of the level pass: input and output widths and whether it
// scatters (every level but the last).  A level launch whose items all take
// one variant is built for that variant alone (its registers, no others').
constexpr uint32_t vcode(uint32_t win, uint32_t wout, bool scatter) {
    return 1u + (win << 8) + (scatter ? (wout << 4) + 1u : 0u);
}
constexpr bool var_has(uint32_t var, uint32_t code) { return var == 0 || var == code; }

// Waves per SIMD each kernel is compiled for: the register budget that
// keeps its code free of spills (the per-phase kernels inline several tile
// variants, and the job records take many scalar registers), except for the
// fused tail levels and the mixed wider tiles, which run faster at five
// waves with a few spilled registers than at four without (measured).
constexpr int waves_for(uint32_t kinds, uint32_t var = 0) {
    return kinds == kHasPrep ? 2 : (var != 0 ? (var == vcode(1, 1, true) ? 4 : 5) : (kinds == kHasLevelWide || kinds == kHasFused ? 5 : 4));
}

// Control words of one job (cleared by every run): status, done counters
// (histogram, then one per level), ready flags (one per level).
constexpr int kCtlWords = 64;
constexpr int kCtlStatus = 0, kCtlDone = 1, kCtlReady = 32, kCtlCDone = 62, kCtlFusedL0 = 63;
constexpr int kMaxLevels = 30;
constexpr uint64_t kHeaderBytes = 512;  // queue heads [0, 32), abort flag [32], live counts [64, 128)
constexpr int kAbortWord = 32;
constexpr int kLiveWord = 64;  // entries of each phase's list (per-phase launches)

struct JobDev {
    const void *seq;
    uint64_t n, sigma;
    uint32_t L, in_bytes, mid_bytes, reps;
    uint32_t T0, Tm, Tpad, hist_items;  // hist_items: T0 tile items, or 1 whole-job item
    uint64_t W, rank_len, cap;
    uint64_t *bits, *C, *rank, *sel1, *sel0, *sel_counts;
    uint32_t *ctl, *symcnt, *cnt;
    uint64_t *pre, *D;
    void *S0, *S1;
    uint32_t *segb;  // first position of every fused segment, and n (nseg + 1 entries)
    uint32_t nseg;
    uint32_t id;     // the job's index
};

struct Seg {
    uint32_t job, kind, first, count;
};

struct Args {
    const JobDev *jobs;
    const Seg *segs;
    const uint32_t *seg_of;  // segment of every item
    uint32_t *head;          // queue head of this launch
    uint32_t *abort;
    uint32_t lo, hi;         // item range of this launch
    uint32_t chunk;          // items taken per queue access
    uint32_t spin_limit;
    uint32_t fenced;         // items of one launch depend on each other's writes
    uint32_t fuse;           // tail levels fused in LDS once a job's nodes fit: 0 none, 1 all, m >= 2 at most m
    // Per-phase launches: every level and fused launch takes its items from
    // a list of the live ones, (job, tile or segment), that the tables phase
    // (level 0, fused segments) and the level set-up launches (level l >= 1)
    // append to; the list of a phase sits in that phase's item range.
    uint2 *list;
    uint32_t *live;             // entries of each phase's list
    uint32_t phase, level;      // this launch's phase, and its level (level launches)
    uint32_t base0[2];          // list bases of level 0 (byte tiles, wider tiles)
    uint32_t base_fused, phase_fused;
};

struct LdsHistB {
    uint32_t tab[kHistWords];
    uint32_t red[kWaves];
    uint32_t nused;
};

// Node tables by chunks of C: a chunk of 2^12 symbols holds every node of
// the 12 deepest levels whole, so those levels' tables come from one read of
// C (into LDS) per chunk.
constexpr uint32_t kTabChunkLog = 12, kTabChunk = 1u << kTabChunkLog;
constexpr uint32_t kTabPer = 16;  // chunk symbols per thread
static_assert(kTabChunk == kTabPer * kBlock, "a chunk is 16 symbols per thread");

struct LdsPrep {
    BlockScanTmp scan;
    uint32_t at;                                 // first list entry the block reserved
    unsigned long long nmax[32];                 // wave maxima of a level's node sizes
    uint64_t lmax[32];                           // every level's largest node
    uint32_t cl[kTabChunk + kTabChunk / 16 + 1]; // C over the chunk and the next chunk's first (padded)
    uint32_t wtot[kWaves][5];                    // wave totals of the five scanned values
    uint32_t xs[kBlock];                         // block prefix of the deep nodes' ones
    uint32_t big[32];                            // largest node of each chunked level
};

// Whole-job histogram: two 16-bit counters per word.
struct LdsJobHist {
    uint32_t bins[kJobHistMaxSigma / 2];
    uint32_t wtot[16];  // wave totals of the C scan (1024-thread blocks)
    uint32_t overflow;
};

// Level items: byte tiles and wider tiles run in launches of their own, each
// with only its own LDS (the byte pass keeps eight blocks per CU); the
// persistent form holds every kind.
union LdsLevels8 {
    LdsLevelU8 u8;
    BlockScanTmp scan;
};
union LdsLevelsWide {
    LdsLevelU16 u16;
    LdsLevelU32 u32;
    LdsLevel<uint16_t> g16;
    BlockScanTmp scan;
};
union LdsLevels {
    LdsLevelU8 u8;
    LdsLevelU16 u16;
    LdsLevelU32 u32;
    LdsLevel<uint16_t> g16;
    BlockScanTmp scan;
};

union LdsFusedAll {
    LdsFused<uint8_t, kFusedBytes> f8;
    LdsFused<uint16_t, kFusedBytes> f16;
    LdsFused<uint32_t, kFusedBytes> f32;
};

union LdsBatch {
    LdsHistB hist;
    LdsPrep prep;
    LdsLevels lv;
    LdsFusedAll fu;
};

// A job or segment record: constant while the kernel runs and uniform
// across the block, so it is read through the constant address space
// (scalar loads into SGPRs, which the compiler may reload instead of
// keeping vector registers busy).
template <typename T>
__device__ __forceinline__ T load_const(const T *p) {
#if __HIP_DEVICE_COMPILE__
    typedef const __attribute__((address_space(4))) T *const_ptr;
    return *(const_ptr)(uintptr_t)p;
#else
    return *p;
#endif
}

__device__ __forceinline__ uint32_t ld_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-block hand-off.
//   One launch per phase: an item only reads what earlier launches wrote
//   (kernel boundaries order it), except the count-ahead totals that the
//   last tile of a level scans.  Those are atomics, performed where every
//   XCD sees them; each wave waits for its own to complete before the block
//   counts itself done, and the last block reads them with atomic loads.
//   So no cache maintenance is needed.
//   One persistent launch: items read other items' plain stores, which may
//   sit dirty in another XCD's L2.  A barrier orders nothing beyond the
//   workgroup (it does not even wait for the other waves' stores), so every
//   wave releases its own writes at agent scope (L2 write-back) before the
//   barrier that precedes the signalling atomic, and every wave acquires
//   after the barrier that follows a successful wait.
__device__ __forceinline__ void wait_own_stores() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt left free
}

__device__ __forceinline__ void block_release(bool fenced) {
    if (fenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    else wait_own_stores();
    __syncthreads();
}

__device__ __forceinline__ void block_acquire(bool fenced) {
    if (fenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// The block waits until *p >= target (thread 0 polls), then acquires.
__device__ __forceinline__ void wait_for(const Args &b, const uint32_t *p, uint32_t target, uint32_t *status) {
    if (threadIdx.x == 0) {
        uint32_t spins = 0;
        while (ld_u32(p) < target) {
            if (ld_u32(b.abort)) break;
            if (++spins >= b.spin_limit) {
                atomicOr(b.abort, 1u);
                atomicOr(status, kStatusTimeout);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    block_acquire(b.fenced);
}

// Counts one finished item of a segment (after releasing the block's
// writes); true in every thread of the block that finished the last one,
// which has then acquired the other items' writes.
__device__ __forceinline__ bool finish_item(const Args &b, uint32_t *done, uint32_t count, uint32_t *s_flag) {
    block_release(b.fenced);
    if (threadIdx.x == 0) *s_flag = atomicAdd(done, 1u) == count - 1 ? 1u : 0u;
    __syncthreads();
    const bool last = *s_flag != 0;
    if (last) block_acquire(b.fenced);
    return last;
}

__device__ __forceinline__ void publish(const Args &b, uint32_t *flag) {
    block_release(b.fenced);
    if (threadIdx.x == 0) __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void hist_item(const JobDev &j, uint32_t tile, LdsHistB &s) {
    const uint32_t shift = tile_shift_for(sizeof(T));
    const uint64_t base = (uint64_t)tile << shift;
    const uint32_t len = (uint32_t)min(1ull << shift, j.n - base);
    hist_init<kHistH>(s.tab, &s.nused, j.reps, j.sigma);
    bool bad = false;
    const uint32_t zeros = hist_count<T, kHistH>(reinterpret_cast<const T *>(j.seq), base, len, j.sigma, j.reps,
                                                 j.L ? j.L - 1 : 0u, s.tab, &s.nused, j.symcnt, bad);
    if (j.reps) hist_flush_replicas(s.tab, j.reps, j.sigma, j.symcnt);
    if (__ballot(bad) && lane_id() == 0) atomicOr(j.ctl + kCtlStatus, kStatusSymbol);
    if (j.L) {
        const uint32_t t = block_sum_u32(zeros, s.red);
        if (threadIdx.x == 0) j.cnt[tile] = t;
    }
}

// A whole job's histogram in one block of 1024 threads (alphabets of up to
// 2^16 symbols whose counters do not fit as LDS replicas; 16 waves cover the
// latency of the LDS atomics): packed 16-bit counters in LDS, so no global
// atomic is needed per symbol, and the block writes C itself.  A counter
// that reaches 2^15 gives 2^15 to the job's global count of that symbol
// (the thread whose add crossed the mark does it, so a half never carries
// into its neighbour).  Also the per-tile zeros of the top bit (one atomic
// per wave into the cleared counts).
constexpr int kJHThreads = 1024, kJHWaves = kJHThreads / kWave;
constexpr int kJHTiles = 4;  // 16 KiB tiles in flight per group (one 16-byte vector per thread each)

template <typename T>
__device__ __forceinline__ void job_hist_block(const JobDev &j, LdsJobHist &s) {
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t nwords = (uint32_t)((j.sigma + 1) / 2);
    for (uint32_t i = tid; i < nwords; i += kJHThreads) s.bins[i] = 0;
    if (tid == 0) s.overflow = 0;
    __syncthreads();
    const T *S = reinterpret_cast<const T *>(j.seq);
    const uint32_t shift = tile_shift_for(sizeof(T)), ktop = j.L ? j.L - 1 : 0u;
    constexpr int V = 16 / sizeof(T);
    static_assert((16384 / 16) == kJHThreads, "one vector per thread and tile");
    bool bad = false, ovf = false;
    auto count = [&](uint32_t x) -> uint32_t {
        if (x >= j.sigma) {
            bad = true;
        } else {
            const uint32_t hi = x & 1u, inc = hi ? 0x10000u : 1u;
            const uint32_t old = atomicAdd(s.bins + (x >> 1), inc);
            if (((old >> (16 * hi)) & 0xFFFFu) == 0x7FFFu) {
                atomicSub(s.bins + (x >> 1), inc << 15);
                atomicAdd(j.symcnt + x, 0x8000u);
                ovf = true;
            }
        }
        return ((x >> ktop) & 1u) ^ 1u;
    };
    union Vec {
        uint4 q;
        T e[V];
    };
    const uint32_t Tfull = (uint32_t)(j.n >> shift);
    Vec cur[kJHTiles], nxt[kJHTiles];
    auto load = [&](uint32_t t0, Vec (&q)[kJHTiles]) {
#pragma unroll
        for (int r = 0; r < kJHTiles; ++r)
            if (t0 + r < Tfull) q[r].q = reinterpret_cast<const uint4 *>(S + ((uint64_t)(t0 + r) << shift))[tid];
    };
    if (Tfull) load(0, cur);
    for (uint32_t t0 = 0; t0 < Tfull; t0 += kJHTiles) {
        if (t0 + kJHTiles < Tfull) load(t0 + kJHTiles, nxt);
#pragma unroll
        for (int r = 0; r < kJHTiles; ++r) {
            if (t0 + r >= Tfull) break;
            uint32_t zeros = 0;
#pragma unroll
            for (int e = 0; e < V; ++e) zeros += count((uint32_t)cur[r].e[e]);
            const uint32_t wz = wave_sum_u32(zeros);
            if (j.L && lane == 0) atomicAdd(j.cnt + t0 + r, wz);
        }
#pragma unroll
        for (int r = 0; r < kJHTiles; ++r) cur[r] = nxt[r];
    }
    if (Tfull < j.T0) {  // the ragged last tile
        const uint64_t base = (uint64_t)Tfull << shift;
        const uint32_t len = (uint32_t)(j.n - base);
        uint32_t zeros = 0;
        for (uint32_t e = tid; e < len; e += kJHThreads) zeros += count((uint32_t)S[base + e]);
        const uint32_t wz = wave_sum_u32(zeros);
        if (j.L && lane == 0) atomicAdd(j.cnt + Tfull, wz);
    }
    if (__ballot(bad) && lane == 0) atomicOr(j.ctl + kCtlStatus, kStatusSymbol);
    if (__ballot(ovf) && lane == 0) atomicOr(&s.overflow, 1u);
    __syncthreads();
    // C = exclusive prefix of the counts (plus what reached the global
    // counters): wave w takes bins [4096 w, 4096 w + 4096), first its total,
    // then 64-bin rounds of wave scans stored coalesced.
    const bool spill = s.overflow != 0;
    auto value = [&](uint64_t g) -> uint32_t {
        if (g >= j.sigma) return 0u;
        const uint32_t w = s.bins[g >> 1];
        return ((w >> (16 * (g & 1))) & 0xFFFFu) +
               (spill ? __hip_atomic_load(j.symcnt + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u);
    };
    constexpr uint32_t kPerWave = kJobHistMaxSigma / kJHWaves;
    const uint64_t g0 = (uint64_t)wave * kPerWave;
    uint32_t own = 0;
    for (uint32_t r = 0; r < kPerWave; r += kWave) own += value(g0 + r + lane);
    own = wave_sum_u32(own);
    if (lane == 0) s.wtot[wave] = own;
    __syncthreads();
    uint64_t carry = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kJHWaves; ++w) {
        const uint32_t t = s.wtot[w];
        carry += w < wave ? t : 0u;
        total += t;
    }
    for (uint32_t r = 0; r < kPerWave && g0 + r < j.sigma; r += kWave) {
        const uint64_t g = g0 + r + lane;
        const uint32_t v = value(g), inc = wave_incl_scan_u32(v, lane);
        if (g < j.sigma) j.C[g] = carry + inc - v;
        carry += __shfl(inc, kWave - 1, kWave);
    }
    if (tid == 0) {
        j.C[j.sigma] = total;
        j.ctl[kCtlCDone] = 1;
    }
}

// Per-phase launches: the whole-job histogram items, one block each.
__global__ __launch_bounds__(kJHThreads) void job_hist_kernel(Args b) {
    __shared__ LdsJobHist s;
    for (uint32_t it = b.lo + blockIdx.x; it < b.hi; it += gridDim.x) {
        __syncthreads();  // the previous job is done with the LDS
        const uint32_t si = __builtin_amdgcn_readfirstlane(b.seg_of[it]);
        const Seg sg = load_const(b.segs + si);
        const JobDev j = load_const(b.jobs + __builtin_amdgcn_readfirstlane(sg.job));
        if (j.in_bytes == 2) job_hist_block<uint16_t>(j, s);
        else job_hist_block<uint32_t>(j, s);
        wait_own_stores();
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(j.ctl + kCtlDone, 1u);
    }
}

// The same job with a small LDS (the persistent kernel): tile by tile
// through the hashed counts of hist_count, flushed to the global counts.
template <typename T>
__device__ __forceinline__ void job_hist_small(const JobDev &j, LdsHistB &s) {
    for (uint32_t tile = 0; tile < j.T0; ++tile) {
        __syncthreads();
        hist_item<T>(j, tile, s);
    }
}

__host__ __device__ inline uint64_t fused_half(uint32_t mid) {
    return mid == 1 ? FusedCfg<uint8_t, kFusedBytes>::kHalf
                    : (mid == 2 ? FusedCfg<uint16_t, kFusedBytes>::kHalf : FusedCfg<uint32_t, kFusedBytes>::kHalf);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int m = kWave / 2; m >= 1; m >>= 1) v = max(v, (uint32_t)__shfl_xor(v, m, kWave));
    return v;
}

// Node tables of every level and each level's largest node, for one job by
// one block.  The levels whose nodes span at most 2^12 symbols go chunk by
// chunk (C of the chunk into LDS: one coalesced read of C in all):
//  * thread t owns the chunk's symbols [16t, 16t + 16); the nodes of depth
//    d <= 3 (2^(d+1) symbols, level L-1-d) inside them come from its 17 C
//    values in registers;
//  * each deeper node of the chunk (255 of them for a full chunk) belongs to
//    one thread, depth by depth, and reads its three C values from LDS;
// then one block scan of five values per thread (the ones of its depth-0..3
// nodes, its deep node's ones) gives every node's ones before it in the
// chunk; a deep depth's own prefix is the scan minus the scan at its first
// thread.  Each thread carries its depths' totals from chunk to chunk.  The
// few levels above (nodes wider than a chunk) come straight from C.  Counts
// fit 32 bits (n < 2^32); the tables are 64-bit.
__device__ __forceinline__ uint32_t tab_pad(uint32_t i) { return i + (i >> 4); }  // conflict-free strided reads

__device__ __forceinline__ void tables_chunked(const JobDev &j, LdsPrep &lp) {
    const uint32_t L = j.L, CHL = min(kTabChunkLog, L), lc = L - CHL;
    const uint32_t CH = 1u << CHL, S = min(kTabPer, CH), nloc = min(4u, CHL);
    const uint64_t nchunks = 1ull << lc;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    for (uint32_t l = 0; l < lc; ++l) {
        const uint64_t m = table_level_block<4>(j.C, j.sigma, L, l, j.D, lp.scan, lp.nmax);
        if (tid == 0) lp.lmax[l] = m;
    }
    // This thread's deep node: depth dd, index ii; depth dd's nodes are the
    // threads [off, off + nk).
    uint32_t dd = 0, ii = 0, off = 0, nk = 0;
    bool deep = false;
    for (uint32_t d = 4, o = 0; d < CHL; ++d) {
        const uint32_t k = CH >> (d + 1);
        if ((uint32_t)tid >= o && (uint32_t)tid < o + k) {
            dd = d;
            ii = tid - o;
            off = o;
            nk = k;
            deep = true;
        }
        o += k;
    }
    const bool owner = (uint32_t)tid * kTabPer < CH;
    uint64_t carry[4] = {0, 0, 0, 0}, dcarry = 0;
    uint32_t bigloc[4] = {0, 0, 0, 0}, bigdeep = 0;
    if (tid < 32) lp.big[tid] = 0;
    // A chunk's C in registers: every load of it in flight at once, the
    // next chunk's issued before this one's tables are computed.
    constexpr int kPer = kTabChunk / kBlock + 1;
    uint32_t cv[kPer];
    auto load_chunk = [&](uint64_t c0) {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const uint64_t i = (uint64_t)r * kBlock + tid, c = min(c0 + i, j.sigma);
            cv[r] = i <= CH ? (uint32_t)j.C[c] : 0u;
        }
    };
    load_chunk(0);
    for (uint64_t ch = 0; ch < nchunks; ++ch) {
        __syncthreads();  // the previous chunk is done with cl and xs
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const uint32_t i = (uint32_t)r * kBlock + tid;
            if (i <= CH) lp.cl[tab_pad(i)] = cv[r];
        }
        if (ch + 1 < nchunks) load_chunk((ch + 1) << CHL);
        __syncthreads();
        uint32_t c[kTabPer + 1];
#pragma unroll
        for (uint32_t q = 0; q <= kTabPer; ++q) c[q] = owner && q <= S ? lp.cl[tab_pad(tid * kTabPer + q)] : 0u;
        uint32_t v[5];
#pragma unroll
        for (uint32_t d = 0; d < 4; ++d) {
            v[d] = 0;
#pragma unroll
            for (uint32_t i = 0; i < (kTabPer >> (d + 1)); ++i)
                if (owner && d < nloc && i < (S >> (d + 1))) {
                    v[d] += c[(i + 1) << (d + 1)] - c[(2 * i + 1) << d];
                    bigloc[d] = max(bigloc[d], c[(i + 1) << (d + 1)] - c[i << (d + 1)]);
                }
        }
        uint32_t dce = 0;
        v[4] = 0;
        if (deep) {
            dce = lp.cl[tab_pad((ii + 1) << (dd + 1))];
            v[4] = dce - lp.cl[tab_pad((2 * ii + 1) << dd)];
            bigdeep = max(bigdeep, dce - lp.cl[tab_pad(ii << (dd + 1))]);
        }
        uint32_t inc[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) inc[q] = wave_incl_scan_u32(v[q], lane);
        if (lane == kWave - 1)
#pragma unroll
            for (int q = 0; q < 5; ++q) lp.wtot[wave][q] = inc[q];
        __syncthreads();
        uint32_t ex[5], tot[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            uint32_t before = 0, all = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t t = lp.wtot[w][q];
                before += w < wave ? t : 0u;
                all += t;
            }
            ex[q] = before + inc[q] - v[q];
            tot[q] = all;
        }
        lp.xs[tid] = ex[4];
        __syncthreads();
        // Depths 0..3: the thread's nodes, in order.
#pragma unroll
        for (uint32_t d = 0; d < 4; ++d) {
            if (d >= nloc) continue;
            if (owner) {
                uint64_t *Dl = j.D + (2ull << (L - 1 - d)) - 2;
                const uint64_t p0 = (ch * CH + (uint64_t)tid * kTabPer) >> (d + 1);
                uint64_t run = carry[d] + ex[d];
#pragma unroll
                for (uint32_t i = 0; i < (kTabPer >> (d + 1)); ++i)
                    if (i < (S >> (d + 1))) {
                        const uint32_t ce = c[(i + 1) << (d + 1)], ones = ce - c[(2 * i + 1) << d];
                        ulonglong2 e;
                        e.x = run;                          // ones of the level before the node
                        e.y = (uint64_t)ce - (run + ones);  // zeros before the next node
                        *reinterpret_cast<ulonglong2 *>(Dl + 2 * (p0 + i)) = e;
                        run += ones;
                    }
            }
            carry[d] += tot[d];
        }
        // The deep node.
        if (deep) {
            const uint32_t first = lp.xs[off];
            const uint64_t run = dcarry + (ex[4] - first);
            uint64_t *Dl = j.D + (2ull << (L - 1 - dd)) - 2;
            const uint64_t p = ch * nk + ii;
            ulonglong2 e;
            e.x = run;
            e.y = (uint64_t)dce - (run + v[4]);
            *reinterpret_cast<ulonglong2 *>(Dl + 2 * p) = e;
            dcarry += lp.xs[off + nk] - first;
        }
    }
    // Largest node of each chunked level.
#pragma unroll
    for (uint32_t d = 0; d < 4; ++d) {
        const uint32_t m = wave_max_u32(bigloc[d]);
        if (lane == 0 && d < nloc) atomicMax(&lp.big[d], m);
    }
    if (deep) atomicMax(&lp.big[dd], bigdeep);
    __syncthreads();
    if ((uint32_t)tid < CHL) lp.lmax[L - 1 - tid] = lp.big[tid];
    __syncthreads();
}

// Segments of a job whose levels from l0 on run fused in LDS.  Segment s
// starts at the first node start of level l0 at or after s * half (n if
// none), so each node lies in exactly one segment.  Segment s is empty when
// its start is n or lies at or beyond (s + 1) * half (the next segment then
// starts at the same node).  With lists, the nonempty ones are appended to
// the fused list.
__device__ __forceinline__ void fused_segments(const JobDev &j, uint32_t l0, const Args &b, LdsPrep &lp) {
    const uint64_t half = fused_half(j.mid_bytes), n = j.n, P = 1ull << l0;
    const uint32_t shift = j.L - l0;
    auto Cc = [&](uint64_t x) { return j.C[x < j.sigma ? x : j.sigma]; };
    // Thread t handles nodes p = t + 1, t + 1 + kBlock, ...: segments s with
    // start(p - 1) < s * half <= start(p) start at start(p).
    auto visit = [&](auto &&fn) {
        for (uint64_t p = 1 + threadIdx.x; p <= P; p += kBlock) {
            const uint64_t c0 = Cc((p - 1) << shift), c = Cc(p << shift);
            for (uint64_t sg = c0 / half + 1; sg * half <= c && sg <= j.nseg; ++sg) fn(sg, c);
        }
    };
    if (threadIdx.x == 0) {
        j.segb[0] = 0;
        j.segb[j.nseg] = (uint32_t)n;
    }
    visit([&](uint64_t sg, uint64_t c) { j.segb[sg] = (uint32_t)c; });
    if (!b.list) return;
    uint32_t mine = threadIdx.x == 0 && n > 0 ? 1u : 0u;  // segment 0 starts at 0 < half
    visit([&](uint64_t sg, uint64_t c) { mine += c < n && c < (sg + 1) * half ? 1u : 0u; });
    uint64_t v[1] = {mine}, total;
    block_excl_scan<1>(v, lp.scan, total);
    if (threadIdx.x == 0) lp.at = total ? atomicAdd(b.live + b.phase_fused, (uint32_t)total) : 0u;
    __syncthreads();
    uint2 *out = b.list + b.base_fused + lp.at + v[0];
    if (threadIdx.x == 0 && n > 0) *out++ = make_uint2(j.id, 0u);
    visit([&](uint64_t sg, uint64_t c) {
        if (c < n && c < (sg + 1) * half) *out++ = make_uint2(j.id, (uint32_t)sg);
    });
}

// C (unless the job's histogram already wrote it), node tables, directory
// tails, level-0 tile prefixes and the first fused level of one job.  N:
// values per thread in the block scans (more is faster, and costs registers).
template <int N>
__device__ __forceinline__ void prep_item(const JobDev &j, LdsPrep &lp, uint32_t fuse, const Args &b) {
    BlockScanTmp &tmp = lp.scan;
    if (!__hip_atomic_load(j.ctl + kCtlCDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        const uint64_t total = block_scan_all<N>(
            j.sigma, tmp, [&](uint64_t g) -> uint64_t { return j.symcnt[g]; },
            [&](uint64_t g, uint64_t ex) { j.C[g] = ex; });
        if (threadIdx.x == 0) j.C[j.sigma] = total;
        __syncthreads();  // the block reads C back below (workgroup scope)
    }
    if (j.L == 0) return;
    // Node tables, with each level's largest node (the fusion plan's input).
    tables_chunked(j, lp);
    for (uint32_t l = 0; l < j.L; ++l)
        dir_tail(l, j.D[(1ull << (l + 2)) - 3], j.n, j.L, j.rank, j.rank_len, j.sel1, j.sel0, j.cap, j.sel_counts,
                 threadIdx.x, kBlock);
    tile_prefix_block(j.cnt, j.pre, j.T0, tmp);
    uint32_t l0 = j.L;
    if (fuse && j.L >= 2 && j.n > 0) l0 = fused_from(lp.lmax, j.L, fused_half(j.mid_bytes), fuse);
    if (threadIdx.x == 0) j.ctl[kCtlFusedL0] = l0;
    if (l0 < j.L) fused_segments(j, l0, b, lp);
    if (b.list && j.n > 0 && l0 > 0) {
        // Level 0's tiles are live.
        __syncthreads();  // every thread has read lp.at of the fused list
        const uint32_t wide = j.in_bytes > 1 ? 1u : 0u;
        if (threadIdx.x == 0) lp.at = atomicAdd(b.live + 3 + wide, j.T0);
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < j.T0; t += kBlock) b.list[b.base0[wide] + lp.at + t] = make_uint2(j.id, t);
    }
}

template <uint32_t KINDS, uint32_t VAR = 0, typename LV>
__device__ __forceinline__ void level_item(const JobDev &j, uint32_t l, uint32_t tile, LV &s, bool listed) {
    const bool scatter = l + 1 < j.L;
    const uint32_t win = l == 0 ? j.in_bytes : j.mid_bytes, wout = j.mid_bytes;
    LevelArgs a;
    a.in = l == 0 ? j.seq : ((l - 1) % 2 == 0 ? j.S0 : j.S1);
    a.out = scatter ? (l % 2 == 0 ? j.S0 : j.S1) : nullptr;
    a.bits = j.bits + (uint64_t)l * j.W;
    a.D = j.D + ((2ull << l) - 2);
    a.nD = 2ull << l;
    a.tile_prefix = j.pre + (uint64_t)l * j.Tpad;
    a.next_cnt = scatter ? j.cnt + (uint64_t)(l + 1) * j.Tpad : nullptr;
    a.next_shift = tile_shift_for(j.mid_bytes);
    a.status = j.ctl + kCtlStatus;
    a.rank = j.rank + (uint64_t)l * j.rank_len;
    a.sel1 = j.sel1 + (uint64_t)l * j.cap;
    a.sel0 = j.sel0 + (uint64_t)l * j.cap;
    a.n = j.n;
    a.k = j.L - 1 - l;
    a.level = l;
    a.fused_l0 = listed ? nullptr : j.ctl + kCtlFusedL0;  // a listed tile is live
    a.qmask = ~0u;
    if (win == 1) {
        if constexpr ((KINDS & kHasLevel8) != 0) {
            if (scatter) {
                if constexpr (var_has(VAR, vcode(1, 1, true))) level_tile_u8<true, true>(a, tile, s.u8);
            } else {
                if constexpr (var_has(VAR, vcode(1, 0, false))) level_tile_u8<false, true>(a, tile, s.u8);
            }
        }
        return;
    }
    if constexpr ((KINDS & kHasLevelWide) != 0) {
        // The SWAR passes of wt_build for 16- and 32-bit levels (a job has
        // n < 2^32); the generic pass for a 16-bit input with byte levels
        // after it.
        if (scatter) {
            if (win == 2 && wout == 1) {
                if constexpr (var_has(VAR, vcode(2, 1, true))) level_tile<uint16_t, uint8_t, true, true>(a, tile, s.g16);
            } else if (win == 2) {
                if constexpr (var_has(VAR, vcode(2, 2, true))) level_tile_u16<true, true>(a, tile, s.u16);
            } else if (wout == 1) {
                if constexpr (var_has(VAR, vcode(4, 1, true))) level_tile_u32<uint8_t, true, true>(a, tile, s.u32);
            } else if (wout == 2) {
                if constexpr (var_has(VAR, vcode(4, 2, true))) level_tile_u32<uint16_t, true, true>(a, tile, s.u32);
            } else {
                if constexpr (var_has(VAR, vcode(4, 4, true))) level_tile_u32<uint32_t, true, true>(a, tile, s.u32);
            }
        } else {
            if (win == 2) {
                if constexpr (var_has(VAR, vcode(2, 0, false))) level_tile_u16<false, true>(a, tile, s.u16);
            } else {
                if constexpr (var_has(VAR, vcode(4, 0, false))) level_tile_u32<uint32_t, false, true>(a, tile, s.u32);
            }
        }
    }
}

__device__ __forceinline__ void fused_item(const JobDev &j, uint32_t seg, LdsFusedAll &s) {
    FusedArgs f;
    f.in0 = j.seq;
    f.S0 = j.S0;
    f.S1 = j.S1;
    f.C = j.C;
    f.D = j.D;
    f.sigma = j.sigma;
    f.n = j.n;
    f.L = j.L;
    f.bits = j.bits;
    f.W = j.W;
    f.rank = j.rank;
    f.rank_len = j.rank_len;
    f.sel1 = j.sel1;
    f.sel0 = j.sel0;
    f.cap = j.cap;
    f.status = j.ctl + kCtlStatus;
    f.l0 = j.ctl + kCtlFusedL0;
    f.segb = j.segb;
    const uint32_t wi = j.in_bytes, wm = j.mid_bytes;
    if (wm == 1) {
        if (wi == 1) fused_segment<uint8_t, uint8_t, kFusedBytes>(f, seg, s.f8);
        else if (wi == 2) fused_segment<uint16_t, uint8_t, kFusedBytes>(f, seg, s.f8);
        else fused_segment<uint32_t, uint8_t, kFusedBytes>(f, seg, s.f8);
    } else if (wm == 2) {
        if (wi == 2) fused_segment<uint16_t, uint16_t, kFusedBytes>(f, seg, s.f16);
        else fused_segment<uint32_t, uint16_t, kFusedBytes>(f, seg, s.f16);
    } else {
        fused_segment<uint32_t, uint32_t, kFusedBytes>(f, seg, s.f32);
    }
}

// One work item.  KINDS: the item kinds this kernel is built for; LDS: its
// shared-memory type (one of the Lds* types above).
template <uint32_t KINDS, typename LDS>
__device__ __forceinline__ void run_item(const Args &b, uint32_t it, LDS &s, uint32_t *s_flag) {
    const uint32_t si = __builtin_amdgcn_readfirstlane(b.seg_of[it]);
    const Seg sg = load_const(b.segs + si);
    const uint32_t jid = __builtin_amdgcn_readfirstlane(sg.job), kind = __builtin_amdgcn_readfirstlane(sg.kind);
    const uint32_t count = __builtin_amdgcn_readfirstlane(sg.count);
    const uint32_t tile = it - __builtin_amdgcn_readfirstlane(sg.first);
    const JobDev j = load_const(b.jobs + jid);
    uint32_t *ctl = j.ctl;
    if (kind == kKindHist) {
        if constexpr ((KINDS & kHasTileHist) != 0) {
            LdsHistB &h = [&]() -> LdsHistB & {
                if constexpr (KINDS == kHasAll) return s.hist;
                else return s;
            }();
            if (j.in_bytes == 1) hist_item<uint8_t>(j, tile, h);
            else if (j.in_bytes == 2) hist_item<uint16_t>(j, tile, h);
            else hist_item<uint32_t>(j, tile, h);
            finish_item(b, ctl + kCtlDone, count, s_flag);
        }
    } else if (kind == kKindJobHist) {
        if constexpr (KINDS == kHasAll) {
            if (j.in_bytes == 2) job_hist_small<uint16_t>(j, s.hist);
            else job_hist_small<uint32_t>(j, s.hist);
            finish_item(b, ctl + kCtlDone, count, s_flag);
        }
    } else if (kind == kKindPrep) {
        if constexpr ((KINDS & kHasPrep) != 0) {
            wait_for(b, ctl + kCtlDone, j.hist_items, ctl + kCtlStatus);
            if constexpr (KINDS == kHasAll) prep_item<4>(j, s.prep, b.fuse, b);
            else prep_item<4>(j, s, b.fuse, b);
            publish(b, ctl + kCtlReady);
        }
    } else if (kind == kKindFused) {
        if constexpr ((KINDS & kHasFused) != 0) {
            wait_for(b, ctl + kCtlReady, 1u, ctl + kCtlStatus);  // tables and the fused level are known
            const uint32_t l0 = ld_u32(ctl + kCtlFusedL0);
            if (l0 >= j.L) return;
            if (l0 > 0) wait_for(b, ctl + kCtlReady + l0, 1u, ctl + kCtlStatus);
            if constexpr (KINDS == kHasAll) fused_item(j, tile, s.fu);
            else fused_item(j, tile, s);
        }
    } else {
        if constexpr ((KINDS & kHasLevel) != 0) {
            auto &lv = [&]() -> auto & {
                if constexpr (KINDS == kHasAll) return s.lv;
                else return s;
            }();
            const uint32_t l = kind - kKindLevel;
            wait_for(b, ctl + kCtlReady + l, 1u, ctl + kCtlStatus);
            level_item<KINDS>(j, l, tile, lv, false);
            if (finish_item(b, ctl + kCtlDone + 1 + l, count, s_flag) && l + 1 < j.L) {
                tile_prefix_block(j.cnt + (uint64_t)(l + 1) * j.Tpad, j.pre + (uint64_t)(l + 1) * j.Tpad, j.Tm,
                                  lv.scan);
                publish(b, ctl + kCtlReady + 1 + l);
            }
        }
    }
}

// A listed item of a per-phase level or fused launch: (job, tile or segment).
template <uint32_t KINDS, typename LDS, uint32_t VAR>
__device__ __forceinline__ void run_listed(const Args &b, uint2 e, LDS &s) {
    const uint32_t jid = __builtin_amdgcn_readfirstlane(e.x), it = __builtin_amdgcn_readfirstlane(e.y);
    const JobDev j = load_const(b.jobs + jid);
    if constexpr (KINDS == kHasFused) {
        fused_item(j, it, s);
    } else if constexpr ((KINDS & kHasLevel) != 0 && (KINDS & ~kHasLevel) == 0) {
        level_item<KINDS, VAR>(j, b.level, it, s, true);
    }
}

template <uint32_t KINDS, typename LDS, uint32_t VAR = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(waves_for(KINDS, VAR)))) void
work_kernel(Args b) {
    __shared__ LDS s;
    __shared__ uint32_t s_first, s_flag;
    if constexpr (KINDS == kHasFused || ((KINDS & kHasLevel) != 0 && (KINDS & ~kHasLevel) == 0)) {
        if (b.list) {
            // The phase's live items, a chunk per block and grid stride.
            const uint32_t count = __builtin_amdgcn_readfirstlane(ld_u32(b.live + b.phase));
            for (uint64_t first = (uint64_t)blockIdx.x * b.chunk; first < count;
                 first += (uint64_t)gridDim.x * b.chunk) {
                const uint32_t last = (uint32_t)min(first + b.chunk, (uint64_t)count);
                for (uint32_t i = (uint32_t)first; i < last; ++i) {
                    __syncthreads();  // the previous item's LDS is free
                    run_listed<KINDS, LDS, VAR>(b, load_const(b.list + b.lo + i), s);
                }
            }
            return;
        }
    }
    if constexpr (VAR != 0) return;  // built for listed launches only
    if (!b.fenced) {
        // One launch per phase: no item waits for another of the same
        // launch, so blocks take their chunks by index (no shared queue head,
        // whose atomics would serialise the launch).
        for (uint64_t first = b.lo + (uint64_t)blockIdx.x * b.chunk; first < b.hi;
             first += (uint64_t)gridDim.x * b.chunk) {
            const uint32_t last = (uint32_t)min(first + b.chunk, (uint64_t)b.hi);
            for (uint32_t it = (uint32_t)first; it < last; ++it) {
                __syncthreads();  // the previous item's LDS is free
                run_item<KINDS, LDS>(b, it, s, &s_flag);
            }
        }
        return;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint64_t f = (uint64_t)b.lo + atomicAdd(b.head, b.chunk);
            s_first = (uint32_t)min(f, (uint64_t)b.hi);
        }
        __syncthreads();
        const uint32_t first = s_first;
        if (first >= b.hi) break;
        const uint32_t last = min(first + b.chunk, b.hi);
        for (uint32_t it = first; it < last; ++it) {
            __syncthreads();  // the previous item's LDS is free
            run_item<KINDS, LDS>(b, it, s, &s_flag);
        }
    }
}

__global__ void clear_kernel(uint64_t *a, uint64_t na) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += stride) a[i] = 0;
}

// Per-phase launches, before level l >= 1: one wave per job scans the
// level's count-ahead totals (atomics of the previous launch) into its tile
// prefixes and lists the level's tiles unless the level is fused.
__global__ __launch_bounds__(kBlock) void level_setup_kernel(Args b, uint32_t njobs, uint32_t l, uint32_t base_byte,
                                                             uint32_t base_wide) {
    const uint32_t jid = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + threadIdx.x / kWave);
    if (jid >= njobs) return;
    const JobDev j = load_const(b.jobs + jid);
    if (j.n == 0 || l >= j.L || ld_u32(j.ctl + kCtlFusedL0) <= l) return;
    const uint32_t lane = lane_id(), T = j.Tm;
    const uint32_t *cnt = j.cnt + (uint64_t)l * j.Tpad;
    uint64_t *pre = j.pre + (uint64_t)l * j.Tpad;
    uint64_t carry = 0;
    for (uint32_t t0 = 0; t0 < T; t0 += kWave) {
        const uint32_t t = t0 + lane, c = t < T ? ld_u32(cnt + t) : 0u;
        const uint32_t inc = wave_incl_scan_u32(c, lane);
        if (t < T) pre[t] = carry + inc - c;
        carry += __shfl(inc, kWave - 1, kWave);
    }
    const uint32_t wide = j.mid_bytes > 1 ? 1u : 0u;
    uint32_t at = 0;
    if (lane == 0) at = atomicAdd(b.live + 3 + 2 * l + wide, T);
    at = __shfl(at, 0, kWave);
    uint2 *out = b.list + (wide ? base_wide : base_byte) + at;
    for (uint32_t t = lane; t < T; t += kWave) out[t] = make_uint2(jid, t);
}

// ---------------------------------------------------------------------------
// Host side.
struct HostJob {
    uint64_t n, sigma;
    uint32_t L, in_bytes, mid_bytes, reps, T0, Tm, Tpad;
    bool job_hist;  // counted by one whole-job item (large alphabet that fits packed LDS bins)
    uint64_t off_ctl, off_symcnt, off_cnt, off_pre, off_D, off_S0, off_S1, off_segb;
    uint32_t nseg;
};

struct HostPlan {
    std::vector<HostJob> jobs;
    std::vector<Seg> segs;
    std::vector<uint32_t> phase_first;
    std::vector<uint32_t> phase_var;  // per phase: the one tile variant of a level phase, else 0
    uint64_t items = 0, off_jobs = 0, off_segs = 0, off_seg_of = 0, off_list = 0, clear_bytes = 0, total = 0;
};

static uint32_t levels_of(uint64_t sigma) {
    uint32_t L = 0;
    while (L < 64 && (1ull << L) < sigma) ++L;
    return L;
}

static int make_batch_plan(const wt_job *jobs, uint32_t njobs, HostPlan &hp) {
    if (njobs > 0 && !jobs) return WT_ERR_ARG;
    hp.jobs.resize(njobs);
    uint32_t maxL = 0;
    for (uint32_t i = 0; i < njobs; ++i) {
        const wt_job &q = jobs[i];
        HostJob &h = hp.jobs[i];
        if (q.sigma == 0 || (q.sym_bytes != 1 && q.sym_bytes != 2 && q.sym_bytes != 4)) return WT_ERR_ARG;
        if (q.sigma > (1ull << (8 * q.sym_bytes))) return WT_ERR_ARG;
        if (q.n >= (1ull << 32)) return WT_ERR_RANGE;
        h.n = q.n;
        h.sigma = q.sigma;
        h.L = levels_of(q.sigma);
        if (h.L > (uint32_t)kMaxLevels) return WT_ERR_RANGE;
        h.in_bytes = q.sym_bytes;
        h.mid_bytes = h.L <= 8 ? 1u : (h.L <= 16 ? 2u : 4u);
        h.reps = q.sigma + 1 <= kHistWords ? (uint32_t)std::min<uint64_t>(16, kHistWords / (q.sigma + 1)) : 0u;
        h.T0 = (uint32_t)cdiv(q.n, 1ull << tile_shift_for(h.in_bytes));
        h.Tm = (uint32_t)cdiv(q.n, 1ull << tile_shift_for(h.mid_bytes));
        h.Tpad = (uint32_t)align_up(std::max<uint32_t>(std::max(h.T0, h.Tm), 1), 4);
        h.job_hist = h.reps == 0 && q.sigma <= kJobHistMaxSigma && q.n > 0;
        maxL = std::max(maxL, h.n ? h.L : 0u);
    }
    // Clear region: header, control words of every job, then every job's
    // symbol counts and count-ahead totals.
    uint64_t o = kHeaderBytes;
    for (auto &h : hp.jobs) {
        h.off_ctl = o;
        o += kCtlWords * 4;
    }
    for (auto &h : hp.jobs) {
        h.off_symcnt = o;
        o = align_up(o + 4 * h.sigma, 256);
        h.off_cnt = o;
        o = align_up(o + 4ull * h.L * h.Tpad, 256);
    }
    hp.clear_bytes = o;
    // Segments in queue order.
    hp.segs.clear();
    hp.phase_first.clear();
    uint64_t items = 0;
    auto add = [&](uint32_t job, uint32_t kind, uint32_t count) {
        if (count == 0) return;
        hp.segs.push_back(Seg{job, kind, (uint32_t)items, count});
        items += count;
    };
    // Phases: tile histograms, whole-job histograms, tables, level 0, 1, ...,
    // fused tail levels.
    hp.phase_first.push_back(0);
    for (uint32_t i = 0; i < njobs; ++i)
        if (!hp.jobs[i].job_hist) add(i, kKindHist, hp.jobs[i].T0);
    // The whole-job histograms and the tables run one block per job, so a
    // large job started last would set the phase's end: their items go
    // largest first (by n, resp. by sigma, then n).
    std::vector<uint32_t> ord(njobs);
    for (uint32_t i = 0; i < njobs; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return hp.jobs[x].n > hp.jobs[y].n; });
    hp.phase_first.push_back((uint32_t)items);
    for (uint32_t i : ord)
        if (hp.jobs[i].job_hist) add(i, kKindJobHist, 1);
    hp.phase_first.push_back((uint32_t)items);
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) {
        return hp.jobs[x].sigma != hp.jobs[y].sigma ? hp.jobs[x].sigma > hp.jobs[y].sigma : hp.jobs[x].n > hp.jobs[y].n;
    });
    for (uint32_t i : ord) add(i, kKindPrep, 1);
    for (uint32_t l = 0; l < maxL; ++l) {
        for (int wide = 0; wide < 2; ++wide) {  // byte-symbol tiles, then wider ones
            hp.phase_first.push_back((uint32_t)items);
            uint32_t var = ~0u;  // the one variant of the phase's tiles, 0 when they mix
            for (uint32_t i = 0; i < njobs; ++i) {
                const HostJob &h = hp.jobs[i];
                const uint32_t win = l == 0 ? h.in_bytes : h.mid_bytes;
                if (h.n > 0 && l < h.L && (win > 1) == (wide != 0)) {
                    add(i, kKindLevel + l, l == 0 ? h.T0 : h.Tm);
                    const bool scatter = l + 1 < h.L;
                    const uint32_t v = vcode(win, scatter ? h.mid_bytes : 0u, scatter);
                    var = var == ~0u || var == v ? v : 0u;
                }
            }
            hp.phase_var.push_back(var == ~0u ? 0u : var);
        }
        if (items >= (1ull << 31)) return WT_ERR_RANGE;
    }
    hp.phase_first.push_back((uint32_t)items);
    for (uint32_t i = 0; i < njobs; ++i) {  // fused tail levels: one item per segment
        HostJob &h = hp.jobs[i];
        h.nseg = h.n > 0 && h.L >= 2 ? (uint32_t)cdiv(h.n, fused_half(h.mid_bytes)) : 0u;
        add(i, kKindFused, h.nseg);
    }
    if (items >= (1ull << 31)) return WT_ERR_RANGE;
    hp.phase_first.push_back((uint32_t)items);
    hp.items = items;
    o = align_up(o, 256);
    hp.off_jobs = o;
    o = align_up(o + sizeof(JobDev) * njobs, 256);
    hp.off_segs = o;
    o = align_up(o + sizeof(Seg) * hp.segs.size(), 256);
    hp.off_seg_of = o;
    o = align_up(o + 4 * items, 256);
    hp.off_list = o;
    o = align_up(o + 8 * items, 256);
    for (auto &h : hp.jobs) {
        h.off_pre = o;
        o = align_up(o + 8ull * h.L * h.Tpad, 256);
        h.off_D = o;
        o = align_up(o + (h.L ? 8ull * ((2ull << h.L) - 2) : 0), 256);
        const uint64_t sbytes = h.L >= 2 ? align_up(h.n * h.mid_bytes, 256) : 0;
        h.off_S0 = o;
        o += sbytes;
        h.off_S1 = o;
        o += h.L >= 3 ? sbytes : 0;
        h.off_segb = o;
        o = align_up(o + 4ull * (h.nseg + 1), 256);
    }
    hp.total = std::max<uint64_t>(o, 256);
    return WT_OK;
}

// Resident blocks of work_kernel: per CU and CUs of the current device.
static int residency(uint32_t &per_cu, uint32_t &cus) {
    static int s_per_cu = 0, s_cus = 0;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (!s_per_cu) {
        int dev = 0, c = 0, b = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            return WT_ERR_HIP;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, work_kernel<kHasAll, LdsBatch>, kBlock, 0) != hipSuccess ||
            b <= 0)
            b = 1;
        s_cus = c;
        s_per_cu = b;
    }
    per_cu = (uint32_t)s_per_cu;
    cus = (uint32_t)s_cus;
    return WT_OK;
}

}  // namespace batch
}  // namespace wt

using namespace wt;
using namespace wt::batch;

extern "C" int wt_batch_plan(const wt_job *jobs, uint32_t njobs, wt_batch_layout *out) {
    if (!out) return WT_ERR_ARG;
    HostPlan hp;
    int rc = make_batch_plan(jobs, njobs, hp);
    if (rc) return rc;
    *out = wt_batch_layout{};
    out->scratch_bytes = hp.total;
    out->clear_bytes = hp.clear_bytes;
    out->njobs = njobs;
    out->nsegs = (uint32_t)hp.segs.size();
    out->items = (uint32_t)hp.items;
    out->phases = (uint32_t)hp.phase_first.size() - 1;
    for (size_t i = 0; i < hp.phase_first.size(); ++i) out->phase_first[i] = hp.phase_first[i];
    for (size_t i = 0; i < hp.phase_var.size(); ++i) out->phase_var[3 + i] = hp.phase_var[i];
    out->off_jobs = hp.off_jobs;
    out->off_segs = hp.off_segs;
    out->off_seg_of = hp.off_seg_of;
    out->off_list = hp.off_list;
    return WT_OK;
}

extern "C" int wt_batch_prepare(const wt_job *jobs, uint32_t njobs, const wt_batch_layout *lay, void *d_scratch,
                                uint64_t scratch_bytes, void *stream) {
    if (!lay || !d_scratch || ((uintptr_t)d_scratch & 255u)) return WT_ERR_ARG;
    HostPlan hp;
    int rc = make_batch_plan(jobs, njobs, hp);
    if (rc) return rc;
    if (lay->njobs != njobs || lay->items != hp.items || lay->scratch_bytes != hp.total || lay->off_list != hp.off_list)
        return WT_ERR_ARG;
    if (scratch_bytes < hp.total) return WT_ERR_SCRATCH;
    unsigned char *sc = (unsigned char *)d_scratch;
    std::vector<JobDev> dev(njobs);
    for (uint32_t i = 0; i < njobs; ++i) {
        const wt_job &q = jobs[i];
        const HostJob &h = hp.jobs[i];
        const wt_outputs &o = q.out;
        if (!o.C) return WT_ERR_ARG;
        if (h.L > 0 && (!o.rank || !o.sel1 || !o.sel0 || !o.sel_counts)) return WT_ERR_ARG;  // directories required
        if (h.n > 0 && (!q.seq || ((uintptr_t)q.seq & 15u))) return WT_ERR_ARG;
        if (h.n > 0 && h.L > 0 && !o.bits) return WT_ERR_ARG;
        JobDev &d = dev[i];
        d = JobDev{};
        d.seq = q.seq;
        d.n = h.n;
        d.sigma = h.sigma;
        d.L = h.L;
        d.in_bytes = h.in_bytes;
        d.mid_bytes = h.mid_bytes;
        d.reps = h.reps;
        d.T0 = h.T0;
        d.Tm = h.Tm;
        d.Tpad = h.Tpad;
        d.hist_items = h.job_hist ? 1u : h.T0;
        d.W = cdiv(h.n, 64);
        d.rank_len = cdiv(h.n, WT_RANK_BLOCK_BITS) + 1;
        d.cap = cdiv(h.n, WT_SELECT_SAMPLE) + 1;
        d.bits = o.bits;
        d.C = o.C;
        d.rank = o.rank;
        d.sel1 = o.sel1;
        d.sel0 = o.sel0;
        d.sel_counts = o.sel_counts;
        d.ctl = (uint32_t *)(sc + h.off_ctl);
        d.symcnt = (uint32_t *)(sc + h.off_symcnt);
        d.cnt = (uint32_t *)(sc + h.off_cnt);
        d.pre = (uint64_t *)(sc + h.off_pre);
        d.D = (uint64_t *)(sc + h.off_D);
        d.S0 = sc + h.off_S0;
        d.S1 = sc + h.off_S1;
        d.segb = (uint32_t *)(sc + h.off_segb);
        d.nseg = h.nseg;
        d.id = i;
    }
    std::vector<uint32_t> seg_of(hp.items);
    for (uint32_t s = 0; s < hp.segs.size(); ++s)
        for (uint32_t t = 0; t < hp.segs[s].count; ++t) seg_of[hp.segs[s].first + t] = s;
    hipStream_t st = (hipStream_t)stream;
    if (njobs && hipMemcpyAsync(sc + hp.off_jobs, dev.data(), sizeof(JobDev) * njobs, hipMemcpyHostToDevice, st))
        return WT_ERR_HIP;
    if (!hp.segs.empty() &&
        hipMemcpyAsync(sc + hp.off_segs, hp.segs.data(), sizeof(Seg) * hp.segs.size(), hipMemcpyHostToDevice, st))
        return WT_ERR_HIP;
    if (hp.items && hipMemcpyAsync(sc + hp.off_seg_of, seg_of.data(), 4 * hp.items, hipMemcpyHostToDevice, st))
        return WT_ERR_HIP;
    // The host tables are released on return: wait for the copies.
    return hipStreamSynchronize(st) == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_batch_run(const wt_batch_layout *lay, const wt_tune *tune, void *d_scratch, void *stream) {
    if (!lay || !d_scratch || ((uintptr_t)d_scratch & 255u)) return WT_ERR_ARG;
    wt_tune t = tune ? *tune : wt_tune{};
    if (t.mode > WT_BATCH_PER_PHASE) return WT_ERR_ARG;
    const uint32_t chunk = t.chunk ? t.chunk : 1u;
    const uint32_t spin = t.spin_limit ? t.spin_limit : (1u << 22);
    if (chunk > 4096) return WT_ERR_ARG;
    uint32_t max_per_cu = 0, cus = 0;
    if (residency(max_per_cu, cus) != WT_OK) return WT_ERR_HIP;
    const uint32_t per_cu = t.blocks_per_cu ? std::min(t.blocks_per_cu, max_per_cu) : max_per_cu;
    const uint64_t resident = (uint64_t)per_cu * cus;
    hipStream_t s = (hipStream_t)stream;
    unsigned char *sc = (unsigned char *)d_scratch;
    const uint64_t nclear = lay->clear_bytes / 8;
    clear_kernel<<<(unsigned)std::max<uint64_t>(1, std::min<uint64_t>(cdiv(nclear, kBlock), 8192)), kBlock, 0, s>>>(
        (uint64_t *)sc, nclear);
    Args a;
    a.jobs = (const JobDev *)(sc + lay->off_jobs);
    a.segs = (const Seg *)(sc + lay->off_segs);
    a.seg_of = (const uint32_t *)(sc + lay->off_seg_of);
    a.abort = (uint32_t *)sc + kAbortWord;
    a.chunk = chunk;
    a.spin_limit = spin;
    a.fenced = t.mode == WT_BATCH_PERSISTENT ? 1u : 0u;
    a.fuse = fused_levels_setting();
    const uint32_t last = lay->phases - 1;
    // Lists of live items (per-phase launches only).
    a.list = a.fenced ? nullptr : (uint2 *)(sc + lay->off_list);
    a.live = (uint32_t *)sc + kLiveWord;
    a.base0[0] = lay->phase_first[std::min(3u, last)];
    a.base0[1] = lay->phase_first[std::min(4u, last)];
    a.base_fused = lay->phase_first[last];
    a.phase_fused = last;
    auto launch = [&](uint32_t phase, uint32_t lo, uint32_t hi) {
        if (hi <= lo) return;
        a.head = (uint32_t *)sc + phase;
        a.lo = lo;
        a.hi = hi;
        a.phase = phase;
        a.level = phase >= 3 && phase < last ? (phase - 3) / 2 : 0u;
        // Persistent launch: resident blocks take items from the queue.  One
        // launch per phase: one block per chunk unless blocks_per_cu caps it;
        // a listed launch (levels, fused) at most two rounds of resident
        // blocks, which stride over the live items.
        const uint64_t chunks = cdiv(hi - lo, chunk);
        const bool listed = !a.fenced && phase >= 3;
        const uint64_t cap = (a.fenced || t.blocks_per_cu) ? resident : (listed ? 2 * resident : (1ull << 31) - 1);
        const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(cap, chunks));
        if (a.fenced) work_kernel<kHasAll, LdsBatch><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if (phase == 0) work_kernel<kHasTileHist, LdsHistB><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if (phase == 1) job_hist_kernel<<<(unsigned)std::min<uint64_t>(hi - lo, 1u << 20), kJHThreads, 0, s>>>(a);
        else if (phase == 2) work_kernel<kHasPrep, LdsPrep><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if (phase == last) work_kernel<kHasFused, LdsFusedAll><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if (listed && lay->phase_var[phase] == vcode(1, 1, true))
            work_kernel<kHasLevel8, LdsLevels8, vcode(1, 1, true)><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if (listed && lay->phase_var[phase] == vcode(1, 0, false))
            work_kernel<kHasLevel8, LdsLevels8, vcode(1, 0, false)><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if (listed && lay->phase_var[phase] == vcode(2, 2, true))
            work_kernel<kHasLevelWide, LdsLevelsWide, vcode(2, 2, true)><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if (listed && lay->phase_var[phase] == vcode(2, 0, false))
            work_kernel<kHasLevelWide, LdsLevelsWide, vcode(2, 0, false)><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if (listed && lay->phase_var[phase] == vcode(4, 4, true))
            work_kernel<kHasLevelWide, LdsLevelsWide, vcode(4, 4, true)><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else if ((phase - 3) % 2 == 0) work_kernel<kHasLevel8, LdsLevels8><<<(unsigned)grid, kBlock, 0, s>>>(a);
        else work_kernel<kHasLevelWide, LdsLevelsWide><<<(unsigned)grid, kBlock, 0, s>>>(a);
    };
    if (t.mode == WT_BATCH_PERSISTENT) {
        launch(0, 0, lay->items);
    } else {
        for (uint32_t p = 0; p < lay->phases; ++p) {
            if (p >= 5 && p < last && (p - 3) % 2 == 0 && lay->phase_first[p] < lay->phase_first[p + 2]) {
                const uint32_t l = (p - 3) / 2;  // level l >= 1 has tiles: prefixes and lists first
                level_setup_kernel<<<(unsigned)std::max<uint64_t>(1, cdiv(lay->njobs, kWaves)), kBlock, 0, s>>>(
                    a, lay->njobs, l, lay->phase_first[p], lay->phase_first[p + 1]);
            }
            launch(p, lay->phase_first[p], lay->phase_first[p + 1]);
        }
    }
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_batch_status(const wt_batch_layout *lay, const void *d_scratch, int32_t *codes, void *stream) {
    if (!lay || !d_scratch) return WT_ERR_ARG;
    std::vector<uint32_t> ctl((size_t)lay->njobs * kCtlWords);
    hipStream_t s = (hipStream_t)stream;
    if (lay->njobs && hipMemcpyAsync(ctl.data(), (const unsigned char *)d_scratch + kHeaderBytes, ctl.size() * 4,
                                     hipMemcpyDeviceToHost, s) != hipSuccess)
        return WT_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return WT_ERR_HIP;
    int worst = WT_OK;
    for (uint32_t i = 0; i < lay->njobs; ++i) {
        const uint32_t st = ctl[(size_t)i * kCtlWords + kCtlStatus];
        const int code = (st & kStatusTimeout) ? WT_ERR_TIMEOUT : (st & kStatusSymbol) ? WT_ERR_SYMBOL : WT_OK;
        if (codes) codes[i] = code;
        if (code == WT_ERR_TIMEOUT || worst == WT_OK) worst = code == WT_OK ? worst : code;
    }
    return worst;
}
