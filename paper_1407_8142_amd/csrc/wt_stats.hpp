// Byte alphabets without a histogram pass.
//
// Level l's node table D_l needs the start and the zeros of each of its 2^l
// nodes.  Both follow from what the level above counts while it scatters:
//   - a piece of level l is the part of one of its tiles inside one of its
//     nodes (the common refinement of the tile and node partitions of the
//     level's positions).  Piece (tile t, node p) gets index t + p: going
//     along the positions, each next piece moves to a later tile, a later
//     node or both, so the indices of the nonempty pieces strictly increase
//     with their positions (and are at most T + P - 1).
//   - level l-1's count-ahead adds, for every symbol it scatters, a zero of
//     bit k_l to the piece the symbol lands in (destination tile plus its
//     top l bits, its node at level l).
//   - an exclusive scan E of the piece counts then gives the zeros of B_l
//     before any position x as E[tile(x) + node(x)], where node(x) is the
//     last node starting at or before x: every piece before x has a smaller
//     index, every piece at or after x an index at least that large.  So
//     one scan yields both the tile prefixes (x = a tile start) and the
//     zeros before every node (x = a node start, also for empty nodes).
//   - node starts CL_l[p] = C[p * 2^(L-l)] follow level by level:
//     CL_{l+1}[2p] = CL_l[p], CL_{l+1}[2p+1] = CL_l[p] + NZ_l[p], with NZ_l[p]
//     the zeros of node p; the last level's give C.
// Level 0 has one node, so its pieces are its tiles: a read-only pass
// counts the zeros of the top bit per tile (and checks the symbols).
//
// Pipeline (one stream): stats_prep_u8, then per level stats_scan and the
// byte level pass counting per piece of the next level.
#pragma once

#include "wt_kernels.hpp"

namespace wt {

constexpr uint32_t kBadTile = 1u << 31;  // in a level-0 tile count: the tile holds a symbol >= sigma
constexpr int kStatsMaxNodes = 128;      // nodes of a byte alphabet's deepest level

// Entries per level of the piece counts: T tiles + at most 2^(L-1) nodes,
// plus the total.
__host__ __device__ inline uint64_t piece_stride(uint64_t T, uint32_t L) {
    return align_up(T + (1ull << (L - 1)) + 1, 64);  // a multiple of 4: vector loads of 4 counts
}

// ---------------------------------------------------------------------------
// One wave per level-0 tile of 16 KiB (kPrepWaves tiles per block, no
// barrier): sixteen 16-byte loads per lane in flight, cnt0[tile] = zeros of
// bit k in the tile, with kBadTile set when CHECK (sigma < 256) finds a
// byte >= sigma.  The threads also clear [0, nclear) of `clear`, counters
// that the level passes accumulate into.
constexpr int kPrepWaves = 4;

template <bool CHECK>
__global__ __launch_bounds__(kPrepWaves * kWave) void stats_prep_u8(const uint8_t *__restrict__ S, uint32_t n,
                                                                    uint32_t k, uint32_t sigma, uint32_t *cnt0,
                                                                    uint32_t *clear, uint64_t nclear) {
    constexpr int kLoads = 16384 / 16 / kWave;  // 16
    const int lane = lane_id();
    const uint64_t gtid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // Counters for the level passes (nothing reads them before this kernel ends).
    for (uint64_t i = gtid; i < nclear; i += (uint64_t)gridDim.x * blockDim.x) clear[i] = 0;
    const uint32_t tile = blockIdx.x * kPrepWaves + threadIdx.x / kWave;
    const uint32_t ntiles = (n + 16383u) / 16384u;
    if (tile >= ntiles) return;
    const uint32_t t0 = tile * 16384u;
    const uint32_t len = min(16384u, n - t0);
    const uint4 *in = reinterpret_cast<const uint4 *>(S + t0) + lane;
    uint4 d[kLoads];
    if (len == 16384u) {
#pragma unroll
        for (int r = 0; r < kLoads; ++r) d[r] = in[r * kWave];
    } else {
#pragma unroll
        for (int r = 0; r < kLoads; ++r) {
            const uint32_t p = (uint32_t)(r * kWave + lane) * 16u;
            if (p + 16 <= len) {
                d[r] = in[r * kWave];
            } else {
                const uint32_t nv = clamp_count(len, p, 16u);
                uint32_t w[4] = {0, 0, 0, 0};  // past the end: byte 0, no one and no bad symbol
                for (uint32_t j = 0; j < nv; ++j) w[j >> 2] |= (uint32_t)S[t0 + p + j] << (8 * (j & 3));
                d[r] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    const uint32_t M = 0x01010101u << k;
    uint32_t ones = 0;
    uint32_t hi = 0;  // largest byte seen (CHECK)
#pragma unroll
    for (int r = 0; r < kLoads; ++r) {
        const uint32_t w[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ones += (uint32_t)__popc(w[j] & M);
            if (CHECK)
                hi = max(hi, max(max(w[j] & 0xFFu, (w[j] >> 8) & 0xFFu), max((w[j] >> 16) & 0xFFu, w[j] >> 24)));
        }
    }
    const bool bad = __ballot(CHECK && hi >= sigma) != 0;
    const uint32_t t = wave_sum_u32(ones);
    if (lane == 0) cnt0[tile] = (len - t) | (bad ? kBadTile : 0u);
}

// ---------------------------------------------------------------------------
// Level l's statistics, one block of kStatsThreads:
//   E        = exclusive scan of the piece counts (at level 0 the tiles'
//              kBadTile flags are ORed into the status word);
//   CL_l     = node starts, from CL_{l-1} and NZ_{l-1} (CL_0 = {0, n});
//   E        also goes to memory: the passes of level l take a tile's zero
//            prefix as E[t + node of its first position];
//   ZB[p]    = zeros before node p = E[tile(CL_l[p]) + p], NZ_l[p] = ZB[p+1] - ZB[p];
//   D_l      = the level pass's node table: D_l[2p] = ones of B_l before
//              node p = CL_l[p] - ZB[p], D_l[2p+1] = zeros before node p+1;
//   at the last level, C[c] = CL_L[c] for c <= sigma.
struct StatsArgs {
    const uint32_t *pieces; // level l's piece counts (T + 2^l + 1 used)
    uint32_t *E;            // their exclusive prefixes (read by the level's passes; may be `pieces`)
    uint64_t T;             // tiles of the level
    uint32_t tile_shift;    // log2 positions per tile
    uint32_t level, L;
    uint64_t n, sigma;
    uint32_t *status;       // written at level 0
    uint64_t *NZ, *CL;      // every level's: NZ_l at 2^l - 1, CL_l at 2^l - 1 + l
    uint64_t *D;            // D_l (2^(l+1) entries)
    uint64_t *C;            // written at the last level
};

constexpr int kStatsThreads = 1024;
constexpr int kStatsPer = 20;                            // piece counts per thread and round
constexpr int kStatsRound = kStatsThreads * kStatsPer;   // 20480: one round up to n = 2^28 + ...

__global__ __launch_bounds__(kStatsThreads) void stats_scan(StatsArgs a) {
    __shared__ uint32_t s_w[kStatsThreads / kWave];
    __shared__ uint32_t s_e[kStatsRound];  // this round's exclusive prefixes
    __shared__ uint64_t s_cl[kStatsMaxNodes + 1];
    __shared__ uint64_t s_zb[kStatsMaxNodes + 1];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t l = a.level, P = 1u << l;
    const bool lvl0 = l == 0;
    const uint64_t npieces = a.T + P;  // E[npieces] is the level's total

    // 1. Node starts of this level (their loads go out with the first round's).
    uint64_t *NZ = a.NZ + (P - 1), *CL = a.CL + (P - 1) + l;
    if ((uint32_t)tid <= P) {
        uint64_t start = a.n;
        if ((uint32_t)tid < P) {
            if (lvl0) {
                start = 0;
            } else {
                const uint64_t *NZp = a.NZ + (P / 2 - 1), *CLp = a.CL + (P / 2 - 1) + (l - 1);
                const uint32_t q = (uint32_t)tid >> 1;
                start = CLp[q] + ((tid & 1) ? NZp[q] : 0ull);
            }
        }
        s_cl[tid] = start;
        CL[tid] = start;
    }

    // 2. Exclusive scan of the piece counts, a round of kStatsRound at a time
    //    (one round for up to 2^28 byte symbols), to memory and, for the
    //    round, to LDS, where node p's prefix (index tile(CL[p]) + p) is
    //    picked.
    uint64_t carry = 0;
    bool bad = false;
    for (uint64_t c0 = 0; c0 <= npieces; c0 += kStatsRound) {
        const uint64_t base = c0 + (uint64_t)tid * kStatsPer;
        uint32_t v[kStatsPer], own = 0;
        if (base + kStatsPer <= npieces + 1) {
            const uint4 *p4 = reinterpret_cast<const uint4 *>(a.pieces + base);
#pragma unroll
            for (int q = 0; q < kStatsPer / 4; ++q) {
                const uint4 x = p4[q];
                v[4 * q] = x.x;
                v[4 * q + 1] = x.y;
                v[4 * q + 2] = x.z;
                v[4 * q + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kStatsPer; ++j) v[j] = base + j <= npieces ? a.pieces[base + j] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kStatsPer; ++j) {
            if (lvl0) {
                bad |= (v[j] & kBadTile) != 0;
                v[j] &= ~kBadTile;
            }
            own += v[j];
        }
        const uint32_t inc = wave_incl_scan_u32(own, lane);
        if (lane == kWave - 1) s_w[wave] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kStatsThreads / kWave; ++w) {
            const uint32_t x = s_w[w];
            before += w < wave ? x : 0u;
            total += x;
        }
        uint32_t run = (uint32_t)carry + before + inc - own;  // n < 2^32
        uint32_t ex[kStatsPer];
#pragma unroll
        for (int j = 0; j < kStatsPer; ++j) {
            ex[j] = run;
            s_e[tid * kStatsPer + j] = run;
            run += v[j];
        }
        if (base + kStatsPer <= npieces + 1) {
            uint4 *e4 = reinterpret_cast<uint4 *>(a.E + base);
#pragma unroll
            for (int q = 0; q < kStatsPer / 4; ++q)
                e4[q] = make_uint4(ex[4 * q], ex[4 * q + 1], ex[4 * q + 2], ex[4 * q + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < kStatsPer; ++j)
                if (base + j <= npieces) a.E[base + j] = ex[j];
        }
        __syncthreads();
        const uint64_t c1 = min(c0 + kStatsRound, npieces + 1);  // this round: indices [c0, c1)
        if ((uint32_t)tid <= P) {
            const uint64_t g = min((s_cl[tid] >> a.tile_shift) + (uint64_t)tid, npieces);
            if (g >= c0 && g < c1) s_zb[tid] = s_e[g - c0];
        }
        carry += total;
        __syncthreads();
    }
    if (lvl0) {
        bad = __syncthreads_or(bad);
        if (tid == 0) *a.status = bad ? kStatusSymbol : 0u;
    }

    // 3. Node zeros and the node table.
    if ((uint32_t)tid < P) {
        const uint64_t zb = s_zb[tid], z = s_zb[tid + 1] - zb;
        NZ[tid] = z;
        a.D[2 * tid] = s_cl[tid] - zb;
        a.D[2 * tid + 1] = zb + z;
    }

    // 4. The last level: C[c] = starts of the level-L "nodes" (single symbols).
    if (l + 1 == a.L) {
        for (uint64_t c = tid; c <= a.sigma; c += kStatsThreads) {
            const uint64_t q = c >> 1;
            a.C[c] = q >= P ? a.n : s_cl[q] + ((c & 1) ? s_zb[q + 1] - s_zb[q] : 0ull);
        }
    }
}

}  // namespace wt
