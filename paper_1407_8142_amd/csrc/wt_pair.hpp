// Two levels per read of S (byte symbols).
//
// levelWT (Fig. 1 of "Parallel Wavelet Tree Construction") splits every
// node stably by one bit per level.  Two consecutive splits are one stable
// split by the two-bit digit d = (bit k, bit k-1): level l+2's sequence is
// level l's sequence stably sorted by (node, d), as the sortWT view of the
// levels shows (level l is S stably sorted by its top l bits).  So one pass
// over S_l can produce B_l, B_{l+1}, both levels' directories and S_{l+2}.
//
// With G_d(i) = symbols of digit d among positions [0, i) of S_l (over the
// whole level), a symbol at position i of node p goes to
//   S_{l+1}: D_l[2p+b] + (b ? i - Z(i) : Z(i))            Z = G_0 + G_1
//   S_{l+2}: E_l[4p+d] + G_d(i)
// with E_l[4p+d] = C[(4p+d) 2^(k-1)] - G_d(start of node p), a table from C
// alone (the count of digit d in node q < p is a difference of two C
// entries).  A tile needs the three prefixes G_0, G_1, G_2 at its start;
// they come, as for a single level, from counts that the previous pass
// accumulated per destination tile (three 16-bit fields, a tile holds at
// most 2^14 symbols), or from the histogram for level 0.
//
// Inside a tile:
//   A = the tile split stably by bit k (as a single level pass does); the
//       bits k-1 of A, in A order, are B_{l+1}'s bits of this tile's symbols:
//       the symbols of one (node p, bit b) group are consecutive in A and
//       land on consecutive positions of S_{l+1}, a constant shift apart;
//   B = A split stably by bit k-1 inside each half: the digit-ordered tile,
//       scattered to S_{l+2} in runs of one (node, digit).
// B_{l+1} words wholly inside one group are stored; a word shared with a
// neighbouring group (of this tile or another) is cleared and set over the
// group's bits only, by atomics on disjoint masks.  The last group of the
// level also clears the padding bits.  Level l+1's directory entries follow
// from its zero count at any position of a group, which is a table entry
// plus in-tile counts:
//   Z_{l+1}(pos) = E_l[4p+2b] - D_{l+1}[2(2p+b)] + G_{2b}(t0) - (b ? T_0 : 0)
//                  + (zeros of bit k-1 among A slots before pos - shift)
// (T_0 = digit-0 symbols of the tile).
#pragma once

#include <type_traits>

#include "wt_kernels.hpp"

namespace wt {

// Per-lane count-ahead with a count type of its own (uint32 zeros for a
// single next level, or three packed 16-bit digit counts for a next pair).
template <typename CNT>
struct CountTableT {
    uint32_t key[kCountSlots];
    CNT cnt[kCountSlots];
};

template <typename CNT>
__device__ __forceinline__ void count_init_t(CountTableT<CNT> &t, int tid) {
    if (tid < kCountSlots) {
        t.key[tid] = kNoTile;
        t.cnt[tid] = 0;
    }
}

template <typename CNT>
__device__ __forceinline__ void global_add(CNT *p, CNT v) {
    if constexpr (sizeof(CNT) == 8) atomicAdd((unsigned long long *)p, (unsigned long long)v);
    else atomicAdd(p, v);
}

template <typename CNT>
__device__ __forceinline__ void count_add_t(CountTableT<CNT> &t, CNT *next_cnt, uint32_t ntile, CNT c) {
    uint32_t slot = (ntile * 0x9E3779B9u) >> 26;
#pragma unroll 1
    for (int probe = 0; probe < 8; ++probe) {
        const uint32_t old = atomicCAS(&t.key[slot], kNoTile, ntile);
        if (old == kNoTile || old == ntile) {
            if constexpr (sizeof(CNT) == 8) atomicAdd((unsigned long long *)&t.cnt[slot], (unsigned long long)c);
            else atomicAdd(&t.cnt[slot], c);
            return;
        }
        slot = (slot + 1) & (kCountSlots - 1);
    }
    global_add(next_cnt + ntile, c);
}

template <typename CNT>
__device__ __forceinline__ void count_flush_t(CountTableT<CNT> &t, CNT *next_cnt, int tid) {
    if (tid < kCountSlots && t.key[tid] != kNoTile && t.cnt[tid]) global_add(next_cnt + t.key[tid], t.cnt[tid]);
}

// Sum over the 64 lanes of a wave of packed counts (all lanes active): the
// 16-bit fields of one tile's counts never carry, so the halves of a 64-bit
// word are summed as two 32-bit values.
template <typename CNT>
__device__ __forceinline__ CNT wave_sum_cnt(CNT v) {
    if constexpr (sizeof(CNT) == 8)
        return (uint64_t)wave_sum_u32((uint32_t)v) | ((uint64_t)wave_sum_u32((uint32_t)(v >> 32)) << 32);
    else
        return wave_sum_u32(v);
}

// count_add_wave for packed counts: one table update per distinct tile of
// the wave.  Called by all lanes of the wave.
template <typename CNT>
__device__ __forceinline__ void count_add_wave_t(CountTableT<CNT> &t, CNT *next_cnt, bool want, uint32_t tile,
                                                 CNT c, int lane) {
    uint64_t pend = __ballot(want);
    while (pend) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const uint32_t kt = (uint32_t)__builtin_amdgcn_readlane((int)tile, leader);
        const bool mine = want && tile == kt;
        const CNT tot = wave_sum_cnt<CNT>(mine ? c : (CNT)0);
        if (lane == leader) count_add_t(t, next_cnt, kt, tot);
        pend &= ~__ballot(mine);
    }
}

template <typename CNT>
struct LaneCountT {
    uint32_t tile = kNoTile;
    CNT cnt = 0;
    __device__ __forceinline__ void add(CountTableT<CNT> &t, CNT *next_cnt, uint32_t ntile, CNT c) {
        if (ntile != tile) {
            if (cnt) count_add_t(t, next_cnt, tile, cnt);
            tile = ntile;
            cnt = 0;
        }
        cnt += c;
    }
    // As add, but a finished tile's count is returned for a wave-wide hand-over.
    __device__ __forceinline__ void step(uint32_t ntile, CNT c, uint32_t &ftile, CNT &fcnt) {
        if (ntile != tile) {
            ftile = tile;
            fcnt = cnt;
            tile = ntile;
            cnt = 0;
        }
        cnt += c;
    }
    __device__ __forceinline__ void flush(CountTableT<CNT> &t, CNT *next_cnt) {
        if (cnt) count_add_t(t, next_cnt, tile, cnt);
        cnt = 0;
    }
    __device__ __forceinline__ void flush_wave(CountTableT<CNT> &t, CNT *next_cnt, int lane) {
        count_add_wave_t<CNT>(t, next_cnt, cnt != 0, tile, cnt, lane);
        cnt = 0;
    }
};

// digit_inc summed over the sixteen bytes of v (SWAR: one bit per byte lane).
__device__ __forceinline__ uint64_t digit_inc16(const uint4 &v, uint32_t lo) {
    const uint32_t M = 0x01010101u;
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    uint32_t hi = 0, lw = 0, both = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t h = (w[i] >> (lo + 1u)) & M, l = (w[i] >> lo) & M;
        hi += (uint32_t)__popc(h);
        lw += (uint32_t)__popc(l);
        both += (uint32_t)__popc(h & l);
    }
    const uint32_t c2 = hi - both, c1 = lw - both, c0 = 16u - hi - c1;
    return (uint64_t)c0 | ((uint64_t)c1 << 16) | ((uint64_t)c2 << 32);
}

// Zeros of bit `bit` over the sixteen bytes of v.
__device__ __forceinline__ uint32_t zeros16(const uint4 &v, uint32_t bit) {
    const uint32_t M = 0x01010101u << bit;
    return 16u - (uint32_t)(__popc(v.x & M) + __popc(v.y & M) + __popc(v.z & M) + __popc(v.w & M));
}

struct PairArgs {
    const uint8_t *in;        // S_l, 16-byte aligned
    uint8_t *out;             // S_{l+2}
    uint64_t *bits0, *bits1;  // B_l, B_{l+1}
    const uint64_t *C;        // C[0..sigma]
    uint64_t sigma;
    const uint64_t *D0;       // D_l: 2^(l+1) entries
    const uint64_t *D1;       // D_{l+1}: 2^(l+2) entries
    const uint32_t *E;        // E_l: 2^(l+2) entries
    const uint4 *pre;         // (G_0, G_1, G_2) before each tile of level l
    void *next_cnt;           // count-ahead: uint64 digit counts (next pass a pair) or uint32 zeros
    uint32_t next_shift;      // log2(positions per tile of the next pass)
    const uint32_t *status;   // non-zero: input rejected, do nothing
    uint64_t *rank0, *sel10, *sel00;  // directory rows of level l
    uint64_t *rank1, *sel11, *sel01;  // directory rows of level l+1
    uint32_t n;               // < 2^32
    uint32_t k;               // bit of level l: L-1-l >= 1
    uint32_t level;           // l (<= 6: byte symbols)
};

struct LdsPair {
    static constexpr int kTile = 16384, kRows = 4, kRowBytes = 4096, kWords = kTile / 64;
    __align__(16) uint8_t buf[kTile];        // A, then B in place
    __align__(16) uint16_t m16[kTile / 16];  // bit k in position order: B_l's words
    __align__(16) uint16_t c16[kTile / 16];  // bit k-1 in A order
    uint32_t wz[kRows][kWaves];              // scan partials
    uint32_t zpre[kWords];                   // zeros of bit k before each position word
    uint32_t cpre[kWords];                   // zeros of bit k-1 before each A word
    uint32_t D0[128];
    uint32_t D1[256];
    uint32_t E[256];
    uint32_t NS[65];                         // node starts of level l
    uint32_t pf, pl;                         // first and last node of the tile
    union {
        CountTableT<uint64_t> c64;
        CountTableT<uint32_t> c32;
    } ct;
};

// Exclusive prefix, in position order (rows outer, threads inner), of four
// per-thread counts of at most 16; returns the block total.  Ends with a
// barrier after which s.wz may be reused.
__device__ __forceinline__ uint32_t rows_scan(const uint32_t (&z)[4], uint32_t (&zl)[4], uint32_t (&wz)[4][kWaves],
                                              int lane, int wave) {
    const uint32_t v01 = z[0] | (z[1] << 16), v23 = z[2] | (z[3] << 16);
    const uint32_t i01 = wave_incl_scan_u32(v01, lane), i23 = wave_incl_scan_u32(v23, lane);
    if (lane == kWave - 1) {
        wz[0][wave] = i01 & 0xFFFFu;
        wz[1][wave] = i01 >> 16;
        wz[2][wave] = i23 & 0xFFFFu;
        wz[3][wave] = i23 >> 16;
    }
    __syncthreads();
    const uint32_t e01 = i01 - v01, e23 = i23 - v23;
    const uint32_t we[4] = {e01 & 0xFFFFu, e01 >> 16, e23 & 0xFFFFu, e23 >> 16};
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t x = wz[r][w];
            before += w < wave ? x : 0u;
            tot += x;
        }
        zl[r] = acc + before + we[r];
        acc += tot;
    }
    __syncthreads();
    return acc;
}

// `nbits` (1..64) bits of a slot-ordered bit array starting at slot o.
__device__ __forceinline__ uint64_t bits_at(const uint64_t *w64, uint32_t o, uint32_t nbits, uint32_t nwords) {
    const uint32_t i = o >> 6, sh = o & 63u;
    uint64_t v = w64[i] >> sh;
    if (sh && i + 1 < nwords) v |= w64[i + 1] << (64u - sh);
    return nbits >= 64u ? v : (v & ((1ull << nbits) - 1ull));
}

template <bool SCATTER, bool NEXT_PAIR, bool DIRS>
__device__ __forceinline__ void pair_tile_u8(const PairArgs &a, uint32_t tile, LdsPair &s) {
    constexpr int kTile = LdsPair::kTile, kRows = LdsPair::kRows, kRowBytes = LdsPair::kRowBytes;
    constexpr uint32_t S = WT_SELECT_SAMPLE;
    using CNT = typename std::conditional<NEXT_PAIR, uint64_t, uint32_t>::type;
    CountTableT<CNT> &ct = *reinterpret_cast<CountTableT<CNT> *>(&s.ct);

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t t0 = tile * (uint32_t)kTile;
    const uint32_t len = min((uint32_t)kTile, a.n - t0);
    const uint32_t k = a.k, l = a.level;
    const uint4 P = a.pre[tile];
    const uint32_t G0t = P.x, G1t = P.y, G2t = P.z, G3t = t0 - P.x - P.y - P.z;
    const uint32_t Z0 = G0t + G1t, O0 = t0 - Z0;
    const uint32_t nnodes = 1u << l;

    // Load: thread t, row r holds positions r*4096 + 16t .. +15 (a whole
    // tile's loads back to back, then the tables).
    const uint8_t *in = a.in + t0;
    uint4 d[kRows];
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
                    if ((uint32_t)j < nv) w[j >> 2] |= (uint32_t)in[p + j] << (8 * (j & 3));
                d[r] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    for (int i = tid; i < (int)(2u * nnodes); i += kBlock) s.D0[i] = (uint32_t)a.D0[i];
    if (DIRS)
        for (int i = tid; i < (int)(4u * nnodes); i += kBlock) s.D1[i] = (uint32_t)a.D1[i];
    for (int i = tid; i < (int)(4u * nnodes); i += kBlock) s.E[i] = a.E[i];
    for (int i = tid; i <= (int)nnodes; i += kBlock) {
        const uint64_t c = (uint64_t)i << (k + 1u);
        s.NS[i] = (uint32_t)a.C[c < a.sigma ? c : a.sigma];
    }
    if (SCATTER) count_init_t(ct, tid);
    if (*a.status) return;  // grid-uniform: the input was rejected (nothing written yet)

    uint32_t m[kRows], z[kRows], zl[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid);
        const uint32_t nv = clamp_count(len, p, 16u);
        m[r] = mask16_bit(d[r], k) & ((1u << nv) - 1u);
        z[r] = nv - (uint32_t)__popc(m[r]);
        s.m16[r * kBlock + tid] = (uint16_t)m[r];
        if (p == 0) s.pf = byte_of(d[r], 0) >> (k + 1u);
        if (nv > 0 && p + nv == len) s.pl = byte_of(d[r], (int)nv - 1) >> (k + 1u);
    }
    const uint32_t Zt = rows_scan(z, zl, s.wz, lane, wave);
    if ((tid & 3) == 0)
#pragma unroll
        for (int r = 0; r < kRows; ++r) s.zpre[r * (kBlock / 4) + tid / 4] = zl[r];

    // Stable split by bit k into A (zeros at [0, Zt), ones at [Zt, len)).
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t e0 = (uint32_t)(r * kRowBytes + 16 * tid);
        const uint32_t nv = clamp_count(len, e0, 16u);
        uint32_t zc = zl[r], oc = Zt + e0 - zl[r];
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const uint32_t bit = (m[r] >> b) & 1u;
            if ((uint32_t)b < nv) s.buf[bit ? oc : zc] = (uint8_t)byte_of(d[r], b);
            zc += bit ^ 1u;
            oc += bit;
        }
    }
    __syncthreads();

    // B_l's words and level l's directory entries (wave w covers row w).
    const uint64_t *m64 = reinterpret_cast<const uint64_t *>(s.m16);
    if ((uint32_t)tid * 64u < len) a.bits0[(t0 >> 6) + tid] = m64[tid];
    if (DIRS) {
        const uint32_t wbase = (uint32_t)wave * kRowBytes;
        if (wbase < len) {
            const uint32_t zb = s.zpre[wave * kWave];
            const uint32_t ze = wave + 1 < kWaves && (uint32_t)(wave + 1) * kRowBytes < len ? s.zpre[(wave + 1) * kWave]
                                                                                            : Zt;
            const uint64_t wd[1] = {m64[tid]};
            const uint32_t zp[1] = {s.zpre[tid] - zb};
            emit_directories<1>(wd, zp, (uint64_t)Z0 + zb, (uint64_t)t0 + wbase,
                                clamp_count(len, wbase, (uint32_t)kRowBytes), ze - zb, a.n, a.rank0, a.sel10,
                                a.sel00, lane);
        }
    }

    // A in registers; bit k-1 in A order and its zero-count scan.
    uint4 dA[kRows];
    uint32_t mc[kRows], zc[kRows], zcl[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t e0 = (uint32_t)(r * kRowBytes + 16 * tid);
        const uint32_t nv = clamp_count(len, e0, 16u);
        dA[r] = *reinterpret_cast<const uint4 *>(s.buf + e0);
        mc[r] = mask16_bit(dA[r], k - 1u) & ((1u << nv) - 1u);
        zc[r] = nv - (uint32_t)__popc(mc[r]);
        s.c16[r * kBlock + tid] = (uint16_t)mc[r];
    }
    const uint32_t ZCt = rows_scan(zc, zcl, s.wz, lane, wave);  // its barriers also retire every read of A
    if ((tid & 3) == 0)
#pragma unroll
        for (int r = 0; r < kRows; ++r) s.cpre[r * (kBlock / 4) + tid / 4] = zcl[r];
    __syncthreads();

    const uint64_t *c64 = reinterpret_cast<const uint64_t *>(s.c16);
    // Zeros of bit k among tile positions [0, x), of bit k-1 among A slots [0, x); x <= len.
    auto zk_at = [&](uint32_t x) -> uint32_t {
        if (x >= len) return Zt;
        const uint32_t w = x >> 6, b = x & 63u;
        return s.zpre[w] + b - (uint32_t)__popcll(m64[w] & ((1ull << b) - 1ull));
    };
    auto zc_at = [&](uint32_t x) -> uint32_t {
        if (x >= len) return ZCt;
        const uint32_t w = x >> 6, b = x & 63u;
        return s.cpre[w] + b - (uint32_t)__popcll(c64[w] & ((1ull << b) - 1ull));
    };
    const uint32_t T0 = zc_at(Zt);  // digit-0 symbols of the tile

    if (SCATTER) {
        // B: A split by bit k-1 inside each half; digit regions start at
        // 0, T0, Zt, Zt + (ZCt - T0).
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const uint32_t e0 = (uint32_t)(r * kRowBytes + 16 * tid);
            const uint32_t nv = clamp_count(len, e0, 16u);
            uint32_t zcs = zcl[r];  // zeros of bit k-1 among A slots before the current one
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                const uint32_t sl = e0 + (uint32_t)b, c = (mc[r] >> b) & 1u;
                const bool h1 = sl >= Zt;
                const uint32_t dest = c ? sl - zcs + (h1 ? ZCt : T0) : zcs + (h1 ? Zt - T0 : 0u);
                if ((uint32_t)b < nv) s.buf[dest] = (uint8_t)byte_of(dA[r], b);
                zcs += c ^ 1u;
            }
        }
    }

    // B_{l+1}: the groups (node p, bit b) of the tile, each a run of A slots
    // [sa, sb) at positions sa + delta of S_{l+1}.
    const uint32_t pf = s.pf, pl = s.pl;
#pragma unroll 1
    for (uint32_t p = pf; p <= pl; ++p) {
        const uint32_t ns = s.NS[p], ne = s.NS[p + 1];
        const uint32_t ls = ns > t0 ? ns - t0 : 0u;
        const uint32_t le = ne - t0 < len ? ne - t0 : len;  // ne > t0 for p <= pl
        if (ls >= le) continue;
        const uint32_t zs = zk_at(ls), ze = zk_at(le);
#pragma unroll 1
        for (uint32_t b = 0; b < 2; ++b) {
            const uint32_t sa = b ? Zt + (ls - zs) : zs;
            const uint32_t sb = b ? Zt + (le - ze) : ze;
            if (sa == sb) continue;
            const uint32_t delta = b ? s.D0[2 * p + 1] + O0 - Zt : s.D0[2 * p] + Z0;
            const uint32_t Pg = sa + delta, cnt = sb - sa;
            const uint32_t zb1 = DIRS ? s.E[4 * p + 2 * b] - s.D1[2 * (2 * p + b)] + (b ? G2t : G0t) - (b ? T0 : 0u)
                                      : 0u;
            const uint32_t w0 = Pg >> 6, w1 = (Pg + cnt - 1u) >> 6;
            for (uint32_t w = w0 + (uint32_t)tid; w <= w1; w += kBlock) {
                const uint32_t lo_pos = max(Pg, w * 64u), hi_pos = min(Pg + cnt, w * 64u + 64u);
                const uint32_t lo = lo_pos - w * 64u, nb = hi_pos - lo_pos;
                const uint32_t o = lo_pos - delta;  // A slot of lo_pos
                const uint64_t v = bits_at(c64, o, nb, (uint32_t)LdsPair::kWords);
                const uint64_t vm = nb >= 64u ? ~0ull : ((1ull << nb) - 1ull);
                uint64_t mask = vm << lo;
                if (hi_pos == a.n && hi_pos - w * 64u < 64u) mask |= ~0ull << (hi_pos - w * 64u);  // padding
                const uint64_t val = v << lo;
                if (mask == ~0ull) {
                    a.bits1[w] = val;
                } else {
                    atomicAnd((unsigned long long *)(a.bits1 + w), (unsigned long long)~mask);
                    if (val) atomicOr((unsigned long long *)(a.bits1 + w), (unsigned long long)val);
                }
                if (DIRS) {
                    const uint32_t Z1 = zb1 + zc_at(o), O1 = lo_pos - Z1;
                    if (lo == 0 && (w & 7u) == 0) a.rank1[w >> 3] = O1;
                    const uint32_t ones = (uint32_t)__popcll(v), zeros = nb - ones;
                    const uint64_t to = ((uint64_t)O1 + S - 1) / S * S, tz = ((uint64_t)Z1 + S - 1) / S * S;
                    if (to < (uint64_t)O1 + ones) a.sel11[to / S] = lo_pos + select_in_word(v, (uint32_t)(to - O1));
                    if (tz < (uint64_t)Z1 + zeros)
                        a.sel01[tz / S] = lo_pos + select_in_word(~v & vm, (uint32_t)(tz - Z1));
                }
            }
        }
    }
    if (!SCATTER) return;
    __syncthreads();  // B complete

    // Scatter B to S_{l+2}: digit d's region is in position order, so slot
    // sl of it is the symbol with G_d = Gt[d] + (sl - region start).
    const uint32_t kd = k - 1u;
    uint32_t base4[4];
    base4[0] = G0t;
    base4[1] = G1t - T0;
    base4[2] = G2t - Zt;
    base4[3] = G3t - (Zt + ZCt - T0);
    CNT *next = reinterpret_cast<CNT *>(a.next_cnt);
    const uint32_t nlo = NEXT_PAIR ? k - 3u : 0u;  // next pass's low digit bit (or its single bit - 0)
    auto tally16 = [&](const uint4 &v) -> CNT {
        if constexpr (NEXT_PAIR) return digit_inc16(v, nlo);
        else return zeros16(v, k - 2u);
    };
    auto tally1 = [&](uint32_t x) -> CNT {
        if constexpr (NEXT_PAIR) return digit_inc(x, nlo);
        else return ((x >> (k - 2u)) & 1u) ^ 1u;
    };
    const uint32_t n16 = a.n > 15u ? a.n - 15u : 0u;
    const uint4 *b128 = reinterpret_cast<const uint4 *>(s.buf);
    // Wave w walks chunks [256w, 256w + 256) of the split tile, 64 at a time
    // (a lane's chunks mostly share a destination tile; counts reach the
    // table wave-wide, as in the one-level pass).
    constexpr int kChunksPerWave = kTile / 16 / kWaves;
    LaneCountT<CNT> lc;
#pragma unroll
    for (int i = 0; i < kChunksPerWave / kWave; ++i) {
        const uint32_t j = (uint32_t)(wave * kChunksPerWave + i * kWave + lane), sl = 16u * j;
        uint32_t ftile = kNoTile;
        CNT fcnt = 0;
        if (sl < len) {
            const uint4 v = b128[j];
            const uint32_t q0 = (v.x & 0xFFu) >> kd, q15 = (v.w >> 24) >> kd;
            if (sl + 15u < len && q0 == q15) {
                const uint32_t dest = s.E[q0] + base4[q0 & 3u] + sl;
                if (dest < n16) {
                    *reinterpret_cast<u128_unaligned *>(a.out + dest) = u128_unaligned{v.x, v.y, v.z, v.w};
                    const uint32_t nt = dest >> a.next_shift;
                    if (((dest + 15u) >> a.next_shift) == nt) {
                        lc.step(nt, tally16(v), ftile, fcnt);
                    } else {
                        for (uint32_t c = 0; c < 16; ++c) {
                            const CNT t = tally1(byte_of(v, (int)c));
                            if (t) count_add_t(ct, next, (dest + c) >> a.next_shift, t);
                        }
                    }
                }
            } else {
                const uint32_t nc = clamp_count(len, sl, 16u);
                for (uint32_t c = 0; c < nc; ++c) {
                    const uint32_t x = byte_of(v, (int)c), q = x >> kd;
                    const uint32_t dest = s.E[q] + base4[q & 3u] + sl + c;
                    if (dest < a.n) {
                        a.out[dest] = (uint8_t)x;
                        const CNT t = tally1(x);
                        if (t) count_add_t(ct, next, dest >> a.next_shift, t);
                    }
                }
            }
        }
        count_add_wave_t<CNT>(ct, next, fcnt != 0, ftile, fcnt, lane);
    }
    lc.flush_wave(ct, next, lane);
    __syncthreads();
    count_flush_t(ct, next, tid);
}

}  // namespace wt
