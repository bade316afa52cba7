// Multiary wavelet tree with d = 4, byte symbols: one pass per level.
//
// The paper's multiary tree stores on level j the 2-bit digit j (from the
// top) of every symbol, listed in the order of S sorted stably by its top j
// digits; level j+1's order is level j's with every node (a run of equal top
// j digits) sorted stably by digit j.  A level pass here reads S_j once and
// writes its entries, the digit directories and S_{j+1}:
//   entries   the two digit bits of sixteen bytes as 16-bit masks (the same
//             byte transpose as the binary pass), interleaved into 32 bits;
//   counts    G_v(i) = symbols of digit v in S_j[0, i): tile prefixes (from
//             the previous pass's count-ahead, or the histogram for j = 0)
//             plus a block scan per digit value;
//   S_{j+1}   symbol i of node q with digit v goes to E_j[4q+v] + G_v(i),
//             E_j[4q+v] = C[(4q+v) 4^(Lq-1-j)] - (digit-v symbols of the nodes
//             before q), a table from C; the tile is split 4 ways in LDS and
//             leaves in runs of one (node, digit).
#pragma once

#include "wt_pair.hpp"

namespace wt {

struct QuadArgs {
    const uint8_t *in;        // S_j, 16-byte aligned
    uint8_t *out;             // S_{j+1}
    uint32_t *entries;        // level j: 16 entries per 32-bit word, entry i at bits 2(i%16), 2(i%16)+1
    uint64_t nwords32;        // 2 * ceil(n/32) (whole 64-bit words)
    const uint32_t *E;        // E_j: 4^(j+1) entries
    uint32_t nkeys;           // 4^(j+1)
    const uint4 *pre;         // (G_0, G_1, G_2) before each tile of level j
    uint64_t *next_cnt;       // packed digit counts of level j+1 per tile (count-ahead)
    uint32_t next_shift;      // log2(positions per tile of the next level)
    const uint32_t *status;   // non-zero: input rejected, do nothing
    uint64_t *rank4;          // level j: [ceil(n/512)+1][4]
    uint64_t *sel4;           // level j: [4][cap]
    uint64_t cap;
    uint32_t n;               // < 2^32
    uint32_t kq;              // digit j = (x >> kq) & 3
};

struct LdsQuad {
    static constexpr int kTile = 16384, kRows = 4, kRowBytes = 4096;
    __align__(16) uint8_t buf[kTile];  // the tile split 4 ways by digit
    uint32_t wz[kRows][kWaves];
    uint32_t E[256];
    CountTableT<uint64_t> ct;
};

// The sixteen bits of m spread to the even bits of a 32-bit word.
__device__ __forceinline__ uint32_t spread16(uint32_t m) {
    m = (m | (m << 8)) & 0x00FF00FFu;
    m = (m | (m << 4)) & 0x0F0F0F0Fu;
    m = (m | (m << 2)) & 0x33333333u;
    m = (m | (m << 1)) & 0x55555555u;
    return m;
}

template <bool SCATTER>
__device__ __forceinline__ void quad_tile_u8(const QuadArgs &a, uint32_t tile, LdsQuad &s) {
    constexpr int kTile = LdsQuad::kTile, kRows = LdsQuad::kRows, kRowBytes = LdsQuad::kRowBytes;
    constexpr uint32_t S = WT_SELECT_SAMPLE;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t t0 = tile * (uint32_t)kTile;
    const uint32_t len = min((uint32_t)kTile, a.n - t0);
    const uint32_t kq = a.kq;
    const uint4 P = a.pre[tile];
    const uint32_t Gt[4] = {P.x, P.y, P.z, t0 - P.x - P.y - P.z};

    // Load (a whole tile's loads back to back), then the table.  Positions
    // past the end of a short tile read as 0xFF (see the split).
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
                    w[j >> 2] |= ((uint32_t)j < nv ? (uint32_t)in[p + j] : 0xFFu) << (8 * (j & 3));
                d[r] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    if (SCATTER) {
        for (int i = tid; i < (int)a.nkeys; i += kBlock) s.E[i] = a.E[i];
        count_init_t(s.ct, tid);
    }
    if (*a.status) return;  // grid-uniform: the input was rejected (nothing written yet)

    // Digit bit masks, counts and the interleaved entries of every chunk
    // (the mask of digit v is rebuilt from the two bit masks where needed).
    uint32_t mh[kRows], ml[kRows], w32[kRows];
    uint32_t c0[kRows], c1[kRows], c2[kRows];
    auto digit_mask = [&](int r, int v) -> uint32_t {
        const uint32_t nv = clamp_count(len, (uint32_t)(r * kRowBytes + 16 * tid), 16u);
        const uint32_t h = (v & 2) ? mh[r] : ~mh[r], l = (v & 1) ? ml[r] : ~ml[r];
        return h & l & ((1u << nv) - 1u);
    };
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid);
        const uint32_t nv = clamp_count(len, p, 16u);
        const uint32_t vm = (1u << nv) - 1u;
        mh[r] = mask16_bit(d[r], kq + 1u) & vm;
        ml[r] = mask16_bit(d[r], kq) & vm;
        c0[r] = (uint32_t)__popc(~mh[r] & ~ml[r] & vm);
        c1[r] = (uint32_t)__popc(~mh[r] & ml[r]);
        c2[r] = (uint32_t)__popc(mh[r] & ~ml[r]);
        w32[r] = spread16(ml[r]) | (spread16(mh[r]) << 1);
    }
    uint32_t l0[kRows], l1[kRows], l2[kRows];
    const uint32_t T0 = rows_scan(c0, l0, s.wz, lane, wave);
    const uint32_t T1 = rows_scan(c1, l1, s.wz, lane, wave);
    const uint32_t T2 = rows_scan(c2, l2, s.wz, lane, wave);

    // Entries, rank entries (a 512-entry block starts at every 32nd chunk)
    // and select samples of every digit value.
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid), pos = t0 + p;
        const uint32_t lv[4] = {l0[r], l1[r], l2[r], p - l0[r] - l1[r] - l2[r]};
        if ((uint64_t)(pos >> 4) < a.nwords32) a.entries[pos >> 4] = w32[r];
        if (p < len) {
            if ((pos & 511u) == 0) {
                uint64_t *re = a.rank4 + (uint64_t)(pos >> 9) * 4;
#pragma unroll
                for (int v = 0; v < 4; ++v) re[v] = (uint64_t)Gt[v] + lv[v];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t gm = digit_mask(r, v);
                const uint32_t o0 = Gt[v] + lv[v], cnt = (uint32_t)__popc(gm);
                const uint64_t tt = ((uint64_t)o0 + S - 1) / S * S;
                if (tt < (uint64_t)o0 + cnt && tt < a.n)  // an ordinal is below n
                    a.sel4[(uint64_t)v * a.cap + tt / S] = pos + select_in_word(gm, (uint32_t)(tt - o0));
            }
        }
    }
    if (!SCATTER) return;

    // Split 4 ways: digit v's region starts at off[v]; inside it, the tile's
    // order.  A lane's four cursors share one 64-bit word (16 bits each);
    // 16 times a byte's digit is the shift that reads its cursor and the one
    // that advances it.  The 0xFF bytes past the end of a short tile have
    // digit 3 and follow every valid byte, so position e >= len goes to slot
    // e: slots [len, kTile), which nothing reads.
    const uint32_t off[4] = {0u, T0, T0 + T1, T0 + T1 + T2};
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid);
        uint64_t A = (uint64_t)(off[0] + l0[r]) | ((uint64_t)(off[1] + l1[r]) << 16) |
                     ((uint64_t)(off[2] + l2[r]) << 32) | ((uint64_t)(off[3] + p - l0[r] - l1[r] - l2[r]) << 48);
        const uint32_t dw[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // Bits 8i+4, 8i+5 of T are the digit of byte i (a rotation right by kq-4 mod 32).
            const uint32_t T = __builtin_amdgcn_alignbit(dw[j], dw[j], (kq + 28u) & 31u) & 0x30303030u;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t sh = (T >> (8 * i)) & 0x30u;
                s.buf[(uint32_t)(A >> sh) & 0xFFFFu] = (uint8_t)(dw[j] >> (8 * i));
                A += 1ull << sh;
            }
        }
    }
    __syncthreads();

    // Scatter: slot sl of digit v's region is the symbol with
    // G_v = Gt[v] + (sl - off[v]); its destination is E[x >> kq] + that.
    uint32_t base4[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) base4[v] = Gt[v] - off[v];
    const uint32_t n16 = a.n > 15u ? a.n - 15u : 0u;
    const uint4 *b128 = reinterpret_cast<const uint4 *>(s.buf);
    // Wave w walks chunks [256w, 256w + 256) of the split tile, 64 at a time
    // (see the one-level pass: counts reach the table wave-wide).
    constexpr int kChunksPerWave = kTile / 16 / kWaves;
    LaneCountT<uint64_t> lc;
#pragma unroll
    for (int i = 0; i < kChunksPerWave / kWave; ++i) {
        const uint32_t j = (uint32_t)(wave * kChunksPerWave + i * kWave + lane), sl = 16u * j;
        uint32_t ftile = kNoTile;
        uint64_t fcnt = 0;
        if (sl < len) {
            const uint4 v = b128[j];
            const uint32_t k0 = (v.x & 0xFFu) >> kq, k15 = (v.w >> 24) >> kq;
            if (sl + 15u < len && k0 == k15) {
                const uint32_t dest = s.E[k0] + base4[k0 & 3u] + sl;
                if (dest < n16) {
                    *reinterpret_cast<u128_unaligned *>(a.out + dest) = u128_unaligned{v.x, v.y, v.z, v.w};
                    const uint32_t nt = dest >> a.next_shift;
                    if (((dest + 15u) >> a.next_shift) == nt) {
                        lc.step(nt, digit_inc16(v, kq - 2u), ftile, fcnt);
                    } else {
                        for (uint32_t c = 0; c < 16; ++c) {
                            const uint64_t t = digit_inc(byte_of(v, (int)c), kq - 2u);
                            if (t) count_add_t(s.ct, a.next_cnt, (dest + c) >> a.next_shift, t);
                        }
                    }
                }
            } else {
                const uint32_t nc = clamp_count(len, sl, 16u);
                for (uint32_t c = 0; c < nc; ++c) {
                    const uint32_t x = byte_of(v, (int)c), key = x >> kq;
                    const uint32_t dest = s.E[key] + base4[key & 3u] + sl + c;
                    if (dest < a.n) {
                        a.out[dest] = (uint8_t)x;
                        const uint64_t t = digit_inc(x, kq - 2u);
                        if (t) count_add_t(s.ct, a.next_cnt, dest >> a.next_shift, t);
                    }
                }
            }
        }
        count_add_wave_t<uint64_t>(s.ct, a.next_cnt, fcnt != 0, ftile, fcnt, lane);
    }
    lc.flush_wave(s.ct, a.next_cnt, lane);
    __syncthreads();
    count_flush_t(s.ct, a.next_cnt, tid);
}

}  // namespace wt
