// Level pass for 16-bit symbols in and out (n < 2^32): the byte pass's
// scheme at two bytes per symbol.  A tile is 4 rows of 2048 symbols; thread
// t owns symbols [8t, 8t+8) of every row as one 16-byte load.
//   bits:    bit k of the eight halfwords by shift-and-or, an 8-bit mask per
//            row; the LDS array of masks read as 64-bit words is the tile's
//            slice of B_l;
//   scan:    two rows per 32-bit value, one wave scan each;
//   split:   both cursors of a lane in one word (16 times the level bit
//            selects the half), one 2-byte LDS write per symbol; positions
//            past a short tile read as 0xFFFF, ones that land on unread slots;
//   scatter: eight slots per lane; a run (same node, same bit) leaves as one
//            unaligned 16-byte store.  Node tables of up to kD16 entries are
//            kept in LDS, larger ones read from global memory per chunk.
#pragma once

#include "wt_kernels.hpp"

namespace wt {

constexpr int kD16 = 1024;

struct LdsLevelU16 {
    static constexpr int kTile = 8192, kRows = 4, kRowSyms = 2048;
    __align__(16) uint16_t stage[kTile];
    __align__(16) uint8_t m8[kTile / 8];  // 128 words of B_l
    uint32_t wz[kRows][kWaves];
    uint32_t zpre[kTile / 64];  // zeros of the tile before each word
    uint32_t D[kD16];
    CountTable ct;
};

// Bit k of the two halfwords of x at bits 0 and 1.
__device__ __forceinline__ uint32_t bits2_of(uint32_t x, uint32_t k) {
    const uint32_t y = (x >> k) & 0x00010001u;
    return (y | (y >> 15)) & 3u;
}

template <bool SCATTER, bool DIRS>
__device__ __forceinline__ void level_tile_u16(const LevelArgs &a, uint32_t tile, LdsLevelU16 &s) {
    constexpr int kTile = LdsLevelU16::kTile, kRows = LdsLevelU16::kRows, kRowSyms = LdsLevelU16::kRowSyms;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t t0 = tile * (uint32_t)kTile;
    const uint32_t len = (uint32_t)min((uint64_t)kTile, a.n - t0);
    const uint32_t k = a.k;
    const uint32_t Z0 = (uint32_t)a.tile_prefix[tile];

    const uint16_t *in = reinterpret_cast<const uint16_t *>(a.in) + t0;
    uint4 d[kRows];
    uint32_t m[kRows], z[kRows];
    if (len == (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) d[r] = *reinterpret_cast<const uint4 *>(in + r * kRowSyms + 8 * tid);
    } else {
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const uint32_t p = (uint32_t)(r * kRowSyms + 8 * tid);
            if (p + 8 <= len) {
                d[r] = *reinterpret_cast<const uint4 *>(in + p);
            } else {
                const uint32_t nv = clamp_count(len, p, 8u);
                uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    w[j >> 1] |= ((uint32_t)j < nv ? (uint32_t)in[p + j] : 0xFFFFu) << (16 * (j & 1));
                d[r] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    const bool d_lds = SCATTER && a.nD <= (uint64_t)kD16;
    if (SCATTER) {
        if (d_lds)
            for (int i = tid; i < (int)a.nD; i += kBlock) s.D[i] = (uint32_t)a.D[i];
        count_init(s.ct, tid);
    }
    if (*a.status) return;
    if (a.fused_l0 && a.level >= *a.fused_l0) return;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowSyms + 8 * tid);
        const uint32_t nv = clamp_count(len, p, 8u);
        const uint32_t mm = bits2_of(d[r].x, k) | (bits2_of(d[r].y, k) << 2) | (bits2_of(d[r].z, k) << 4) |
                            (bits2_of(d[r].w, k) << 6);
        m[r] = mm & ((1u << nv) - 1u);
        z[r] = nv - (uint32_t)__popc(m[r]);
        s.m8[r * kBlock + tid] = (uint8_t)m[r];
    }

    const uint32_t v01 = z[0] | (z[1] << 16), v23 = z[2] | (z[3] << 16);
    const uint32_t i01 = wave_incl_scan_u32(v01, lane), i23 = wave_incl_scan_u32(v23, lane);
    if (lane == kWave - 1) {
        s.wz[0][wave] = i01 & 0xFFFFu;
        s.wz[1][wave] = i01 >> 16;
        s.wz[2][wave] = i23 & 0xFFFFu;
        s.wz[3][wave] = i23 >> 16;
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
            const uint32_t x = s.wz[r][w];
            before += w < wave ? x : 0u;
            tot += x;
        }
        zl[r] = acc + before + we[r];
        acc += tot;
    }
    const uint32_t Zt = acc;
    if ((tid & 7) == 0)
#pragma unroll
        for (int r = 0; r < kRows; ++r) s.zpre[r * (kBlock / 8) + tid / 8] = zl[r];
    __syncthreads();

    // Bit words of the tile (word w = m8[8w .. 8w + 7]).
    const uint64_t *s_w64 = reinterpret_cast<const uint64_t *>(s.m8);
    if (tid < kTile / 64 && (uint32_t)tid * 64u < len) a.bits[(t0 >> 6) + tid] = s_w64[tid];

    // Directory entries: waves 0 and 1 cover words 64w .. 64w+63 (two rows).
    if (DIRS && wave < 2) {
        const uint32_t wbase = (uint32_t)wave * 4096u;
        if (wbase < len) {
            const uint32_t zb = s.zpre[wave * kWave];
            const uint32_t ze = wave == 0 ? s.zpre[kWave] : Zt;
            const uint64_t wd[1] = {s_w64[wave * kWave + lane]};
            const uint32_t zp[1] = {s.zpre[wave * kWave + lane] - zb};
            emit_directories<1>(wd, zp, (uint64_t)Z0 + zb, (uint64_t)t0 + wbase, clamp_count(len, wbase, 4096u),
                                ze - zb, a.n, a.rank, a.sel1, a.sel0, lane);
        }
    }
    if (!SCATTER) return;

#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t e0 = (uint32_t)(r * kRowSyms + 8 * tid);
        uint32_t A = zl[r] | ((Zt + e0 - zl[r]) << 16);
        const uint32_t dw[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // Bits 4 and 20 of T are bit k of the two halfwords (a rotation right by k-4 mod 32).
            const uint32_t T = __builtin_amdgcn_alignbit(dw[j], dw[j], (k + 28u) & 31u) & 0x00100010u;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const uint32_t sh = (T >> (16 * i)) & 31u;
                s.stage[__builtin_amdgcn_ubfe(A, sh, 16u)] = (uint16_t)(dw[j] >> (16 * i));
                A += 1u << sh;
            }
        }
    }
    __syncthreads();

    const uint32_t O0 = t0 - Z0;
    const uint32_t kn = k - 1;
    const uint32_t Mn = 0x00010001u << kn;
    const uint32_t n8 = a.n > 7 ? (uint32_t)(a.n - 7) : 0u;  // dest < n8 <=> dest + 7 < n
    const uint32_t qmax = (uint32_t)a.nD - 1u;
    uint16_t *out = reinterpret_cast<uint16_t *>(a.out);
    auto dbase = [&](uint32_t q) -> uint32_t { return d_lds ? s.D[q] : (uint32_t)a.D[q]; };
    const uint4 *s_st128 = reinterpret_cast<const uint4 *>(s.stage);
    constexpr int kChunksPerWave = kTile / 8 / kWaves;
    LaneCount lc;
#pragma unroll
    for (int i = 0; i < kChunksPerWave / kWave; ++i) {
        const uint32_t j = (uint32_t)(wave * kChunksPerWave + i * kWave + lane), sl = 8u * j;
        uint32_t ftile = kNoTile, fcnt = 0;
        if (sl < len) {
            const uint4 v = s_st128[j];
            const uint32_t q0 = min(((v.x & 0xFFFFu) >> k) & a.qmask, qmax);
            const uint32_t q7 = min(((v.w >> 16) >> k) & a.qmask, qmax);
            if (sl + 7 < len && q0 == q7) {
                const uint32_t dest = dbase(q0) + ((q0 & 1u) ? O0 + sl - Zt : Z0 + sl);
                if (dest < n8) {
                    *reinterpret_cast<u128_unaligned *>(out + dest) = u128_unaligned{v.x, v.y, v.z, v.w};
                    const uint32_t nt = dest >> a.next_shift;
                    if (((dest + 7) >> a.next_shift) == nt) {
                        const uint32_t ones = (uint32_t)(__popc(v.x & Mn) + __popc(v.y & Mn) + __popc(v.z & Mn) +
                                                         __popc(v.w & Mn));
                        lc.step(nt, 8u - ones, ftile, fcnt);
                    } else {
                        for (uint32_t c = 0; c < 8; ++c) {
                            const uint32_t x = ((c < 2 ? v.x : c < 4 ? v.y : c < 6 ? v.z : v.w) >> (16 * (c & 1))) &
                                               0xFFFFu;
                            if (!((x >> kn) & 1u)) count_add(s.ct, a.next_cnt, (dest + c) >> a.next_shift, 1u);
                        }
                    }
                }
            } else {
                const uint32_t nc = clamp_count(len, sl, 8u);
                for (uint32_t c = 0; c < nc; ++c) {
                    const uint32_t x = ((c < 2 ? v.x : c < 4 ? v.y : c < 6 ? v.z : v.w) >> (16 * (c & 1))) & 0xFFFFu;
                    const uint32_t qc = min((x >> k) & a.qmask, qmax), sc = sl + c;
                    const uint32_t dest = dbase(qc) + ((qc & 1u) ? O0 + sc - Zt : Z0 + sc);
                    if (dest < a.n) {
                        out[dest] = (uint16_t)x;
                        if (!((x >> kn) & 1u)) count_add(s.ct, a.next_cnt, dest >> a.next_shift, 1u);
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

}  // namespace wt
