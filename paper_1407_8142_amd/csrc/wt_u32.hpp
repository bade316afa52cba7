// Level pass for 32-bit symbols in and out (n < 2^32): the byte pass's
// scheme at four bytes per symbol.  A tile is 4 rows of 1024 symbols; thread
// t owns symbols [4t, 4t+4) of every row as one 16-byte load.
//   bits:    a 4-bit mask per row; the masks of lanes 2i and 2i+1 make one
//            byte, and the LDS array of those bytes read as 64-bit words is
//            the tile's slice of B_l;
//   scan:    two rows per 32-bit value, one wave scan each;
//   split:   both cursors of a lane in one word (16 times the level bit
//            selects the half), one 4-byte LDS write per symbol; positions
//            past a short tile read as 0xFFFFFFFF, ones that land on unread
//            slots;
//   scatter: four slots per lane; a run (same node, same bit) leaves as one
//            store (16 bytes, or 8 / 4 when the next level is 16 / 8 bits
//            wide: a 32-bit input whose alphabet fits fewer bits).  Node
//            tables of up to kD32 entries are kept in LDS, larger ones read
//            from global memory per chunk.
#pragma once

#include "wt_kernels.hpp"

namespace wt {

constexpr int kD32 = 1024;

struct LdsLevelU32 {
    static constexpr int kTile = 4096, kRows = 4, kRowSyms = 1024;
    __align__(16) uint32_t stage[kTile];
    __align__(16) uint8_t m8[kTile / 8];  // 64 words of B_l
    uint32_t wz[kRows][kWaves];
    uint32_t zpre[kTile / 64];  // zeros of the tile before each word
    uint32_t D[kD32];
    CountTable ct;
};

template <typename TOUT, bool SCATTER, bool DIRS>
__device__ __forceinline__ void level_tile_u32(const LevelArgs &a, uint32_t tile, LdsLevelU32 &s) {
    constexpr int kTile = LdsLevelU32::kTile, kRows = LdsLevelU32::kRows, kRowSyms = LdsLevelU32::kRowSyms;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t t0 = tile * (uint32_t)kTile;
    const uint32_t len = (uint32_t)min((uint64_t)kTile, a.n - t0);
    const uint32_t k = a.k;
    const uint32_t Z0 = (uint32_t)a.tile_prefix[tile];

    const uint32_t *in = reinterpret_cast<const uint32_t *>(a.in) + t0;
    uint4 d[kRows];
    uint32_t m[kRows], z[kRows];
    if (len == (uint32_t)kTile) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) d[r] = *reinterpret_cast<const uint4 *>(in + r * kRowSyms + 4 * tid);
    } else {
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const uint32_t p = (uint32_t)(r * kRowSyms + 4 * tid);
            if (p + 4 <= len) {
                d[r] = *reinterpret_cast<const uint4 *>(in + p);
            } else {
                const uint32_t nv = clamp_count(len, p, 4u);
                uint32_t w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) w[j] = (uint32_t)j < nv ? in[p + j] : 0xFFFFFFFFu;
                d[r] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    const bool d_lds = SCATTER && a.nD <= (uint64_t)kD32;
    if (SCATTER) {
        if (d_lds)
            for (int i = tid; i < (int)a.nD; i += kBlock) s.D[i] = (uint32_t)a.D[i];
        count_init(s.ct, tid);
    }
    if (*a.status) return;
    if (a.fused_l0 && a.level >= *a.fused_l0) return;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowSyms + 4 * tid);
        const uint32_t nv = clamp_count(len, p, 4u);
        const uint32_t mm = ((d[r].x >> k) & 1u) | (((d[r].y >> k) & 1u) << 1) | (((d[r].z >> k) & 1u) << 2) |
                            (((d[r].w >> k) & 1u) << 3);
        m[r] = mm & ((1u << nv) - 1u);
        z[r] = nv - (uint32_t)__popc(m[r]);
        const uint32_t pair = m[r] | ((uint32_t)__shfl_xor((int)m[r], 1, kWave) << 4);  // lanes 2i, 2i+1
        if ((tid & 1) == 0) s.m8[r * (kBlock / 2) + tid / 2] = (uint8_t)pair;
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
    if ((tid & 15) == 0)
#pragma unroll
        for (int r = 0; r < kRows; ++r) s.zpre[r * (kBlock / 16) + tid / 16] = zl[r];
    __syncthreads();

    // Bit words of the tile (word w = m8[8w .. 8w + 7]).
    const uint64_t *s_w64 = reinterpret_cast<const uint64_t *>(s.m8);
    if (tid < kTile / 64 && (uint32_t)tid * 64u < len) a.bits[(t0 >> 6) + tid] = s_w64[tid];

    // Directory entries: wave 0 covers the tile's 64 words.
    if (DIRS && wave == 0) {
        const uint64_t wd[1] = {s_w64[lane]};
        const uint32_t zp[1] = {s.zpre[lane]};
        emit_directories<1>(wd, zp, (uint64_t)Z0, (uint64_t)t0, len, Zt, a.n, a.rank, a.sel1, a.sel0, lane);
    }
    if (!SCATTER) return;

#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t e0 = (uint32_t)(r * kRowSyms + 4 * tid);
        uint32_t A = zl[r] | ((Zt + e0 - zl[r]) << 16);
        const uint32_t dw[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // Bit 4 of the rotation right by k-4 mod 32 is bit k.
            const uint32_t sh = __builtin_amdgcn_alignbit(dw[j], dw[j], (k + 28u) & 31u) & 16u;
            s.stage[__builtin_amdgcn_ubfe(A, sh, 16u)] = dw[j];
            A += 1u << sh;
        }
    }
    __syncthreads();

    const uint32_t O0 = t0 - Z0;
    const uint32_t kn = k - 1;
    const uint32_t n4 = a.n > 3 ? (uint32_t)(a.n - 3) : 0u;  // dest < n4 <=> dest + 3 < n
    const uint32_t qmax = (uint32_t)a.nD - 1u;
    TOUT *out = reinterpret_cast<TOUT *>(a.out);
    auto dbase = [&](uint32_t q) -> uint32_t { return d_lds ? s.D[q] : (uint32_t)a.D[q]; };
    const uint4 *s_st128 = reinterpret_cast<const uint4 *>(s.stage);
    constexpr int kChunksPerWave = kTile / 4 / kWaves;
    LaneCount lc;
#pragma unroll
    for (int i = 0; i < kChunksPerWave / kWave; ++i) {
        const uint32_t j = (uint32_t)(wave * kChunksPerWave + i * kWave + lane), sl = 4u * j;
        uint32_t ftile = kNoTile, fcnt = 0;
        if (sl < len) {
            const uint4 v = s_st128[j];
            const uint32_t q0 = min((v.x >> k) & a.qmask, qmax);
            const uint32_t q3 = min((v.w >> k) & a.qmask, qmax);
            if (sl + 3 < len && q0 == q3) {
                const uint32_t dest = dbase(q0) + ((q0 & 1u) ? O0 + sl - Zt : Z0 + sl);
                if (dest < n4) {
                    if constexpr (sizeof(TOUT) == 4) {
                        *reinterpret_cast<u128_unaligned *>(out + dest) = u128_unaligned{v.x, v.y, v.z, v.w};
                    } else if constexpr (sizeof(TOUT) == 2) {
                        typedef uint32_t u64_unaligned __attribute__((ext_vector_type(2), aligned(2)));
                        *reinterpret_cast<u64_unaligned *>(out + dest) =
                            u64_unaligned{(v.x & 0xFFFFu) | (v.y << 16), (v.z & 0xFFFFu) | (v.w << 16)};
                    } else {
                        typedef uint32_t u32_unaligned __attribute__((aligned(1)));
                        *reinterpret_cast<u32_unaligned *>(out + dest) =
                            (v.x & 0xFFu) | ((v.y & 0xFFu) << 8) | ((v.z & 0xFFu) << 16) | (v.w << 24);
                    }
                    const uint32_t nt = dest >> a.next_shift;
                    const uint32_t ones = ((v.x >> kn) & 1u) + ((v.y >> kn) & 1u) + ((v.z >> kn) & 1u) +
                                          ((v.w >> kn) & 1u);
                    if (((dest + 3) >> a.next_shift) == nt) {
                        lc.step(nt, 4u - ones, ftile, fcnt);
                    } else {
                        const uint32_t xs[4] = {v.x, v.y, v.z, v.w};
                        for (uint32_t c = 0; c < 4; ++c)
                            if (!((xs[c] >> kn) & 1u)) count_add(s.ct, a.next_cnt, (dest + c) >> a.next_shift, 1u);
                    }
                }
            } else {
                const uint32_t nc = clamp_count(len, sl, 4u);
                const uint32_t xs[4] = {v.x, v.y, v.z, v.w};
                for (uint32_t c = 0; c < nc; ++c) {
                    const uint32_t x = xs[c];
                    const uint32_t qc = min((x >> k) & a.qmask, qmax), sc = sl + c;
                    const uint32_t dest = dbase(qc) + ((qc & 1u) ? O0 + sc - Zt : Z0 + sc);
                    if (dest < a.n) {
                        out[dest] = (TOUT)x;
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
