// Huffman-shaped wavelet tree for byte alphabets (section "Extensions").
//
// Shape: the canonical tree of the Huffman code lengths of the symbols that
// occur (two smallest nodes joined first, in (weight, leaves before internal
// nodes, symbol / creation) order; codes in (length, symbol) order, 0 =
// left), so the in-order leaf order is (length, symbol) and the internal
// nodes of depth d are the distinct code prefixes of length d among the
// leaves deeper than d.  Level d holds the code bit d of every symbol whose
// code is longer than d, in the order of S stably sorted by its depth-d
// prefix; its length nd[d] shrinks as leaves end.
//
// The paper decides a symbol's side at a node by comparing its in-order leaf
// id with the node's split; with canonical codes that side is the code bit,
// and the whole decision for level d is a 256-entry table per level:
//   lut[d][c] = bit | next bit << 1 | continues << 2 | key << 8,
//   key = 2 * (node index of c at depth d, left to right) + bit,
// with `continues` when c's code is longer than d + 1 (else c's leaf is the
// child and c leaves the sequence here).  The level pass is the byte pass
// with table lookups for the bits: an element of run `key` (node, bit) goes
// to Dh[d][key] + (zeros, resp. ones, of the level before it), Dh holding
// the child's start in level d+1 minus the node's zeros (ones) before it.
#pragma once

#include "wt_huff_tab.hpp"
#include "wt_kernels.hpp"

namespace wt {

// Code lengths and canonical codes, one block of 256 threads (thread c is
// symbol c).  Weights come from C.  The two-queue merge is sequential (at
// most 255 joins); everything else is a count over the other symbols.
__global__ __launch_bounds__(kHuffSyms) void huff_codes(const uint64_t *C, uint32_t sigma, HuffTab *t) {
    __shared__ uint64_t w[kHuffSyms], iw[kHuffSyms], wq[kHuffSyms];
    __shared__ uint32_t lparent[kHuffSyms], len[kHuffSyms];
    __shared__ uint32_t iparent[kHuffSyms], idepth[kHuffSyms];
    __shared__ uint32_t s_m, s_h;
    const uint32_t c = threadIdx.x;
    w[c] = c < sigma ? C[c + 1] - C[c] : 0ull;
    len[c] = 0;
    if (c == 0) {
        s_m = 0;
        s_h = 0;
    }
    __syncthreads();
    const bool here = w[c] != 0;
    uint32_t rq = 0;  // rank in (weight, symbol) order: the leaf queue
    if (here) {
        for (uint32_t x = 0; x < kHuffSyms; ++x) rq += w[x] != 0 && (w[x] < w[c] || (w[x] == w[c] && x < c));
        wq[rq] = w[c];
        atomicAdd(&s_m, 1u);
    }
    __syncthreads();
    const uint32_t m = s_m;
    if (m >= 2 && c == 0) {
        // Join the two smallest of (leaf queue head, internal queue head):
        // a leaf comes first on equal weight; internal nodes appear in
        // non-decreasing weight, so their queue is their creation order.
        // The two heads stay in registers (one LDS read per join step).
        constexpr uint64_t kNone = ~0ull;
        uint32_t lh = 0, ih = 0, ni = 0;
        uint64_t lw = wq[0], hw = kNone;
        for (uint32_t s = 0; s + 1 < m; ++s) {
            uint64_t sum = 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (lh < m && (ih >= ni || lw <= hw)) {
                    sum += lw;
                    lparent[lh++] = s;  // by queue rank
                    lw = lh < m ? wq[lh] : kNone;
                } else {
                    sum += hw;
                    iparent[ih++] = s;
                    hw = ih < ni ? iw[ih] : kNone;
                }
            }
            iw[s] = sum;
            if (ih == s) hw = sum;  // the new node heads an empty queue
            ni = s + 1;
        }
        idepth[m - 2] = 0;
        for (int s = (int)m - 3; s >= 0; --s) idepth[s] = idepth[iparent[s]] + 1;
    }
    __syncthreads();
    if (m >= 2 && here) {
        len[c] = idepth[lparent[rq]] + 1;
        atomicMax(&s_h, len[c]);
    }
    __syncthreads();
    // Canonical order and codes: the left-aligned code of a leaf is the sum
    // of 2^(64 - length) over the leaves before it in (length, symbol) order.
    uint64_t code = 0;
    if (here) {
        uint32_t r = 0;
        for (uint32_t x = 0; x < kHuffSyms; ++x) {
            if (!w[x] || !(len[x] < len[c] || (len[x] == len[c] && x < c))) continue;
            ++r;
            if (len[x]) code += 1ull << (64 - len[x]);
        }
        t->order[r] = c;
    }
    t->weight[c] = w[c];
    t->lens[c] = len[c];
    t->codes[c] = code;
    if (c == 0) {
        t->m = m;
        t->h = s_h;
    }
}

// Inclusive scan over the 256 threads of a block (one value each).
template <typename T, typename Op>
__device__ __forceinline__ T huff_block_scan(T v, T *tmp, Op op) {
    const int tid = threadIdx.x;
    tmp[tid] = v;
    __syncthreads();
    for (int s = 1; s < kHuffSyms; s <<= 1) {
        const T x = tid >= s ? tmp[tid - s] : T(0);
        __syncthreads();
        if (tid >= s) tmp[tid] = op(tmp[tid], x);
        __syncthreads();
    }
    const T r = tmp[tid];
    __syncthreads();
    return r;
}

// Per-level tables, block d for level d (thread r is the leaf of canonical
// rank r).  Leaves deeper than d form a suffix of the canonical order, a
// node of depth d is a run of equal prefixes among them, and inside a node
// its left child's leaves precede its right child's.  With exclusive prefix
// sums over that order of w (all deeper leaves), w0 (their zeros) and wd
// (leaves deeper than d+1, i.e. level d+1's elements):
//   start of node q in level d          = Ew[first leaf of q]
//   zeros of level d before q           = Ew0[first leaf of q]
//   start in level d+1 of child (q, b)  = Ewd[first leaf of the child]
__global__ __launch_bounds__(kHuffSyms) void huff_levels(HuffTab *t) {
    __shared__ uint64_t tmp[kHuffSyms], Ew[kHuffSyms], Ew0[kHuffSyms], Ewd[kHuffSyms];
    __shared__ uint32_t tmp32[kHuffSyms];
    const uint32_t d = blockIdx.x, r = threadIdx.x;
    const uint32_t h = t->h, m = t->m;
    if (d >= h) return;
    t->lut[d][r] = 0;  // absent symbols, and symbols not deeper than d
    const bool have = r < m;
    const uint32_t c = have ? t->order[r] : 0u;
    const bool deep = have && t->lens[c] > d;
    const uint32_t L = deep ? t->lens[c] : 0u;
    const uint64_t code = deep ? t->codes[c] : 0ull, w = deep ? t->weight[c] : 0ull;
    const uint32_t b = deep ? (uint32_t)(code >> (63 - d)) & 1u : 0u;
    const uint64_t pref = d ? code >> (64 - d) : 0ull;
    // The previous leaf in canonical order (deep leaves are a suffix).
    const uint32_t cp = r > 0 && have ? t->order[r - 1] : 0u;
    const bool deep_p = have && r > 0 && t->lens[cp] > d;
    const uint64_t code_p = deep_p ? t->codes[cp] : 0ull;
    const uint64_t pref_p = d ? code_p >> (64 - d) : 0ull;
    const uint32_t b_p = deep_p ? (uint32_t)(code_p >> (63 - d)) & 1u : 0u;
    const bool first_g = deep && (!deep_p || pref_p != pref);
    const bool first_s = deep && (first_g || b_p != b);
    // The same for depth d+1 among the leaves deeper than d+1 (the internal
    // nodes of level d+1, for the child links).
    const bool deep1 = deep && L > d + 1, deep1_p = deep_p && t->lens[cp] > d + 1;
    const uint64_t pref1 = deep1 ? code >> (63 - d) : 0ull, pref1_p = deep1_p ? code_p >> (63 - d) : 0ull;
    const bool first_g1 = deep1 && (!deep1_p || pref1_p != pref1);
    auto add = [](uint64_t x, uint64_t y) { return x + y; };
    auto add32 = [](uint32_t x, uint32_t y) { return x + y; };
    auto mx = [](uint32_t x, uint32_t y) { return x > y ? x : y; };
    const uint64_t w0 = b ? 0ull : w, wd = L > d + 1 ? w : 0ull;
    const uint64_t iw = huff_block_scan<uint64_t>(w, tmp, add);
    const uint64_t iw0 = huff_block_scan<uint64_t>(w0, tmp, add);
    const uint64_t iwd = huff_block_scan<uint64_t>(wd, tmp, add);
    Ew[r] = iw - w;
    Ew0[r] = iw0 - w0;
    Ewd[r] = iwd - wd;
    const uint32_t q = huff_block_scan<uint32_t>(first_g ? 1u : 0u, tmp32, add32) - 1u;
    const uint32_t fg = huff_block_scan<uint32_t>(first_g ? r : 0u, tmp32, mx);
    const uint32_t fs = huff_block_scan<uint32_t>(first_s ? r : 0u, tmp32, mx);
    const uint32_t q1 = huff_block_scan<uint32_t>(first_g1 ? 1u : 0u, tmp32, add32) - 1u;
    if (deep) {
        const bool cont = L > d + 1;
        const uint32_t key = 2u * q + b;
        const uint32_t nb = cont ? (uint32_t)(code >> (62 - d)) & 1u : 0u;
        t->lut[d][c] = b | (nb << 1) | (cont ? kHuffCont : 0u) | (key << 8);
        if (cont) {
            const uint64_t before = b ? Ew[fg] - Ew0[fg] : Ew0[fg];
            t->Dh[d][key] = (uint32_t)(Ewd[fs] - before);
        }
        if (r == fg) t->nstart[d][q] = Ew[fg];
        t->child[d][key] = cont ? q1 : (kHuffLeaf | c);
    }
    if (r == kHuffSyms - 1) {
        t->nd[d] = iw;
        t->ones[d] = iw - iw0;
    }
}

// Zeros of level 0 per 16 KiB tile of S (the level-0 bit is a table lookup,
// so the histogram cannot count it).
__global__ __launch_bounds__(kBlock) void huff_count0(const uint8_t *S, uint64_t n, const HuffTab *t,
                                                      uint32_t *cnt0) {
    __shared__ uint32_t lut[kHuffSyms];
    __shared__ uint32_t red[kWaves];
    const int tid = threadIdx.x;
    lut[tid] = t->lut[0][tid];
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * 16384u;
    const uint32_t len = (uint32_t)min((uint64_t)16384u, n - t0);
    uint32_t z = 0;
    for (uint32_t p = 16u * tid; p < len; p += 16u * kBlock) {
        if (p + 16u <= len) {
            const uint4 v = *reinterpret_cast<const uint4 *>(S + t0 + p);
            const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) z += (lut[(dw[j] >> (8 * i)) & 0xFFu] & kHuffBit) ^ 1u;
        } else {
            for (uint32_t e = p; e < len; ++e) z += (lut[S[t0 + e]] & kHuffBit) ^ 1u;
        }
    }
    z = wave_sum_u32(z);
    if (lane_id() == 0) red[tid / kWave] = z;
    __syncthreads();
    if (tid == 0) cnt0[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Directory tails and the bit words past each level's end (grid.y = level):
// rank entries at or past the level's end hold its ones, unused select
// samples hold its length.
__global__ void huff_dir_finish(const HuffTab *t, uint64_t W, uint64_t *bits, uint64_t *rank, uint64_t rank_len,
                                uint64_t *sel1, uint64_t *sel0, uint64_t cap, uint64_t *sel_counts) {
    const uint32_t d = blockIdx.y, h = t->h;
    if (d >= h) return;
    const uint64_t nd = t->nd[d], ones = t->ones[d], zeros = nd - ones;
    const uint64_t c1 = cdiv(ones, WT_SELECT_SAMPLE), c0 = cdiv(zeros, WT_SELECT_SAMPLE);
    const uint64_t j0 = cdiv(nd, WT_RANK_BLOCK_BITS), w0 = cdiv(nd, 64);
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (uint64_t)gridDim.x * blockDim.x;
    if (tid == 0) {
        sel_counts[d] = c1;
        sel_counts[h + d] = c0;
    }
    for (uint64_t j = j0 + tid; j < rank_len; j += nt) rank[(uint64_t)d * rank_len + j] = ones;
    for (uint64_t e = min(c1, c0) + tid; e < cap; e += nt) {
        if (e >= c1) sel1[(uint64_t)d * cap + e] = nd;
        if (e >= c0) sel0[(uint64_t)d * cap + e] = nd;
    }
    for (uint64_t x = w0 + tid; x < W; x += nt) bits[(uint64_t)d * W + x] = 0;
}

struct HuffArgs {
    const uint8_t *in;        // S_d (nd[d] bytes)
    uint8_t *out;             // S_{d+1}
    uint64_t *bits;           // B_d
    const uint32_t *lut;      // lut[d]
    const uint32_t *Dh;       // Dh[d]
    const uint64_t *tile_prefix;
    uint32_t *next_cnt;       // zeros of level d+1 per tile (accumulated here)
    uint32_t next_shift;
    const uint32_t *status;
    uint64_t *rank, *sel1, *sel0;
    uint32_t n;               // nd[d]
    uint32_t out_n;           // nd[d+1]
};

struct LdsHuffU8 {
    static constexpr int kTile = 16384, kRows = 4, kRowBytes = 4096;
    __align__(16) uint8_t stage[kTile];
    __align__(16) uint16_t m16[kTile / 16];
    uint32_t wz[kRows][kWaves];
    uint32_t zpre[kTile / 64];
    uint32_t D[2 * kHuffSyms];
    uint32_t lut[kHuffSyms];
    CountTable ct;
};

// One tile of a Huffman level (the byte level pass with table lookups).
template <bool SCATTER, bool DIRS>
__device__ __forceinline__ void huff_tile_u8(const HuffArgs &a, uint32_t tile, LdsHuffU8 &s) {
    constexpr int kTile = LdsHuffU8::kTile, kRows = LdsHuffU8::kRows, kRowBytes = LdsHuffU8::kRowBytes;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t t0 = tile * (uint32_t)kTile;
    const uint32_t len = min((uint32_t)kTile, a.n - t0);
    const uint32_t Z0 = (uint32_t)a.tile_prefix[tile];

    const uint8_t *in = a.in + t0;
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
                for (int j = 0; j < 16; ++j) w[j >> 2] |= ((uint32_t)j < nv ? (uint32_t)in[p + j] : 0u) << (8 * (j & 3));
                d[r] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
    }
    s.lut[tid] = a.lut[tid];
    if (SCATTER) {
        s.D[tid] = a.Dh[tid];
        s.D[tid + kBlock] = a.Dh[tid + kBlock];
        count_init(s.ct, tid);
    }
    if (*a.status) return;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t p = (uint32_t)(r * kRowBytes + 16 * tid);
        const uint32_t nv = clamp_count(len, p, 16u);
        const uint32_t dw[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
        uint32_t mm = 0;
#pragma unroll
        for (int b = 0; b < 16; ++b) mm |= (s.lut[(dw[b >> 2] >> (8 * (b & 3))) & 0xFFu] & kHuffBit) << b;
        m[r] = mm & ((1u << nv) - 1u);
        z[r] = nv - (uint32_t)__popc(m[r]);
        s.m16[r * kBlock + tid] = (uint16_t)m[r];
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
    if ((tid & 3) == 0)
#pragma unroll
        for (int r = 0; r < kRows; ++r) s.zpre[r * (kBlock / 4) + tid / 4] = zl[r];
    __syncthreads();

    const uint64_t *s_w64 = reinterpret_cast<const uint64_t *>(s.m16);
    if ((uint32_t)tid * 64u < len) a.bits[(t0 >> 6) + tid] = s_w64[tid];
    if (DIRS) {
        const uint32_t wbase = (uint32_t)wave * kRowBytes;
        if (wbase < len) {
            const uint32_t zb = s.zpre[wave * kWave];
            const uint32_t ze = wave + 1 < kWaves ? s.zpre[(wave + 1) * kWave] : Zt;
            const uint64_t wd[1] = {s_w64[tid]};
            const uint32_t zp[1] = {s.zpre[tid] - zb};
            emit_directories<1>(wd, zp, (uint64_t)Z0 + zb, (uint64_t)t0 + wbase,
                                clamp_count(len, wbase, (uint32_t)kRowBytes), ze - zb, a.n, a.rank, a.sel1, a.sel0,
                                lane);
        }
    }
    if (!SCATTER) return;

    // Stable split (as in the byte pass): positions past the end of a short
    // tile count as ones, so they land on slots [len, kTile).
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t e0 = (uint32_t)(r * kRowBytes + 16 * tid);
        const uint32_t nv = clamp_count(len, e0, 16u);
        const uint32_t ms = m[r] | (0xFFFFu & ~((1u << nv) - 1u));
        uint32_t A = zl[r] | ((Zt + e0 - zl[r]) << 16);
        const uint32_t dw[4] = {d[r].x, d[r].y, d[r].z, d[r].w};
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const uint32_t sh = ((ms >> b) & 1u) << 4;
            s.stage[__builtin_amdgcn_ubfe(A, sh, 16u)] = (uint8_t)(dw[b >> 2] >> (8 * (b & 3)));
            A += 1u << sh;
        }
    }
    __syncthreads();

    // Scatter: a run (same node and bit) goes to one child; a leaf child
    // takes nothing (its symbols leave the sequence).
    const uint32_t O0 = t0 - Z0;
    const uint32_t n16 = a.out_n > 15u ? a.out_n - 15u : 0u;
    const uint4 *s_st128 = reinterpret_cast<const uint4 *>(s.stage);
    constexpr int kChunksPerWave = kTile / 16 / kWaves;
    LaneCount lc;
#pragma unroll
    for (int i = 0; i < kChunksPerWave / kWave; ++i) {
        const uint32_t j = (uint32_t)(wave * kChunksPerWave + i * kWave + lane), sl = 16u * j;
        uint32_t ftile = kNoTile, fcnt = 0;
        if (sl < len) {
            const uint4 v = s_st128[j];
            const uint32_t e0 = s.lut[v.x & 0xFFu], e15 = s.lut[v.w >> 24];
            const uint32_t k0 = e0 >> 8;
            if (sl + 15 < len && k0 == (e15 >> 8)) {
                if (e0 & kHuffCont) {
                    const uint32_t dest = s.D[k0] + ((k0 & 1u) ? O0 + sl - Zt : Z0 + sl);
                    if (dest < n16) {
                        *reinterpret_cast<u128_unaligned *>(a.out + dest) = u128_unaligned{v.x, v.y, v.z, v.w};
                        const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
                        uint32_t zn = 0;
#pragma unroll
                        for (int b = 0; b < 16; ++b)
                            zn += ((s.lut[(dw[b >> 2] >> (8 * (b & 3))) & 0xFFu] >> 1) & 1u) ^ 1u;
                        const uint32_t nt = dest >> a.next_shift;
                        if (((dest + 15) >> a.next_shift) == nt) {
                            lc.step(nt, zn, ftile, fcnt);
                        } else {
                            for (uint32_t c = 0; c < 16; ++c)
                                if (!(s.lut[byte_of(v, (int)c)] & kHuffNext))
                                    count_add(s.ct, a.next_cnt, (dest + c) >> a.next_shift, 1u);
                        }
                    }
                }
            } else {
                const uint32_t nc = clamp_count(len, sl, 16u);
                for (uint32_t c = 0; c < nc; ++c) {
                    const uint32_t x = byte_of(v, (int)c), e = s.lut[x], kc = e >> 8, sc = sl + c;
                    if (!(e & kHuffCont)) continue;
                    const uint32_t dest = s.D[kc] + ((kc & 1u) ? O0 + sc - Zt : Z0 + sc);
                    if (dest < a.out_n) {
                        a.out[dest] = (uint8_t)x;
                        if (!(e & kHuffNext)) count_add(s.ct, a.next_cnt, dest >> a.next_shift, 1u);
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

template <bool SCATTER, bool DIRS>
__global__ __launch_bounds__(kBlock) void huff_level_pass(HuffArgs a) {
    __shared__ LdsHuffU8 s;
    huff_tile_u8<SCATTER, DIRS>(a, blockIdx.x, s);
}

}  // namespace wt
