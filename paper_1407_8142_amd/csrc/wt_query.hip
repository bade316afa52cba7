// Batched access / rank / select on a built levelwise wavelet tree (and on
// a wavelet matrix and a 4-ary tree, further down)
// (queries as defined in "Preliminaries"; tree walks without parent/child
// pointers: node offsets come from C, in-node positions from rank/select on
// the level bitmaps).  One thread per query; each query takes L dependent
// steps of a few cached loads, so these kernels are latency-bound.
#include <hip/hip_runtime.h>

#include "../../include/wt.h"
#include "wt_device.hpp"
#include "wt_huff_tab.hpp"

namespace wt {

struct TreeDev {
    const uint64_t *bits, *C, *rank, *sel1, *sel0, *sel_counts;
    uint64_t n, sigma, W, rank_len, cap;
    uint32_t L;
};

__device__ __forceinline__ uint64_t Cat(const TreeDev &t, uint64_t x) { return t.C[x < t.sigma ? x : t.sigma]; }

// Ones of level l in [0, j), j <= n: directory entry + whole words + a partial word.
__device__ __forceinline__ uint64_t rank1(const TreeDev &t, uint32_t l, uint64_t j) {
    const uint64_t *B = t.bits + (uint64_t)l * t.W;
    uint64_t blk = j >> 9;
    uint64_t r = t.rank[(uint64_t)l * t.rank_len + blk];
    uint64_t w_end = j >> 6;
    for (uint64_t w = blk << 3; w < w_end; ++w) r += (uint64_t)__popcll(B[w]);
    if (j & 63) r += (uint64_t)__popcll(B[w_end] & ((1ull << (j & 63)) - 1ull));
    return r;
}

__device__ __forceinline__ uint64_t rank_b(const TreeDev &t, uint32_t l, uint64_t j, uint32_t b) {
    uint64_t r1 = rank1(t, l, j);
    return b ? r1 : j - r1;
}

// Position of the b-bit of level l with 0-based ordinal o (o < count of b-bits).
__device__ uint64_t select_b(const TreeDev &t, uint32_t l, uint32_t b, uint64_t o) {
    const uint64_t *samp = (b ? t.sel1 : t.sel0) + (uint64_t)l * t.cap;
    const uint64_t *R = t.rank + (uint64_t)l * t.rank_len;
    const uint64_t *B = t.bits + (uint64_t)l * t.W;
    uint64_t s = o / WT_SELECT_SAMPLE;
    uint64_t lo_pos = samp[s], hi_pos = samp[s + 1];
    // Largest 512-bit block start whose b-rank is <= o, between the samples.
    uint64_t lo = lo_pos >> 9, hi = (hi_pos >= t.n ? (t.n - 1) : hi_pos) >> 9;
    while (lo < hi) {
        uint64_t mid = (lo + hi + 1) >> 1;
        uint64_t pos = mid << 9;
        uint64_t rb = b ? R[mid] : pos - R[mid];
        if (rb <= o) lo = mid;
        else hi = mid - 1;
    }
    uint64_t pos = lo << 9;
    uint64_t rem = o - (b ? R[lo] : pos - R[lo]);
    for (uint64_t w = lo << 3; w < t.W; ++w) {
        uint64_t x = b ? B[w] : ~B[w];
        if ((w << 6) + 64 > t.n) x &= (1ull << (t.n & 63)) - 1ull;
        uint64_t c = (uint64_t)__popcll(x);
        if (rem < c) return (w << 6) + select_in_word(x, (uint32_t)rem);
        rem -= c;
    }
    return t.n;  // unreachable for a well-formed tree
}

// access(j): the symbol at position j (j < n).
__device__ __forceinline__ uint32_t access_one(const TreeDev &t, uint64_t j) {
    uint64_t p = 0;
    for (uint32_t l = 0; l < t.L; ++l) {
        uint32_t k = t.L - 1 - l;
        uint64_t a = Cat(t, p << (k + 1));
        uint32_t b = (uint32_t)((t.bits[(uint64_t)l * t.W + (j >> 6)] >> (j & 63)) & 1ull);
        uint64_t ones = rank1(t, l, j) - rank1(t, l, a);
        if (b) j = Cat(t, ((2 * p + 1) << k)) + ones;
        else j = j - ones;  // a + (j - a) - ones
        p = 2 * p + b;
        if (j >= t.n && l + 1 < t.L) break;  // unreachable for a well-formed tree
    }
    return (uint32_t)p;
}

// rank(c, i): occurrences of c < sigma in S[0, i), i <= n.
__device__ __forceinline__ uint64_t rank_one(const TreeDev &t, uint64_t c, uint64_t i) {
    if (t.L == 0) return i;
    uint64_t p = 0, r = i;  // r: elements of node p that precede the query position
    for (uint32_t l = 0; l < t.L; ++l) {
        if (r == 0) break;
        uint32_t k = t.L - 1 - l;
        uint64_t a = Cat(t, p << (k + 1));
        uint32_t b = (uint32_t)((c >> k) & 1u);
        if (a + r > t.n) break;  // unreachable for a well-formed tree
        uint64_t ones = rank1(t, l, a + r) - rank1(t, l, a);
        r = b ? ones : r - ones;
        p = 2 * p + b;
    }
    return r;
}

// select(c, kk): position of the kk-th (1-based) c, or -1.
__device__ __forceinline__ int64_t select_one(const TreeDev &t, uint64_t c, uint64_t kk) {
    if (c >= t.sigma || kk == 0 || kk > t.C[c + 1] - t.C[c]) return -1;
    uint64_t r = kk - 1;  // 0-based index inside the current child
    for (uint32_t d = t.L; d-- > 0;) {
        uint32_t k = t.L - 1 - d;
        uint64_t p = c >> (k + 1);
        uint32_t b = (uint32_t)((c >> k) & 1u);
        uint64_t a = Cat(t, p << (k + 1));
        uint64_t j = select_b(t, d, b, rank_b(t, d, a, b) + r);
        if (j >= t.n) return -1;  // unreachable for a well-formed tree
        r = j - a;
    }
    return (int64_t)r;
}

__global__ void access_kernel(TreeDev t, const uint64_t *qi, uint64_t m, uint32_t *out) {
    uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint64_t j = qi[q];
    out[q] = j >= t.n ? 0xFFFFFFFFu : access_one(t, j);
}

__global__ void rank_kernel(TreeDev t, const uint32_t *qc, const uint64_t *qi, uint64_t m, uint64_t *out) {
    uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint64_t c = qc[q], i = min(qi[q], t.n);
    out[q] = c >= t.sigma ? 0 : rank_one(t, c, i);
}

__global__ void select_kernel(TreeDev t, const uint32_t *qc, const uint64_t *qk, uint64_t m, int64_t *out) {
    uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    out[q] = select_one(t, qc[q], qk[q]);
}

__device__ __forceinline__ bool tree_of(const wt_view &v, TreeDev &t) {
    t.bits = v.bits;
    t.C = v.C;
    t.rank = v.rank;
    t.sel1 = v.sel1;
    t.sel0 = v.sel0;
    t.sel_counts = v.sel_counts;
    t.n = v.n;
    t.sigma = v.sigma;
    t.L = v.L;
    t.W = (v.n + 63) / 64;
    t.rank_len = (v.n + WT_RANK_BLOCK_BITS - 1) / WT_RANK_BLOCK_BITS + 1;
    t.cap = (v.n + WT_SELECT_SAMPLE - 1) / WT_SELECT_SAMPLE + 1;
    return v.C != nullptr;
}

// Mixed queries over many trees: query q names its tree, kind and arguments.
__global__ void multi_kernel(const wt_view *views, uint32_t ntrees, const uint32_t *qt, const uint8_t *qkind,
                             const uint64_t *qa, const uint64_t *qb, uint64_t m, int64_t *out) {
    uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint32_t ti = qt[q];
    TreeDev t;
    if (ti >= ntrees || !tree_of(views[ti], t)) {
        out[q] = WT_Q_BAD;
        return;
    }
    const uint64_t a = qa[q], b = qb[q];
    switch (qkind[q]) {
        case WT_Q_ACCESS:
            out[q] = a >= t.n ? (int64_t)0xFFFFFFFFu : (int64_t)access_one(t, a);
            break;
        case WT_Q_RANK:
            out[q] = a >= t.sigma ? 0 : (int64_t)rank_one(t, a, min(b, t.n));
            break;
        case WT_Q_SELECT:
            out[q] = select_one(t, a, b);
            break;
        default:
            out[q] = WT_Q_BAD;
    }
}

// ---- wavelet matrix (TreeDev with C unused and zeros[l] per level) ----
// Position p of level l continues on level l+1 at rank0(p), or at
// zeros[l] + rank1(p) when its bit is 1.
__device__ __forceinline__ uint64_t matrix_next(const TreeDev &t, const uint64_t *zeros, uint32_t l, uint64_t p,
                                                uint32_t b) {
    const uint64_t ones = rank1(t, l, p);
    return b ? zeros[l] + ones : p - ones;
}

__device__ __forceinline__ uint32_t matrix_access_one(const TreeDev &t, const uint64_t *zeros, uint64_t j) {
    uint32_t c = 0;
    for (uint32_t l = 0; l < t.L; ++l) {
        const uint32_t b = (uint32_t)((t.bits[(uint64_t)l * t.W + (j >> 6)] >> (j & 63)) & 1ull);
        c = (c << 1) | b;
        j = matrix_next(t, zeros, l, j, b);
        if (j >= t.n && l + 1 < t.L) break;  // unreachable for a well-formed matrix
    }
    return c;
}

// [s, e): the run of level l holding the symbols whose top bits so far are
// c's, from its start (s) to just past those that came from S[0, i) (e).
__device__ __forceinline__ void matrix_descend(const TreeDev &t, const uint64_t *zeros, uint64_t c, uint64_t &s,
                                               uint64_t &e) {
    for (uint32_t l = 0; l < t.L; ++l) {
        const uint32_t b = (uint32_t)((c >> (t.L - 1 - l)) & 1u);
        s = matrix_next(t, zeros, l, s, b);
        e = matrix_next(t, zeros, l, e, b);
    }
}

__device__ __forceinline__ uint64_t matrix_rank_one(const TreeDev &t, const uint64_t *zeros, uint64_t c,
                                                    uint64_t i) {
    uint64_t s = 0, e = i;
    matrix_descend(t, zeros, c, s, e);
    return e - s;
}

__device__ __forceinline__ int64_t matrix_select_one(const TreeDev &t, const uint64_t *zeros, uint64_t c,
                                                     uint64_t kk) {
    if (c >= t.sigma || kk == 0) return -1;
    uint64_t s = 0, e = t.n;
    matrix_descend(t, zeros, c, s, e);
    if (kk > e - s) return -1;
    uint64_t p = s + kk - 1;
    for (uint32_t l = t.L; l-- > 0;) {
        const uint32_t b = (uint32_t)((c >> (t.L - 1 - l)) & 1u);
        p = select_b(t, l, b, b ? p - zeros[l] : p);
        if (p >= t.n) return -1;  // unreachable for a well-formed matrix
    }
    return (int64_t)p;
}

__global__ void matrix_access_kernel(TreeDev t, const uint64_t *zeros, const uint64_t *qi, uint64_t m,
                                     uint32_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint64_t j = qi[q];
    out[q] = j >= t.n ? 0xFFFFFFFFu : matrix_access_one(t, zeros, j);
}

__global__ void matrix_rank_kernel(TreeDev t, const uint64_t *zeros, const uint32_t *qc, const uint64_t *qi,
                                   uint64_t m, uint64_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint64_t c = qc[q], i = min(qi[q], t.n);
    out[q] = c >= t.sigma ? 0 : matrix_rank_one(t, zeros, c, i);
}

__global__ void matrix_select_kernel(TreeDev t, const uint64_t *zeros, const uint32_t *qc, const uint64_t *qk,
                                     uint64_t m, int64_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    out[q] = matrix_select_one(t, zeros, qc[q], qk[q]);
}

static bool make_matrix(const wt_matrix_view *v, TreeDev &t) {
    if (!v) return false;
    if (v->L > 0 && (!v->zeros || (v->n > 0 && (!v->bits || !v->rank || !v->sel1 || !v->sel0)))) return false;
    t.bits = v->bits;
    t.C = nullptr;
    t.rank = v->rank;
    t.sel1 = v->sel1;
    t.sel0 = v->sel0;
    t.sel_counts = v->sel_counts;
    t.n = v->n;
    t.sigma = v->sigma;
    t.L = v->L;
    t.W = (v->n + 63) / 64;
    t.rank_len = (v->n + WT_RANK_BLOCK_BITS - 1) / WT_RANK_BLOCK_BITS + 1;
    t.cap = (v->n + WT_SELECT_SAMPLE - 1) / WT_SELECT_SAMPLE + 1;
    return true;
}

// ---- multiary tree, d = 4 ----
struct QuadDev {
    const uint64_t *digits, *C, *rank4, *sel4, *counts4;
    uint64_t n, sigma, W4, R, cap;
    uint32_t Lq;
};

// Entries equal to v among the 32 two-bit entries of x, as one bit per
// entry (bit 2i set for entry i).
__device__ __forceinline__ uint64_t match4(uint64_t x, uint32_t v) {
    constexpr uint64_t M = 0x5555555555555555ull;
    const uint64_t lo = x & M, hi = (x >> 1) & M;
    return ((v & 1u) ? lo : (~lo & M)) & ((v & 2u) ? hi : (~hi & M));
}

// Entries equal to v among entries [0, p) of level j, p <= n.
__device__ __forceinline__ uint64_t quad_rank(const QuadDev &t, uint32_t j, uint32_t v, uint64_t p) {
    const uint64_t *Dg = t.digits + (uint64_t)j * t.W4;
    const uint64_t blk = p >> 9;
    uint64_t r = t.rank4[((uint64_t)j * t.R + blk) * 4 + v];
    const uint64_t w_end = p >> 5;
    for (uint64_t w = blk << 4; w < w_end; ++w) r += (uint64_t)__popcll(match4(Dg[w], v));
    if (p & 31) r += (uint64_t)__popcll(match4(Dg[w_end], v) & ((1ull << (2 * (p & 31))) - 1ull));
    return r;
}

// Position of the entry v of level j with 0-based ordinal o (o < its count).
__device__ uint64_t quad_select(const QuadDev &t, uint32_t j, uint32_t v, uint64_t o) {
    const uint64_t *samp = t.sel4 + ((uint64_t)j * 4 + v) * t.cap;
    const uint64_t *R4 = t.rank4 + (uint64_t)j * t.R * 4;
    const uint64_t *Dg = t.digits + (uint64_t)j * t.W4;
    const uint64_t s = o / WT_SELECT_SAMPLE;
    const uint64_t lo_pos = samp[s], hi_pos = samp[s + 1];
    uint64_t lo = lo_pos >> 9, hi = (hi_pos >= t.n ? t.n - 1 : hi_pos) >> 9;
    while (lo < hi) {  // last 512-entry block whose count of v is <= o
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (R4[mid * 4 + v] <= o) lo = mid;
        else hi = mid - 1;
    }
    uint64_t rem = o - R4[lo * 4 + v];
    for (uint64_t w = lo << 4; w < t.W4; ++w) {
        uint64_t x = match4(Dg[w], v);
        if ((w << 5) + 32 > t.n) x &= (1ull << (2 * (t.n & 31))) - 1ull;
        const uint64_t c = (uint64_t)__popcll(x);
        if (rem < c) return (w << 5) + (select_in_word(x, (uint32_t)rem) >> 1);
        rem -= c;
    }
    return t.n;  // unreachable for a well-formed tree
}

__device__ __forceinline__ uint64_t quad_start(const QuadDev &t, uint64_t x) { return t.C[x < t.sigma ? x : t.sigma]; }

__device__ __forceinline__ uint32_t quad_access_one(const QuadDev &t, uint64_t p) {
    uint64_t q = 0;
    for (uint32_t j = 0; j < t.Lq; ++j) {
        const uint32_t sh = 2 * (t.Lq - 1 - j);
        const uint32_t v = (uint32_t)((t.digits[(uint64_t)j * t.W4 + (p >> 5)] >> (2 * (p & 31))) & 3u);
        const uint64_t a = quad_start(t, q << (sh + 2));
        p = quad_start(t, (4 * q + v) << sh) + quad_rank(t, j, v, p) - quad_rank(t, j, v, a);
        q = 4 * q + v;
        if (p >= t.n && j + 1 < t.Lq) break;  // unreachable for a well-formed tree
    }
    return (uint32_t)q;
}

__device__ __forceinline__ uint64_t quad_rank_one(const QuadDev &t, uint64_t c, uint64_t i) {
    uint64_t r = i;
    for (uint32_t j = 0; j < t.Lq && r; ++j) {
        const uint32_t sh = 2 * (t.Lq - 1 - j), v = (uint32_t)((c >> sh) & 3u);
        const uint64_t a = quad_start(t, (c >> (sh + 2)) << (sh + 2));
        if (a + r > t.n) break;  // unreachable for a well-formed tree
        r = quad_rank(t, j, v, a + r) - quad_rank(t, j, v, a);
    }
    return r;
}

__device__ __forceinline__ int64_t quad_select_one(const QuadDev &t, uint64_t c, uint64_t kk) {
    if (c >= t.sigma || kk == 0 || kk > t.C[c + 1] - t.C[c]) return -1;
    uint64_t r = kk - 1;
    for (uint32_t j = t.Lq; j-- > 0;) {
        const uint32_t sh = 2 * (t.Lq - 1 - j), v = (uint32_t)((c >> sh) & 3u);
        const uint64_t a = quad_start(t, (c >> (sh + 2)) << (sh + 2));
        const uint64_t p = quad_select(t, j, v, quad_rank(t, j, v, a) + r);
        if (p >= t.n) return -1;  // unreachable for a well-formed tree
        r = p - a;
    }
    return (int64_t)r;
}

__global__ void quad_access_kernel(QuadDev t, const uint64_t *qi, uint64_t m, uint32_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint64_t j = qi[q];
    out[q] = j >= t.n ? 0xFFFFFFFFu : quad_access_one(t, j);
}

__global__ void quad_rank_kernel(QuadDev t, const uint32_t *qc, const uint64_t *qi, uint64_t m, uint64_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint64_t c = qc[q], i = min(qi[q], t.n);
    out[q] = c >= t.sigma ? 0 : quad_rank_one(t, c, i);
}

__global__ void quad_select_kernel(QuadDev t, const uint32_t *qc, const uint64_t *qk, uint64_t m, int64_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    out[q] = quad_select_one(t, qc[q], qk[q]);
}

static bool make_quad(const wt_multiary_view *v, QuadDev &t) {
    if (!v || !v->C) return false;
    if (v->Lq > 0 && (!v->rank4 || !v->sel4 || (v->n > 0 && !v->digits))) return false;
    t.digits = v->digits;
    t.C = v->C;
    t.rank4 = v->rank4;
    t.sel4 = v->sel4;
    t.counts4 = v->counts4;
    t.n = v->n;
    t.sigma = v->sigma;
    t.Lq = v->Lq;
    t.W4 = (v->n + 31) / 32;
    t.R = (v->n + WT_RANK_BLOCK_BITS - 1) / WT_RANK_BLOCK_BITS + 1;
    t.cap = (v->n + WT_SELECT_SAMPLE - 1) / WT_SELECT_SAMPLE + 1;
    return true;
}

static bool make_tree(const wt_view *v, TreeDev &t) {
    if (!v || !v->C) return false;
    if (v->L > 0 && v->n > 0 && (!v->bits || !v->rank || !v->sel1 || !v->sel0)) return false;
    t.bits = v->bits;
    t.C = v->C;
    t.rank = v->rank;
    t.sel1 = v->sel1;
    t.sel0 = v->sel0;
    t.sel_counts = v->sel_counts;
    t.n = v->n;
    t.sigma = v->sigma;
    t.L = v->L;
    t.W = (v->n + 63) / 64;
    t.rank_len = (v->n + WT_RANK_BLOCK_BITS - 1) / WT_RANK_BLOCK_BITS + 1;
    t.cap = (v->n + WT_SELECT_SAMPLE - 1) / WT_SELECT_SAMPLE + 1;
    return true;
}

constexpr int kQBlock = 256;

// ---------------------------------------------------------------------------
// Huffman-shaped tree (byte alphabets).  Level d has nd[d] bits: rank and
// select run on a copy of the view with n = nd[d] (the strides stay those of
// an n-symbol tree).  A walk follows the node starts and child links of the
// build's tables; node indices are below 256 and are masked so that even a
// malformed table cannot index past them.
struct HuffDev {
    TreeDev t;  // t.L = height
    const HuffTab *tab;
};

__device__ __forceinline__ TreeDev huff_level(const HuffDev &H, uint32_t d) {
    TreeDev x = H.t;
    x.n = H.tab->nd[d];
    return x;
}

__device__ __forceinline__ uint32_t huff_access_one(const HuffDev &H, uint64_t j) {
    const HuffTab *tb = H.tab;
    if (H.t.L == 0) return tb->order[0];  // the only symbol
    uint32_t q = 0;
    for (uint32_t d = 0; d < H.t.L; ++d) {
        const TreeDev tl = huff_level(H, d);
        if (j >= tl.n) break;  // unreachable for a well-formed tree
        const uint64_t s = tb->nstart[d][q];
        const uint32_t b = (uint32_t)((tl.bits[(uint64_t)d * tl.W + (j >> 6)] >> (j & 63)) & 1ull);
        const uint64_t ones = rank1(tl, d, j) - rank1(tl, d, s);
        const uint64_t r = b ? ones : (j - s) - ones;
        const uint32_t ch = tb->child[d][2 * q + b];
        if (ch & kHuffLeaf) return ch & 0xFFu;
        if (d + 1 >= H.t.L) break;  // unreachable for a well-formed tree
        q = ch & 0xFFu;
        j = tb->nstart[d + 1][q] + r;
    }
    return 0xFFFFFFFFu;
}

__device__ __forceinline__ uint64_t huff_rank_one(const HuffDev &H, uint64_t c, uint64_t i) {
    const HuffTab *tb = H.tab;
    if (c >= H.t.sigma || tb->weight[c] == 0) return 0;
    if (H.t.L == 0) return i;  // c is the only symbol
    const uint32_t L = min(tb->lens[c], H.t.L);
    uint64_t r = i;  // elements of the current node before the query position
    for (uint32_t d = 0; d < L && r; ++d) {
        const uint32_t key = tb->lut[d][c] >> 8, q = (key >> 1) & 0xFFu, b = key & 1u;
        const TreeDev tl = huff_level(H, d);
        const uint64_t s = tb->nstart[d][q];
        if (s + r > tl.n) return 0;  // unreachable for a well-formed tree
        const uint64_t ones = rank1(tl, d, s + r) - rank1(tl, d, s);
        r = b ? ones : r - ones;
    }
    return r;
}

__device__ __forceinline__ int64_t huff_select_one(const HuffDev &H, uint64_t c, uint64_t kk) {
    const HuffTab *tb = H.tab;
    if (c >= H.t.sigma || kk == 0 || kk > tb->weight[c]) return -1;
    if (H.t.L == 0) return (int64_t)(kk - 1);
    uint64_t r = kk - 1;  // 0-based index inside the current child
    for (uint32_t d = min(tb->lens[c], H.t.L); d-- > 0;) {
        const uint32_t key = tb->lut[d][c] >> 8, q = (key >> 1) & 0xFFu, b = key & 1u;
        const TreeDev tl = huff_level(H, d);
        const uint64_t s = tb->nstart[d][q];
        const uint64_t j = select_b(tl, d, b, rank_b(tl, d, s, b) + r);
        if (j >= tl.n) return -1;  // unreachable for a well-formed tree
        r = j - s;
    }
    return (int64_t)r;
}

__global__ void huff_access_kernel(HuffDev H, const uint64_t *qi, uint64_t m, uint32_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint64_t j = qi[q];
    out[q] = j >= H.t.n ? 0xFFFFFFFFu : huff_access_one(H, j);
}

__global__ void huff_rank_kernel(HuffDev H, const uint32_t *qc, const uint64_t *qi, uint64_t m, uint64_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    out[q] = huff_rank_one(H, qc[q], min(qi[q], H.t.n));
}

__global__ void huff_select_kernel(HuffDev H, const uint32_t *qc, const uint64_t *qk, uint64_t m, int64_t *out) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    out[q] = huff_select_one(H, qc[q], qk[q]);
}

static bool make_huff(const wt_huffman_view *v, HuffDev &H) {
    if (!v || !v->tables || v->sigma == 0 || v->sigma > (uint64_t)kHuffSyms || v->h > (uint32_t)kHuffMaxLevels)
        return false;
    if (v->h > 0 && v->n > 0 && (!v->bits || !v->rank || !v->sel1 || !v->sel0)) return false;
    TreeDev &t = H.t;
    t.bits = v->bits;
    t.C = nullptr;
    t.rank = v->rank;
    t.sel1 = v->sel1;
    t.sel0 = v->sel0;
    t.sel_counts = nullptr;
    t.n = v->n;
    t.sigma = v->sigma;
    t.L = v->h;
    t.W = (v->n + 63) / 64;
    t.rank_len = (v->n + WT_RANK_BLOCK_BITS - 1) / WT_RANK_BLOCK_BITS + 1;
    t.cap = (v->n + WT_SELECT_SAMPLE - 1) / WT_SELECT_SAMPLE + 1;
    H.tab = (const HuffTab *)v->tables;
    return true;
}

}  // namespace wt

using namespace wt;

extern "C" int wt_access(const wt_view *v, const uint64_t *d_i, uint64_t m, uint32_t *d_sym, void *stream) {
    TreeDev t;
    if (!make_tree(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_i || !d_sym) return WT_ERR_ARG;
    access_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(t, d_i, m, d_sym);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_rank(const wt_view *v, const uint32_t *d_c, const uint64_t *d_i, uint64_t m, uint64_t *d_out,
                       void *stream) {
    TreeDev t;
    if (!make_tree(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_c || !d_i || !d_out) return WT_ERR_ARG;
    rank_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(t, d_c, d_i, m, d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_select(const wt_view *v, const uint32_t *d_c, const uint64_t *d_k, uint64_t m, int64_t *d_out,
                         void *stream) {
    TreeDev t;
    if (!make_tree(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_c || !d_k || !d_out) return WT_ERR_ARG;
    select_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(t, d_c, d_k, m,
                                                                                                 d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_query_multi(const wt_view *d_views, uint32_t ntrees, const uint32_t *d_tree, const uint8_t *d_kind,
                              const uint64_t *d_a, const uint64_t *d_b, uint64_t m, int64_t *d_out, void *stream) {
    if (m == 0) return WT_OK;
    if (!d_views || !d_tree || !d_kind || !d_a || !d_b || !d_out) return WT_ERR_ARG;
    multi_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(
        d_views, ntrees, d_tree, d_kind, d_a, d_b, m, d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_matrix_access(const wt_matrix_view *v, const uint64_t *d_i, uint64_t m, uint32_t *d_sym,
                                void *stream) {
    TreeDev t;
    if (!make_matrix(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_i || !d_sym) return WT_ERR_ARG;
    matrix_access_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(
        t, v->zeros, d_i, m, d_sym);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_matrix_rank(const wt_matrix_view *v, const uint32_t *d_c, const uint64_t *d_i, uint64_t m,
                              uint64_t *d_out, void *stream) {
    TreeDev t;
    if (!make_matrix(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_c || !d_i || !d_out) return WT_ERR_ARG;
    matrix_rank_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(
        t, v->zeros, d_c, d_i, m, d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_matrix_select(const wt_matrix_view *v, const uint32_t *d_c, const uint64_t *d_k, uint64_t m,
                                int64_t *d_out, void *stream) {
    TreeDev t;
    if (!make_matrix(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_c || !d_k || !d_out) return WT_ERR_ARG;
    matrix_select_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(
        t, v->zeros, d_c, d_k, m, d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_multiary_access(const wt_multiary_view *v, const uint64_t *d_i, uint64_t m, uint32_t *d_sym,
                                  void *stream) {
    QuadDev t;
    if (!make_quad(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_i || !d_sym) return WT_ERR_ARG;
    quad_access_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(t, d_i, m,
                                                                                                     d_sym);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_multiary_rank(const wt_multiary_view *v, const uint32_t *d_c, const uint64_t *d_i, uint64_t m,
                                uint64_t *d_out, void *stream) {
    QuadDev t;
    if (!make_quad(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_c || !d_i || !d_out) return WT_ERR_ARG;
    quad_rank_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(t, d_c, d_i, m,
                                                                                                   d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_multiary_select(const wt_multiary_view *v, const uint32_t *d_c, const uint64_t *d_k, uint64_t m,
                                  int64_t *d_out, void *stream) {
    QuadDev t;
    if (!make_quad(v, t)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_c || !d_k || !d_out) return WT_ERR_ARG;
    quad_select_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(t, d_c, d_k,
                                                                                                     m, d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_huffman_access(const wt_huffman_view *v, const uint64_t *d_i, uint64_t m, uint32_t *d_sym,
                                 void *stream) {
    HuffDev H;
    if (!make_huff(v, H)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_i || !d_sym) return WT_ERR_ARG;
    huff_access_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(H, d_i, m,
                                                                                                     d_sym);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_huffman_rank(const wt_huffman_view *v, const uint32_t *d_c, const uint64_t *d_i, uint64_t m,
                               uint64_t *d_out, void *stream) {
    HuffDev H;
    if (!make_huff(v, H)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_c || !d_i || !d_out) return WT_ERR_ARG;
    huff_rank_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(H, d_c, d_i, m,
                                                                                                   d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}

extern "C" int wt_huffman_select(const wt_huffman_view *v, const uint32_t *d_c, const uint64_t *d_k, uint64_t m,
                                 int64_t *d_out, void *stream) {
    HuffDev H;
    if (!make_huff(v, H)) return WT_ERR_ARG;
    if (m == 0) return WT_OK;
    if (!d_c || !d_k || !d_out) return WT_ERR_ARG;
    huff_select_kernel<<<(unsigned)((m + kQBlock - 1) / kQBlock), kQBlock, 0, (hipStream_t)stream>>>(H, d_c, d_k, m,
                                                                                                     d_out);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_HIP;
}
