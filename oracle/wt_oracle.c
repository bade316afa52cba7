/*
 * wt_oracle.c -- plain, slow, sequential reference for wavelet-tree
 * construction (Shun, "Parallel Wavelet Tree Construction").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the HIP library, and the library never calls it.
 *
 * Everything here is integer arithmetic and single-threaded.  No blocking,
 * fusion or reordering beyond what the paper states.
 *
 * Pins (what this file is checked against, in the CPU test suite):
 *   - bits: the sortWT closed form (Fig. 2): level l is S stably sorted by
 *     its top l bits, brute-forced in Python over every tiny input;
 *   - popcount per level equals the count of symbols with that bit set;
 *   - C against a histogram computed by numpy;
 *   - directories against a naive Python popcount / scan;
 *   - tree-walking access/rank/select against naive counting over S;
 *   - hand-derived fixtures under tests/golden/;
 *   - wavelet matrix: its sort view (level l is S stably sorted by the
 *     reverse of its top l bits), per-level zero counts by numpy, equality
 *     with the tree for sigma <= 2, and matrix-walking queries against
 *     naive counting;
 *   - Huffman-shaped tree: hand-derived code lengths on ties, optimality
 *     by brute force over every Kraft-complete length vector, prefix-free
 *     canonical codes, a decoder that walks the levels back to S, level
 *     sizes from the weights, and equality with the binary tree for equal
 *     weights over a power-of-two alphabet;
 *   - planted mutants of this file (ORACLE_MUTANT) must fail those pins.
 *
 * Readings where the paper is silent are listed next to the code below.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_SYMBOL (-2)
#define OR_ERR_NOMEM (-6)

/* Directory constants of the oracle's reading (the paper fixes none, see
 * "Parallel Construction of Rank/Select Structures": Jacobson blocks and
 * Clark samples are sized asymptotically).  One absolute count per 512
 * bits, one sample per 4096 ones and per 4096 zeros. */
#define OR_RANK_BLOCK_BITS 512u
#define OR_SEL_SAMPLE 4096u

/* Read symbol i of a packed little-endian array of sym_bytes-wide symbols. */
static uint64_t sym_at(const void *S, int sym_bytes, uint64_t i)
{
    if (sym_bytes == 1)
        return ((const uint8_t *)S)[i];
    if (sym_bytes == 2)
        return ((const uint16_t *)S)[i];
    return ((const uint32_t *)S)[i];
}

/* L = ceil(log2 sigma), computed with integers (Preliminaries: the root
 * represents [0, 2^ceil(log sigma) - 1]).  sigma = 1 gives L = 0: the
 * levelWT loop over levels runs zero times (reading: no bitmaps at all). */
uint32_t oracle_levels(uint64_t sigma)
{
    uint32_t L = 0;
    while (L < 64 && (((uint64_t)1) << L) < sigma)
        L++;
    return L;
}

static void set_bit(uint64_t *words, uint64_t pos)
{
    /* Reading of the word layout (the paper only says "bit arithmetic"):
     * position i lives in word i/64 at bit i%64. */
    words[pos / 64] |= ((uint64_t)1) << (pos % 64);
}

static int get_bit(const uint64_t *words, uint64_t pos)
{
    return (int)((words[pos / 64] >> (pos % 64)) & 1u);
}

/* One entry of the node array A of Fig. 1: (start, len, id, range), plus
 * the smallest symbol of the node's range, lo, which Fig. 1 carries
 * implicitly through id. */
typedef struct {
    uint64_t start, len, id, range, lo;
} or_node;

/*
 * Level-by-level construction (levelWT of Fig. 1, run sequentially, i.e.
 * the serialWT order of the Experiments section).
 *
 * S: n symbols of sym_bytes each.  Outputs:
 *   bits: L*W words, W = ceil(n/64); level l occupies words [l*W, (l+1)*W)
 *         (the levelwise representation of the Experiments section);
 *   C:    sigma+1 entries, C[c] = number of symbols < c.  The nodes of level
 *         l are determined by C (the node holding symbols [a, b] occupies
 *         positions [C[a], C[b+1]) of every level bitmap it appears in).
 *
 * Returns OR_ERR_SYMBOL if some S[i] >= sigma (the paper assumes symbols lie
 * in [0, sigma); the oracle's reading is to reject other input).
 */
int oracle_build(const void *S, uint64_t n, uint64_t sigma, int sym_bytes,
                 uint64_t *bits, uint64_t *C)
{
    if (sigma == 0 || (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4))
        return OR_ERR_ARG;
    if (sym_bytes < 4 && sigma > (((uint64_t)1) << (8 * sym_bytes)))
        return OR_ERR_ARG;
    if (sym_bytes == 4 && sigma > (((uint64_t)1) << 32))
        return OR_ERR_ARG;

    for (uint64_t i = 0; i < n; i++)
        if (sym_at(S, sym_bytes, i) >= sigma)
            return OR_ERR_SYMBOL;

    /* C[c] = #{i : S[i] < c}: counts, then running sums. */
    memset(C, 0, (size_t)(sigma + 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++)
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 4
        /* planted mistake: C[c] counts symbols <= c */
        C[sym_at(S, sym_bytes, i)] += 1;
#else
        C[sym_at(S, sym_bytes, i) + 1] += 1;
#endif
    for (uint64_t c = 1; c <= sigma; c++)
        C[c] += C[c - 1];

    uint32_t L = oracle_levels(sigma);
    uint64_t W = (n + 63) / 64;
    if (L == 0)
        return OR_OK;
    memset(bits, 0, (size_t)(L * W) * sizeof(uint64_t));
    if (n == 0)
        return OR_OK;

    /* S and S' of Fig. 1, widened to 64 bits. */
    uint64_t *cur = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint64_t *nxt = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    /* X of Fig. 1 (per-node prefix sums of the "left" flags). */
    uint64_t *X = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    /* A and A' hold at most min(n, 2^l) non-empty nodes. */
    uint64_t amax = n < (((uint64_t)1) << (L < 40 ? L : 40)) ? n : (((uint64_t)1) << (L < 40 ? L : 40));
    or_node *A = (or_node *)malloc((size_t)(amax + 1) * sizeof(or_node));
    or_node *A2 = (or_node *)malloc((size_t)(2 * amax + 2) * sizeof(or_node));
    if (!cur || !nxt || !X || !A || !A2) {
        free(cur); free(nxt); free(X); free(A); free(A2);
        return OR_ERR_NOMEM;
    }
    for (uint64_t i = 0; i < n; i++)
        cur[i] = sym_at(S, sym_bytes, i);

    /* A = {(0, n, 0, 2^L)}: the root covers every position and the symbol
     * range [0, 2^L - 1]. */
    uint64_t na = 1;
    A[0].start = 0;
    A[0].len = n;
    A[0].id = 0;
    A[0].range = ((uint64_t)1) << L;
    A[0].lo = 0;

    for (uint32_t l = 0; l < L; l++) {
        uint64_t *B = bits + (uint64_t)l * W;
        uint64_t na2 = 0;
        for (uint64_t j = 0; j < na; j++) {
            const or_node *v = &A[j];
            /* A node of range [a, b] marks a symbol 0 when it lies in
             * [a, (a+b+1)/2 - 1] and 1 otherwise (Preliminaries). */
            uint64_t a = v->lo, b = v->lo + v->range - 1;
            uint64_t mid = (a + b + 1) / 2;
            /* Bits of this node (the loops of Fig. 1 that set B). */
            for (uint64_t i = 0; i < v->len; i++) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 1
                /* planted mistake: off-by-one midpoint */
                if (cur[v->start + i] > mid)
#else
                if (cur[v->start + i] >= mid)
#endif
                    set_bit(B, v->start + i);
            }
            if (v->range <= 2)
                continue; /* no children: the recursion stops at range <= 2 */

            /* X[i] = 1 for symbols going left; exclusive prefix sum gives
             * their offsets, X_s is the total (Fig. 1). */
            uint64_t Xs = 0;
            for (uint64_t i = 0; i < v->len; i++) {
                uint64_t left = cur[v->start + i] < mid ? 1u : 0u;
                X[i] = Xs;
                Xs += left;
            }
            for (uint64_t i = 0; i < v->len; i++) {
                uint64_t s = cur[v->start + i];
                if (s >= mid) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 2
                    /* planted mistake: right child written in reverse */
                    nxt[v->start + v->len - 1 - (i - X[i])] = s;
#else
                    nxt[v->start + Xs + i - X[i]] = s;
#endif
                } else {
                    nxt[v->start + X[i]] = s;
                }
            }
            /* Children, ids 2*id+1 and 2*id+2, each of half the range;
             * empty children are dropped (the filter of Fig. 1). */
            if (Xs > 0) {
                or_node *c = &A2[na2++];
                c->start = v->start;
                c->len = Xs;
                c->id = 2 * v->id + 1;
                c->range = v->range / 2;
                c->lo = a;
            }
            if (v->len - Xs > 0) {
                or_node *c = &A2[na2++];
                c->start = v->start + Xs;
                c->len = v->len - Xs;
                c->id = 2 * v->id + 2;
                c->range = v->range / 2;
                c->lo = mid;
            }
        }
        if (l + 1 < L) {
            /* swap(S, S') and A <- filtered A' */
            uint64_t *t = cur;
            cur = nxt;
            nxt = t;
            memcpy(A, A2, (size_t)na2 * sizeof(or_node));
            na = na2;
        }
    }
    free(cur); free(nxt); free(X); free(A); free(A2);
    return OR_OK;
}

/*
 * Rank/select directories over each level bitmap (section "Parallel
 * Construction of Rank/Select Structures", in a practical fixed-constant
 * reading):
 *   rank[l][j] = number of 1s of B_l in positions [0, min(512 j, n)),
 *                j = 0 .. ceil(n/512)                      (rank_len entries)
 *   sel1[l][t] = position of the 1 whose 0-based ordinal is 4096 t,
 *                t < ceil(ones_l / 4096); the remaining entries up to
 *                sel_cap = ceil(n/4096) + 1 hold n.  sel0 likewise for 0s.
 *   sel_counts[l] = ceil(ones_l/4096), sel_counts[L + l] = ceil(zeros_l/4096).
 */
int oracle_rank_select(const uint64_t *bits, uint64_t n, uint32_t L,
                       uint64_t *rank, uint64_t *sel1, uint64_t *sel0,
                       uint64_t *sel_counts)
{
    uint64_t W = (n + 63) / 64;
    uint64_t rank_len = (n + OR_RANK_BLOCK_BITS - 1) / OR_RANK_BLOCK_BITS + 1;
    uint64_t cap = (n + OR_SEL_SAMPLE - 1) / OR_SEL_SAMPLE + 1;
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t *B = bits + (uint64_t)l * W;
        uint64_t *R = rank + (uint64_t)l * rank_len;
        uint64_t *P1 = sel1 + (uint64_t)l * cap;
        uint64_t *P0 = sel0 + (uint64_t)l * cap;
        uint64_t ones = 0, zeros = 0, t1 = 0, t0 = 0;
        for (uint64_t t = 0; t < cap; t++) {
            P1[t] = n;
            P0[t] = n;
        }
        for (uint64_t i = 0; i < n; i++) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 3
            /* planted mistake: block count includes the bit at the boundary */
            if (i % OR_RANK_BLOCK_BITS == 0)
                R[i / OR_RANK_BLOCK_BITS] = ones + (uint64_t)get_bit(B, i);
#else
            if (i % OR_RANK_BLOCK_BITS == 0)
                R[i / OR_RANK_BLOCK_BITS] = ones;
#endif
            if (get_bit(B, i)) {
                if (ones % OR_SEL_SAMPLE == 0)
                    P1[t1++] = i;
                ones++;
            } else {
                if (zeros % OR_SEL_SAMPLE == 0)
                    P0[t0++] = i;
                zeros++;
            }
        }
        R[rank_len - 1] = ones;
        sel_counts[l] = t1;
        sel_counts[L + l] = t0;
    }
    return OR_OK;
}

/* ---- queries (Preliminaries) -------------------------------------------
 * Naive versions over S itself.  Reading of the conventions:
 *   access(i) = S[i];
 *   rank(c, i) = number of c in S[0, i)  (the paper counts 0..i inclusive,
 *                so the paper's rank_c(S, i) is rank(c, i + 1) here);
 *   select(c, k) = position of the k-th c, k >= 1; -1 when there is none.
 */
uint64_t oracle_access_naive(const void *S, int sym_bytes, uint64_t i)
{
    return sym_at(S, sym_bytes, i);
}

uint64_t oracle_rank_naive(const void *S, int sym_bytes, uint64_t n, uint64_t c, uint64_t i)
{
    uint64_t r = 0;
    if (i > n)
        i = n;
    for (uint64_t j = 0; j < i; j++)
        r += sym_at(S, sym_bytes, j) == c;
    return r;
}

int64_t oracle_select_naive(const void *S, int sym_bytes, uint64_t n, uint64_t c, uint64_t k)
{
    uint64_t seen = 0;
    if (k == 0)
        return -1;
    for (uint64_t j = 0; j < n; j++)
        if (sym_at(S, sym_bytes, j) == c && ++seen == k)
            return (int64_t)j;
    return -1;
}

/* Tree-walking queries over the oracle's own bits and C, counting bits one
 * at a time (no directories), so that they test the tree itself. */
static uint64_t count_ones(const uint64_t *B, uint64_t from, uint64_t to)
{
    uint64_t r = 0;
    for (uint64_t i = from; i < to; i++)
        r += (uint64_t)get_bit(B, i);
    return r;
}

/* Position of the node that holds the symbol range starting at lo. */
static uint64_t node_start(const uint64_t *C, uint64_t sigma, uint64_t lo)
{
    return C[lo < sigma ? lo : sigma];
}

uint64_t oracle_access_tree(const uint64_t *bits, const uint64_t *C, uint64_t n,
                            uint64_t sigma, uint64_t i)
{
    uint32_t L = oracle_levels(sigma);
    uint64_t W = (n + 63) / 64;
    uint64_t lo = 0, range = ((uint64_t)1) << L, j = i;
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t *B = bits + (uint64_t)l * W;
        uint64_t a = node_start(C, sigma, lo);
        uint64_t half = range / 2;
        uint64_t ones_before = count_ones(B, a, j);
        if (get_bit(B, j)) {
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 5
            /* planted mistake: right child placed at the parent's start */
            uint64_t child = node_start(C, sigma, lo);
#else
            uint64_t child = node_start(C, sigma, lo + half);
#endif
            j = child + ones_before;
            lo += half;
        } else {
            j = a + (j - a - ones_before);
        }
        range = half;
    }
    return lo;
}

uint64_t oracle_rank_tree(const uint64_t *bits, const uint64_t *C, uint64_t n,
                          uint64_t sigma, uint64_t c, uint64_t i)
{
    uint32_t L = oracle_levels(sigma);
    uint64_t W = (n + 63) / 64;
    uint64_t lo = 0, range = ((uint64_t)1) << L, r;
    if (c >= sigma)
        return 0;
    if (i > n)
        i = n;
    r = i; /* elements of the current node that precede the query position */
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t *B = bits + (uint64_t)l * W;
        uint64_t a = node_start(C, sigma, lo);
        uint64_t half = range / 2;
        uint64_t ones_before = count_ones(B, a, a + r);
        if (c >= lo + half) {
            r = ones_before;
            lo += half;
        } else {
            r = r - ones_before;
        }
        range = half;
    }
    return r;
}

/* Position of the bit equal to b with 0-based ordinal o among positions
 * [a, n) of B, by a plain scan. */
static uint64_t scan_select(const uint64_t *B, uint64_t a, uint64_t n, int b, uint64_t o)
{
    for (uint64_t i = a; i < n; i++)
        if (get_bit(B, i) == b && o-- == 0)
            return i;
    return n;
}

int64_t oracle_select_tree(const uint64_t *bits, const uint64_t *C, uint64_t n,
                           uint64_t sigma, uint64_t c, uint64_t k)
{
    uint32_t L = oracle_levels(sigma);
    uint64_t W = (n + 63) / 64;
    if (c >= sigma || k == 0 || k > C[c + 1] - C[c])
        return -1;
    /* Ascend from the leaf of c: r is the 0-based index inside the child. */
    uint64_t r = k - 1;
    for (uint32_t d = L; d-- > 0;) {
        const uint64_t *B = bits + (uint64_t)d * W;
        uint64_t range = ((uint64_t)1) << (L - d);
        uint64_t lo = (c / range) * range;
        uint64_t a = node_start(C, sigma, lo);
        int b = c >= lo + range / 2;
        uint64_t j = scan_select(B, a, n, b, r);
        r = j - a;
    }
    return (int64_t)r;
}

/* ---- wavelet matrix (the variant described with the paper's extensions) ---
 * One bitmap per level and no nodes.  Level 0 lists the symbols in input
 * order.  Level l+1 lists level l's symbols with those whose bit (L-1-l) is
 * 0 first and those whose bit is 1 after, each group in its level-l order.
 * The bitmap of level l holds bit (L-1-l) of level l's symbols, and level l
 * keeps its number of 0s, zeros[l].  Written from that definition: one pass
 * to set the bits and count the 0s, two passes for the stable split. */
int oracle_build_matrix(const void *S, uint64_t n, uint64_t sigma, int sym_bytes,
                        uint64_t *bits, uint64_t *zeros)
{
    uint32_t L;
    uint64_t W = (n + 63) / 64;
    uint64_t *cur, *nxt;
    if (sigma == 0 || (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4))
        return OR_ERR_ARG;
    L = oracle_levels(sigma);
    cur = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    nxt = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    if (!cur || !nxt) {
        free(cur);
        free(nxt);
        return OR_ERR_NOMEM;
    }
    for (uint64_t i = 0; i < n; i++) {
        cur[i] = sym_at(S, sym_bytes, i);
        if (cur[i] >= sigma) {
            free(cur);
            free(nxt);
            return OR_ERR_SYMBOL;
        }
    }
    if (L && W)
        memset(bits, 0, (size_t)(L * W) * sizeof(uint64_t));
    for (uint32_t l = 0; l < L; l++) {
        uint32_t k = L - 1 - l;
        uint64_t *B = bits + (uint64_t)l * W;
        uint64_t z = 0, o = 0;
        for (uint64_t i = 0; i < n; i++) {
            if ((cur[i] >> k) & 1)
                set_bit(B, i);
            else
                z++;
        }
        zeros[l] = z;
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 6
        /* planted mistake: the 1s of the level placed first */
        for (uint64_t i = 0; i < n; i++)
            if ((cur[i] >> k) & 1)
                nxt[o++] = cur[i];
        for (uint64_t i = 0; i < n; i++)
            if (!((cur[i] >> k) & 1))
                nxt[o++] = cur[i];
#else
        for (uint64_t i = 0; i < n; i++)
            if (!((cur[i] >> k) & 1))
                nxt[o++] = cur[i];
        for (uint64_t i = 0; i < n; i++)
            if ((cur[i] >> k) & 1)
                nxt[o++] = cur[i];
#endif
        { uint64_t *t = cur; cur = nxt; nxt = t; }
    }
    free(cur);
    free(nxt);
    return OR_OK;
}

/* Matrix-walking queries over the oracle's own bits and zeros, counting bits
 * one at a time.  A position p of level l moves to level l+1 as the number
 * of 0s before it (its bit is 0) or zeros[l] + the number of 1s before it. */
static uint64_t matrix_next(const uint64_t *B, uint64_t z, uint64_t p, int b)
{
    uint64_t ones = count_ones(B, 0, p);
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 7
    /* planted mistake: a 1 moves to its rank among the 1s, without zeros[l] */
    (void)z;
    return b ? ones : p - ones;
#else
    return b ? z + ones : p - ones;
#endif
}

uint64_t oracle_access_matrix(const uint64_t *bits, const uint64_t *zeros, uint64_t n,
                              uint64_t sigma, uint64_t i)
{
    uint32_t L = oracle_levels(sigma);
    uint64_t W = (n + 63) / 64, c = 0, p = i;
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t *B = bits + (uint64_t)l * W;
        int b = get_bit(B, p);
        c = (c << 1) | (uint64_t)b;
        p = matrix_next(B, zeros[l], p, b);
    }
    return c;
}

/* [s, e) is, at every level, the run of positions holding the symbols whose
 * top bits so far match c's (s: where that run starts, e: just past the ones
 * that came from S[0, i)). */
uint64_t oracle_rank_matrix(const uint64_t *bits, const uint64_t *zeros, uint64_t n,
                            uint64_t sigma, uint64_t c, uint64_t i)
{
    uint32_t L = oracle_levels(sigma);
    uint64_t W = (n + 63) / 64, s = 0, e;
    if (c >= sigma)
        return 0;
    e = i > n ? n : i;
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t *B = bits + (uint64_t)l * W;
        int b = (int)((c >> (L - 1 - l)) & 1);
        s = matrix_next(B, zeros[l], s, b);
        e = matrix_next(B, zeros[l], e, b);
    }
    return e - s;
}

/* Descend to the run of c on the last level, take its k-th position, and
 * climb back with the k-th 0 or 1 of each level. */
int64_t oracle_select_matrix(const uint64_t *bits, const uint64_t *zeros, uint64_t n,
                             uint64_t sigma, uint64_t c, uint64_t k)
{
    uint32_t L = oracle_levels(sigma);
    uint64_t W = (n + 63) / 64, s = 0, e = n, p;
    if (c >= sigma || k == 0)
        return -1;
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t *B = bits + (uint64_t)l * W;
        int b = (int)((c >> (L - 1 - l)) & 1);
        s = matrix_next(B, zeros[l], s, b);
        e = matrix_next(B, zeros[l], e, b);
    }
    if (k > e - s)
        return -1;
    p = s + k - 1;
    for (uint32_t l = L; l-- > 0;) {
        const uint64_t *B = bits + (uint64_t)l * W;
        int b = (int)((c >> (L - 1 - l)) & 1);
        p = scan_select(B, 0, n, b, b ? p - zeros[l] : p);
    }
    return (int64_t)p;
}

/* ---- multiary wavelet tree, d = 4 (the paper's multiary variant) ----------
 * Each node has up to 4 children and stores 2-bit entries.  With L binary
 * levels the tree has Lq = ceil(L / 2) levels; codes are read as Lq base-4
 * digits (a leading 0 bit when L is odd).  Level j lists S sorted stably by
 * its top j digits, and its entry for a symbol is the symbol's digit j (from
 * the top).  The construction keeps the sorted sequence from level to level:
 * on level j the sequence is already sorted by the top j digits, so each
 * run of equal top-j digits (a node, found by scanning for where that prefix
 * changes) is sorted stably by digit j with a 4-bucket counting sort.
 * Entry i of level j is bits 2(i mod 32) and 2(i mod 32)+1 of word i / 32 of
 * digits[j * W4 + .], W4 = ceil(n / 32). */
uint32_t oracle_levels4(uint64_t sigma)
{
    return (oracle_levels(sigma) + 1) / 2;
}

static uint32_t digit_at(uint64_t x, uint32_t Lq, uint32_t j)
{
    return (uint32_t)((x >> (2 * (Lq - 1 - j))) & 3);
}

int oracle_build_multiary(const void *S, uint64_t n, uint64_t sigma, int sym_bytes, uint64_t *digits,
                          uint64_t *C)
{
    uint32_t Lq;
    uint64_t W4 = (n + 31) / 32;
    uint64_t *cur, *nxt;
    if (sigma == 0 || (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4))
        return OR_ERR_ARG;
    Lq = oracle_levels4(sigma);
    cur = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    nxt = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    if (!cur || !nxt) {
        free(cur);
        free(nxt);
        return OR_ERR_NOMEM;
    }
    memset(C, 0, (size_t)(sigma + 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++) {
        cur[i] = sym_at(S, sym_bytes, i);
        if (cur[i] >= sigma) {
            free(cur);
            free(nxt);
            return OR_ERR_SYMBOL;
        }
        C[cur[i] + 1]++;
    }
    for (uint64_t c = 0; c < sigma; c++)
        C[c + 1] += C[c];
    if (Lq && W4)
        memset(digits, 0, (size_t)(Lq * W4) * sizeof(uint64_t));
    for (uint32_t j = 0; j < Lq; j++) {
        uint64_t *Dg = digits + (uint64_t)j * W4;
        uint32_t shift = 2 * (Lq - 1 - j) + 2; /* the top j digits are x >> shift */
        for (uint64_t i = 0; i < n; i++)
            Dg[i / 32] |= (uint64_t)digit_at(cur[i], Lq, j) << (2 * (i % 32));
        if (j + 1 == Lq)
            break;
        /* nodes: maximal runs of equal top-j digits; a stable 4-bucket sort in each */
        for (uint64_t a = 0; a < n;) {
            uint64_t e = a + 1, cnt[4] = {0, 0, 0, 0}, off[4];
            while (e < n && (cur[e] >> shift) == (cur[a] >> shift))
                e++;
            for (uint64_t i = a; i < e; i++)
                cnt[digit_at(cur[i], Lq, j)]++;
            off[0] = a;
            for (int v = 1; v < 4; v++)
                off[v] = off[v - 1] + cnt[v - 1];
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 8
            /* planted mistake: buckets 1 and 2 swapped */
            { uint64_t t = off[1]; off[1] = off[0] + cnt[0] + cnt[2]; off[2] = t; }
#endif
            for (uint64_t i = a; i < e; i++)
                nxt[off[digit_at(cur[i], Lq, j)]++] = cur[i];
            a = e;
        }
        { uint64_t *t = cur; cur = nxt; nxt = t; }
    }
    free(cur);
    free(nxt);
    return OR_OK;
}

static uint32_t digit_of(const uint64_t *Dg, uint64_t i)
{
    return (uint32_t)((Dg[i / 32] >> (2 * (i % 32))) & 3);
}

/* Directories of the 4-ary levels (the paper leaves the structure for larger
 * alphabets to its generalized rank/select; this reading keeps one absolute
 * count per digit value every 512 entries and one sample per 4096
 * occurrences of each value):
 *   rank4[(j * R + b) * 4 + v] = occurrences of v among entries [0, min(512 b, n)), b <= ceil(n/512);
 *   sel4[(j * 4 + v) * cap + t] = position of the occurrence of v with 0-based ordinal 4096 t
 *                                 (n past the last), cap = ceil(n/4096) + 1;
 *   counts4[j * 4 + v] = ceil(occurrences of v / 4096). */
int oracle_rank_select4(const uint64_t *digits, uint64_t n, uint32_t Lq, uint64_t *rank4, uint64_t *sel4,
                        uint64_t *counts4)
{
    uint64_t W4 = (n + 31) / 32;
    uint64_t R = (n + OR_RANK_BLOCK_BITS - 1) / OR_RANK_BLOCK_BITS + 1;
    uint64_t cap = (n + OR_SEL_SAMPLE - 1) / OR_SEL_SAMPLE + 1;
    for (uint32_t j = 0; j < Lq; j++) {
        const uint64_t *Dg = digits + (uint64_t)j * W4;
        uint64_t seen[4] = {0, 0, 0, 0};
        for (uint64_t t = 0; t < 4 * cap; t++)
            sel4[(uint64_t)j * 4 * cap + t] = n;
        for (uint64_t i = 0; i <= n; i++) {
            if (i % OR_RANK_BLOCK_BITS == 0)
                for (int v = 0; v < 4; v++)
                    rank4[((uint64_t)j * R + i / OR_RANK_BLOCK_BITS) * 4 + v] = seen[v];
            if (i == n)
                break;
            uint32_t v = digit_of(Dg, i);
            if (seen[v] % OR_SEL_SAMPLE == 0)
                sel4[((uint64_t)j * 4 + v) * cap + seen[v] / OR_SEL_SAMPLE] = i;
            seen[v]++;
        }
        if (n % OR_RANK_BLOCK_BITS != 0)
            for (int v = 0; v < 4; v++)
                rank4[((uint64_t)j * R + R - 1) * 4 + v] = seen[v];
        for (int v = 0; v < 4; v++)
            counts4[(uint64_t)j * 4 + v] = (seen[v] + OR_SEL_SAMPLE - 1) / OR_SEL_SAMPLE;
    }
    return OR_OK;
}

/* Tree-walking queries over the oracle's own digits and C, counting entries
 * one at a time.  Node q of level j holds the symbols whose top j digits are
 * q; it starts at C[q * 4^(Lq-j)] and its child v at C[(4q + v) * 4^(Lq-j-1)]. */
static uint64_t count_digit(const uint64_t *Dg, uint64_t from, uint64_t to, uint32_t v)
{
    uint64_t r = 0;
    for (uint64_t i = from; i < to; i++)
        r += digit_of(Dg, i) == v;
    return r;
}

static uint64_t start_of(const uint64_t *C, uint64_t sigma, uint64_t x)
{
    return C[x < sigma ? x : sigma];
}

uint64_t oracle_access_multiary(const uint64_t *digits, const uint64_t *C, uint64_t n, uint64_t sigma,
                                uint64_t i)
{
    uint32_t Lq = oracle_levels4(sigma);
    uint64_t W4 = (n + 31) / 32, q = 0, p = i;
    for (uint32_t j = 0; j < Lq; j++) {
        const uint64_t *Dg = digits + (uint64_t)j * W4;
        uint32_t sh = 2 * (Lq - 1 - j);
        uint32_t v = digit_of(Dg, p);
        uint64_t a = start_of(C, sigma, q << (sh + 2));
        uint64_t child = start_of(C, sigma, (4 * q + v) << sh);
        p = child + count_digit(Dg, a, p, v);
        q = 4 * q + v;
    }
    return q;
}

uint64_t oracle_rank_multiary(const uint64_t *digits, const uint64_t *C, uint64_t n, uint64_t sigma, uint64_t c,
                              uint64_t i)
{
    uint32_t Lq = oracle_levels4(sigma);
    uint64_t W4 = (n + 31) / 32, r;
    if (c >= sigma)
        return 0;
    r = i > n ? n : i;
    for (uint32_t j = 0; j < Lq; j++) {
        const uint64_t *Dg = digits + (uint64_t)j * W4;
        uint32_t sh = 2 * (Lq - 1 - j);
        uint64_t a = start_of(C, sigma, (c >> (sh + 2)) << (sh + 2));
        r = count_digit(Dg, a, a + r, digit_at(c, Lq, j));
    }
    return r;
}

int64_t oracle_select_multiary(const uint64_t *digits, const uint64_t *C, uint64_t n, uint64_t sigma, uint64_t c,
                               uint64_t k)
{
    uint32_t Lq = oracle_levels4(sigma);
    uint64_t W4 = (n + 31) / 32, r;
    if (c >= sigma || k == 0 || k > C[c + 1] - C[c])
        return -1;
    r = k - 1;
    for (uint32_t j = Lq; j-- > 0;) {
        const uint64_t *Dg = digits + (uint64_t)j * W4;
        uint32_t sh = 2 * (Lq - 1 - j), v = digit_at(c, Lq, j);
        uint64_t a = start_of(C, sigma, (c >> (sh + 2)) << (sh + 2)), i = a;
        for (uint64_t seen = 0; i < n; i++)
            if (digit_of(Dg, i) == v && seen++ == r)
                break;
        r = i - a;
    }
    return (int64_t)r;
}

/* ---- Huffman-shaped wavelet tree (section "Extensions") ---------------
 * Readings (the paper gives the method, not these details):
 *   - the leaves are the symbols that occur in S (weight = count > 0);
 *   - merge order: repeatedly join the two smallest live nodes under the
 *     total order (weight, leaves before internal nodes, then the symbol
 *     of a leaf or the creation order of an internal node);
 *   - the tree is the canonical tree of the resulting code lengths: codes
 *     assigned in (length, symbol) order, bit 0 = left, so the in-order
 *     leaf order is (length, symbol) and every internal node's left
 *     subtree holds consecutive in-order ids below its right subtree's;
 *   - level d holds, for every occurrence of a symbol whose code is longer
 *     than d, that code's bit d, in the order of S stably sorted by the
 *     code prefix of length d (the internal nodes of depth d, left to
 *     right, each listing its symbols in the order of S);
 *   - one distinct symbol, or n = 0, gives a tree of height 0.
 * Codes are kept left-aligned in 64 bits (bit 63 is code bit 0). */
#define OR_HUFF_MAX_SIGMA 256u

/* The merge order: p before q. */
#if defined(ORACLE_MUTANT) && ORACLE_MUTANT == 9
/* planted mistake: internal nodes before leaves on equal weight */
#define OR_KIND_FIRST(p, q) (kind[p] > kind[q])
#else
#define OR_KIND_FIRST(p, q) (kind[p] < kind[q])
#endif
#define OR_LESS(p, q) (wt[p] != wt[q] ? wt[p] < wt[q] : \
                       kind[p] != kind[q] ? OR_KIND_FIRST(p, q) : id[p] < id[q])

/* Code lengths: len[c] = depth of leaf c (0 for absent symbols, and for the
 * only symbol of a one-leaf tree).  Returns the height. */
uint32_t oracle_huffman_lengths(const uint64_t *w, uint32_t sigma, uint32_t *len)
{
    uint64_t wt[2 * OR_HUFF_MAX_SIGMA];
    uint32_t kind[2 * OR_HUFF_MAX_SIGMA], id[2 * OR_HUFF_MAX_SIGMA], parent[2 * OR_HUFF_MAX_SIGMA];
    int live[2 * OR_HUFF_MAX_SIGMA];
    uint32_t leaf_of[OR_HUFF_MAX_SIGMA];
    uint32_t nn = 0, m = 0;
    for (uint32_t c = 0; c < sigma; c++) {
        len[c] = 0;
        if (w[c]) {
            wt[nn] = w[c]; kind[nn] = 0; id[nn] = c; parent[nn] = UINT32_MAX; live[nn] = 1;
            leaf_of[c] = nn++;
            m++;
        }
    }
    if (m <= 1) return 0;
    for (uint32_t step = 0; step + 1 < m; step++) {
        int32_t a = -1, b = -1;  /* smallest, second smallest */
        for (uint32_t x = 0; x < nn; x++) {
            if (!live[x]) continue;
            if (a < 0 || OR_LESS(x, (uint32_t)a)) { b = a; a = (int32_t)x; }
            else if (b < 0 || OR_LESS(x, (uint32_t)b)) b = (int32_t)x;
        }
        wt[nn] = wt[a] + wt[b]; kind[nn] = 1; id[nn] = step; parent[nn] = UINT32_MAX; live[nn] = 1;
        parent[a] = nn; parent[b] = nn; live[a] = 0; live[b] = 0;
        nn++;
    }
    uint32_t h = 0;
    for (uint32_t c = 0; c < sigma; c++) {
        if (!w[c]) continue;
        uint32_t d = 0;
        for (uint32_t x = leaf_of[c]; parent[x] != UINT32_MAX; x = parent[x]) d++;
        len[c] = d;
        if (d > h) h = d;
    }
    return h;
}

/* Canonical codes from the lengths, left-aligned (0 for absent symbols):
 * in (length, symbol) order, the first code is all zeros and each next one
 * is the previous plus one, shifted left by the growth in length. */
void oracle_huffman_codes(const uint32_t *len, uint32_t sigma, uint64_t *code)
{
    uint64_t cur = 0;
    uint32_t prev = 0;
    int first = 1;
    for (uint32_t c = 0; c < sigma; c++) code[c] = 0;
    for (uint32_t l = 1; l < 64; l++) {
        for (uint32_t c = 0; c < sigma; c++) {
            if (len[c] != l) continue;
            if (first) { cur = 0; first = 0; }
            else cur = (cur + 1) << (l - prev);
            prev = l;
            code[c] = cur << (64 - l);
        }
    }
}

typedef struct { uint64_t key, pos; } or_keyed;
static int or_keyed_cmp(const void *x, const void *y)
{
    const or_keyed *p = (const or_keyed *)x, *q = (const or_keyed *)y;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return p->pos < q->pos ? -1 : (p->pos > q->pos);
}

/* Level bitmaps (h levels of W = ceil(n/64) words, zero past nd[d]) and the
 * level sizes nd[d], straight from the sort view above.  S is bytes. */
int oracle_build_huffman(const uint8_t *S, uint64_t n, uint32_t sigma, const uint32_t *len,
                         const uint64_t *code, uint32_t h, uint64_t *bits, uint64_t *nd)
{
    uint64_t W = (n + 63) / 64;
    for (uint64_t i = 0; i < n; i++)
        if (S[i] >= sigma) return OR_ERR_SYMBOL;
    memset(bits, 0, (size_t)(h * W) * sizeof(uint64_t));
    or_keyed *A = (or_keyed *)malloc((size_t)(n ? n : 1) * sizeof(or_keyed));
    if (!A) return OR_ERR_NOMEM;
    for (uint32_t d = 0; d < h; d++) {
        uint64_t m = 0;
        for (uint64_t i = 0; i < n; i++) {
            uint32_t c = S[i];
            if (len[c] <= d) continue;
            A[m].key = d ? code[c] >> (64 - d) : 0;
            A[m].pos = i;
            m++;
        }
        qsort(A, (size_t)m, sizeof(or_keyed), or_keyed_cmp);
        for (uint64_t p = 0; p < m; p++) {
            uint32_t c = S[A[p].pos];
            if ((code[c] >> (63 - d)) & 1u) set_bit(bits + (uint64_t)d * W, p);
        }
        nd[d] = m;
    }
    free(A);
    return OR_OK;
}
