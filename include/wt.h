/*
 * wt.h -- C ABI of the MI355X (gfx950) wavelet-tree construction library.
 *
 * The library builds the levelwise wavelet tree of Shun, "Parallel Wavelet
 * Tree Construction" (the levelWT algorithm, Fig. 1 of section "Parallel
 * Wavelet Tree Construction"), plus rank/select directories over every level
 * bitmap (section "Parallel Construction of Rank/Select Structures"), and
 * answers access/rank/select queries (defined in section "Preliminaries").
 *
 * Conventions shared by every entry point
 *   - Pointers named d_* are device pointers (HIP device memory).  The caller
 *     owns every buffer; the library never allocates or frees on these paths.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     asynchronous on that stream; argument errors are returned synchronously.
 *   - Return value: WT_OK or a negative wt_status code.  Data errors found
 *     on the device (a symbol >= sigma) are written to a status word in the
 *     scratch buffer and read back with wt_status_get; outputs are then
 *     unspecified.
 *   - Calls on different streams may run concurrently only when they use
 *     disjoint scratch and output buffers.
 *
 * Definitions (L = ceil(log2 sigma), 0 when sigma = 1; k_l = L-1-l)
 *   - The root covers the symbol range [0, 2^L - 1]; a node of range [a, b]
 *     marks a symbol 0 iff it is <= (a+b+1)/2 - 1 (Preliminaries).  Level l
 *     of the levelwise representation is one n-bit bitmap holding the nodes
 *     of depth l in order; equivalently B_l[i] is bit k_l of the i-th symbol
 *     of S stably sorted by its top l bits (sortWT, Fig. 2).
 *   - Bits are LSB-first in 64-bit words: position i is bit i%64 of word
 *     i/64 of its level; padding bits are 0.  Level l occupies words
 *     [l*W, (l+1)*W), W = ceil(n/64).
 *   - Node offsets are exported as C[0..sigma], C[c] = #{i : S[i] < c}.  The
 *     node p of level l (heap id 2^l - 1 + p, as in Fig. 2) covers positions
 *     [C[min(p*2^(L-l), sigma)], C[min((p+1)*2^(L-l), sigma)]) of B_l; it is
 *     empty when that range is.
 */
#ifndef WT_H
#define WT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WT_OK = 0,
    WT_ERR_ARG = -1,     /* invalid argument (null pointer, bad width, sigma out of range, misalignment) */
    WT_ERR_SYMBOL = -2,  /* some S[i] >= sigma (reported by wt_status_get) */
    WT_ERR_SCRATCH = -3, /* scratch buffer smaller than the plan requires */
    WT_ERR_RANGE = -4,   /* size beyond what the library supports */
    WT_ERR_HIP = -5,     /* a HIP call or kernel launch failed */
    WT_ERR_NOMEM = -6,   /* host-side allocation failed */
    WT_ERR_TIMEOUT = -7  /* a batched build gave up waiting for its work items (see wt_tune.spin_limit) */
} wt_status;

/* Directory format constants (a practical reading of Jacobson's rank and
 * Clark's select: absolute counts per 512 bits, a sample per 4096 ones and
 * per 4096 zeros; hardware popcount replaces the lookup tables). */
#define WT_RANK_BLOCK_BITS 512
#define WT_SELECT_SAMPLE 4096

/* Sizes of every buffer, a pure function of (n, sigma, sym_bytes). */
typedef struct {
    uint64_t n, sigma;
    uint32_t L;               /* levels = ceil(log2 sigma) */
    uint32_t sym_bytes;       /* input width: 1, 2 or 4 */
    uint64_t words_per_level; /* W = ceil(n/64) */
    uint64_t bits_words;      /* L*W            -> uint64 bits[L][W]        */
    uint64_t C_len;           /* sigma+1        -> uint64 C[sigma+1]        */
    uint64_t rank_len;        /* ceil(n/512)+1  -> uint64 rank[L][rank_len] */
    uint64_t sel_cap;         /* ceil(n/4096)+1 -> uint64 sel1/sel0[L][sel_cap] */
    uint64_t sel_counts_len;  /* 2L             -> uint64 sel_counts[2L]    */
    uint64_t scratch_bytes;   /* device scratch needed by wt_build          */
    uint64_t rs_scratch_bytes;/* device scratch needed by wt_build_rank_select */
} wt_layout;

/* Output buffers of wt_build (device pointers).  bits and C are required
 * (bits may be NULL when L = 0).  The four directory pointers are either all
 * NULL (no directories) or all non-NULL (directories emitted by the level
 * passes themselves). */
typedef struct {
    uint64_t *bits;       /* [L][W]                                            */
    uint64_t *C;          /* [sigma+1]                                         */
    uint64_t *rank;       /* [L][rank_len]: rank[l][j] = ones of B_l in [0, min(512 j, n)) */
    uint64_t *sel1;       /* [L][sel_cap]: sel1[l][t] = position of the 1 with 0-based ordinal 4096 t;
                             entries t >= sel_counts[l] hold n                 */
    uint64_t *sel0;       /* [L][sel_cap]: the same over the 0s                */
    uint64_t *sel_counts; /* [2L]: ceil(ones_l/4096) for l < L, then ceil(zeros_l/4096) */
} wt_outputs;

/* Fill *out with the sizes for (n, sigma, sym_bytes).
 * Valid: sigma >= 1; sym_bytes in {1, 2, 4}; sigma <= 2^(8*sym_bytes) (so
 * L <= 32); n < 2^40.  Returns WT_ERR_ARG / WT_ERR_RANGE otherwise.
 * The scratch holds node tables for every node of every level (2^(L+1)
 * words) when that is small next to the sequence; for 32-bit alphabets
 * with L > 16 much larger than n, and always for L > 30, it holds tables
 * for the nonempty nodes of one level at a time (at most min(n, sigma)),
 * so it grows with n, not with 2^L.  C is always dense (sigma + 1 words). */
int wt_plan(uint64_t n, uint64_t sigma, int sym_bytes, wt_layout *out);

/* Build the tree of d_seq[0..n) (levelWT, Fig. 1): C, every level bitmap
 * and, when requested, the rank/select directories.
 *   d_seq:   n symbols of sym_bytes each, 16-byte aligned; not modified.
 *   out:     host struct of device output pointers (see wt_outputs).
 *   d_scratch: >= wt_plan().scratch_bytes bytes, 256-byte aligned; its
 *            contents on entry do not matter; it holds the status word
 *            afterwards (see wt_status_get).
 * Asynchronous on `stream`. */
int wt_build(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes,
             const wt_outputs *out, void *d_scratch, uint64_t scratch_bytes, void *stream);

/* Build the rank/select directories of existing level bitmaps
 * d_bits[L][ceil(n/64)] (section "Parallel Construction of Rank/Select
 * Structures": a prefix sum for rank, prefix sum + filter for select).
 * Output layout as in wt_outputs.  d_scratch needs
 * wt_plan().rs_scratch_bytes (or wt_rank_select_scratch_bytes(n, L)). */
int wt_build_rank_select(const uint64_t *d_bits, uint64_t n, uint32_t L,
                         uint64_t *d_rank, uint64_t *d_sel1, uint64_t *d_sel0,
                         uint64_t *d_sel_counts, void *d_scratch, uint64_t scratch_bytes,
                         void *stream);

uint64_t wt_rank_select_scratch_bytes(uint64_t n, uint32_t L);

/* Which histogram wt_build runs for (n, sigma, sym_bytes) under the calling
 * thread's settings (host only; for tests and measurement tools).  Every
 * path gives the same C and outputs; they differ in cost:
 *   WT_HIST_NONE       n = 0
 *   WT_HIST_REPLICAS   sigma <= 8192: per-lane LDS replicas of the counts
 *   WT_HIST_HASH       an LDS hash flushed by global atomics
 *   WT_HIST_SLICES     sigma > 8192: 2^16-symbol slices of 16-bit LDS counters, a row per chunk
 *   WT_HIST_TWO_PHASE  more than 16 levels over 32-bit symbols: groups of the top L-16 bits
 *                      before level 0, the low 16 bits per segment of S_(L-16) later
 *   WT_HIST_LEVELS     byte symbols, no fused levels: no histogram pass; level 0's tile
 *                      counts from one read-only pass, every later level's node sizes
 *                      counted by the level above it while it scatters, C at the last level
 * Returns one of these or WT_ERR_ARG / WT_ERR_RANGE as wt_plan. */
#define WT_HIST_NONE 0
#define WT_HIST_REPLICAS 1
#define WT_HIST_HASH 2
#define WT_HIST_SLICES 3
#define WT_HIST_TWO_PHASE 4
#define WT_HIST_LEVELS 5
int wt_histogram_path(uint64_t n, uint64_t sigma, int sym_bytes);

/* Wait for `stream`, then return WT_OK or the data error recorded by the
 * last wt_build that used d_scratch (WT_ERR_SYMBOL). */
int wt_status_get(const void *d_scratch, void *stream);

/* wt_build without any allocation, for callers that cannot call hipMalloc
 * or an allocating library routine (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The build's scratch is
 * a file-scope device array of WT_NOALLOC_SCRATCH_BYTES that every GPU the
 * library runs on holds until the process ends; the caller still passes the
 * input and the outputs.
 *   Arguments, layout and outputs: as wt_build (no d_scratch).
 *   d_status: device int32 (may be NULL): receives WT_OK or WT_ERR_SYMBOL
 *             once the build has run on `stream` (the data error that
 *             wt_status_get reports for wt_build).
 *   Plans whose wt_plan().scratch_bytes exceed WT_NOALLOC_SCRATCH_BYTES are
 *   refused with WT_ERR_SCRATCH before anything is launched.
 * The array belongs to the calling thread's current device (the device of
 * `stream`).  Every call on one GPU shares that GPU's array, which keeps the
 * previous call's contents (the build clears what must start at zero): calls
 * that overlap on one GPU, on any streams or threads, race and give
 * unspecified outputs.  Asynchronous on `stream`. */
#define WT_NOALLOC_SCRATCH_BYTES (64ull << 20)
int wt_build_noalloc(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                     int32_t *d_status, void *stream);

/* A built tree: device pointers to the outputs of wt_build (with
 * directories) plus its sizes. */
typedef struct {
    const uint64_t *bits, *C, *rank, *sel1, *sel0, *sel_counts;
    uint64_t n, sigma;
    uint32_t L;
} wt_view;

/* Batched queries (Preliminaries), one result per query, m queries.
 * wt_access: d_sym[j] = S[d_i[j]]; d_i[j] >= n gives 0xFFFFFFFF (which is
 *            also a valid symbol when sigma = 2^32: check d_i[j] < n).
 * wt_rank:   d_out[j] = number of c = d_c[j] in S[0, min(d_i[j], n))
 *            (the paper's inclusive rank_c(S, i) is wt_rank(c, i+1));
 *            c >= sigma gives 0.
 * wt_select: d_out[j] = position of the d_k[j]-th (1-based) c = d_c[j] in S,
 *            or -1 when k = 0, c >= sigma or there are fewer than k.
 * Queries never fail asynchronously. */
int wt_access(const wt_view *t, const uint64_t *d_i, uint64_t m, uint32_t *d_sym, void *stream);
int wt_rank(const wt_view *t, const uint32_t *d_c, const uint64_t *d_i, uint64_t m,
            uint64_t *d_out, void *stream);
int wt_select(const wt_view *t, const uint32_t *d_c, const uint64_t *d_k, uint64_t m,
              int64_t *d_out, void *stream);

/* ---------------------------------------------------------------------------
 * Wavelet matrix (the variant described with the paper's extensions to
 * levelWT): one bitmap per level and no nodes.  Level 0 lists S in input
 * order; level l+1 lists level l's symbols with bit L-1-l equal to 0 first
 * and equal to 1 after, each group in its level-l order (a stable split of
 * the whole level).  The bitmap of level l holds bit L-1-l of level l's
 * symbols (LSB-first 64-bit words, levels contiguous, as for the tree), and
 * zeros[l] is its number of 0s.
 *
 * wt_build_matrix takes the arguments of wt_build (the same wt_plan layout
 * and scratch; out->C receives C as well, which the matrix queries do not
 * need) plus d_zeros (device, L uint64; may be NULL only when L = 0).  The
 * directories, when requested, are those of the tree's format over the
 * matrix's bitmaps.  Data errors as for wt_build (wt_status_get). */
int wt_build_matrix(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                    uint64_t *d_zeros, void *d_scratch, uint64_t scratch_bytes, void *stream);

typedef struct {
    const uint64_t *bits, *zeros, *rank, *sel1, *sel0, *sel_counts;  /* device */
    uint64_t n, sigma;
    uint32_t L;
} wt_matrix_view;

/* Queries on a wavelet matrix built with directories; the same conventions
 * as wt_access / wt_rank / wt_select (rank counts [0, i); select is 1-based
 * and gives -1 when there is no such occurrence; access of i >= n gives
 * 0xFFFFFFFF).  A position p of level l continues on level l+1 at the number
 * of 0s before it (bit 0) or at zeros[l] plus the number of 1s before it. */
int wt_matrix_access(const wt_matrix_view *m, const uint64_t *d_i, uint64_t count, uint32_t *d_sym, void *stream);
int wt_matrix_rank(const wt_matrix_view *m, const uint32_t *d_c, const uint64_t *d_i, uint64_t count,
                   uint64_t *d_out, void *stream);
int wt_matrix_select(const wt_matrix_view *m, const uint32_t *d_c, const uint64_t *d_k, uint64_t count,
                     int64_t *d_out, void *stream);

/* ---------------------------------------------------------------------------
 * Multiary wavelet tree with d = 4 (the paper's multiary variant), for byte
 * symbols (sym_bytes = 1, n < 2^32; other inputs give WT_ERR_RANGE).  With
 * L = ceil(log2 sigma) binary levels it has Lq = ceil(L/2) levels; codes are
 * read as Lq base-4 digits (a leading 0 bit when L is odd).  Level j lists S
 * sorted stably by its top j digits and stores the 2-bit digit j of each
 * symbol: entry i is bits 2(i%32), 2(i%32)+1 of word i/32 of
 * digits[j * ceil(n/32) + .] (levels contiguous, padding 0).
 * Directories (the paper defers the structure for larger alphabets to its
 * generalized rank/select; this library keeps, per level):
 *   rank4[(j * R + b) * 4 + v] = occurrences of v among entries [0, min(512 b, n)),
 *                                b = 0 .. R-1, R = ceil(n/512) + 1;
 *   sel4[(j * 4 + v) * cap + t] = position of the occurrence of v with 0-based
 *                                ordinal 4096 t, n past the last, cap = ceil(n/4096) + 1;
 *   counts4[j * 4 + v] = ceil(occurrences of v / 4096).
 * All outputs are caller-owned device buffers, all required (digits may be
 * NULL when n = 0); C as for wt_build.  The scratch is wt_plan's for the same
 * (n, sigma, 1).  Data errors as for wt_build (wt_status_get). */
typedef struct {
    uint64_t *digits;   /* [Lq][ceil(n/32)] */
    uint64_t *C;        /* [sigma+1] */
    uint64_t *rank4;    /* [Lq][R][4] */
    uint64_t *sel4;     /* [Lq][4][cap] */
    uint64_t *counts4;  /* [Lq][4] */
} wt_multiary_outputs;

int wt_build_multiary(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_multiary_outputs *out,
                      void *d_scratch, uint64_t scratch_bytes, void *stream);

typedef struct {
    const uint64_t *digits, *C, *rank4, *sel4, *counts4;  /* device */
    uint64_t n, sigma;
    uint32_t Lq;
} wt_multiary_view;

/* Queries on a 4-ary tree; conventions as for wt_access / wt_rank /
 * wt_select.  Node q of level j holds the symbols whose top j digits are q:
 * it starts at C[q 4^(Lq-j)] and its child v at C[(4q+v) 4^(Lq-j-1)]. */
int wt_multiary_access(const wt_multiary_view *t, const uint64_t *d_i, uint64_t count, uint32_t *d_sym,
                       void *stream);
int wt_multiary_rank(const wt_multiary_view *t, const uint32_t *d_c, const uint64_t *d_i, uint64_t count,
                     uint64_t *d_out, void *stream);
int wt_multiary_select(const wt_multiary_view *t, const uint32_t *d_c, const uint64_t *d_k, uint64_t count,
                       int64_t *d_out, void *stream);

/* ---- sortWT (section "sortWT") ------------------------------------------
 * A second construction of the same tree (the same outputs as wt_build with
 * directories, bit for bit), independent of the level passes: level l is
 * bit L-1-l of S stably sorted by its top l bits, so the levels are built
 * side by side: per level a count of each key per tile, a scan of those
 * counts per key, a stable scatter into a sorted copy of S, and the bits of
 * that copy; then the directories by the standalone builder.  Byte symbols
 * only (sym_bytes 1, n < 2^32, else WT_ERR_RANGE).  The scratch
 * (wt_sort_scratch_bytes; 0 when out of range) holds every sorted copy, L n
 * bytes.  Outputs, errors and wt_status_get as for wt_build. */
uint64_t wt_sort_scratch_bytes(uint64_t n, uint64_t sigma);
int wt_build_sort(const void *d_seq, uint64_t n, uint64_t sigma, int sym_bytes, const wt_outputs *out,
                  void *d_scratch, uint64_t scratch_bytes, void *stream);

/* ---- Huffman-shaped wavelet tree (section "Extensions") ----------------
 * Byte symbols only (sym_bytes 1, sigma <= 256, n < 2^32).  The shape is the
 * canonical tree of the Huffman code lengths of the symbols that occur:
 * the two smallest live nodes are joined first, in the order (weight,
 * leaves before internal nodes, symbol for a leaf / creation order for an
 * internal node); codes are assigned in (length, symbol) order with 0 =
 * left, so the in-order leaf order is (length, symbol).  Level d holds the
 * code bit d of every symbol whose code is longer than d, in the order of S
 * stably sorted by the code prefix of length d; its length is nd[d].  One
 * distinct symbol, or n = 0, gives height 0 (no levels).
 *
 * wt_huffman_plan: the largest height an input of (n, sigma) can have
 * (a leaf at depth d needs at least F(d+2) symbols, F the Fibonacci
 * numbers), the scratch the build needs for a tree of up to h_cap levels
 * (256-byte aligned, reused across builds, the status word first as for
 * wt_build) and the size of the tree's tables (an opaque output the
 * queries read: code, level tables, node starts, child links).
 *
 * wt_build_huffman: asynchronous up to the code construction, then it
 * waits once on `stream` for the height and the level sizes (they size the
 * level passes) and enqueues the rest.  Outputs, caller-owned device
 * buffers with the per-level strides of an n-symbol binary tree
 * (W = ceil(n/64), rank_len and sel_cap as from wt_plan(n, sigma, 1)):
 *   bits[d * W + w]             level d's words, zero past nd[d];
 *   rank/sel1/sel0              as for wt_build_rank_select over level d's
 *                               nd[d] bits (rank entries at or past the
 *                               level's end hold its ones, unused samples
 *                               hold nd[d]);
 *   sel_counts[d], [h + d]      ceil(ones / 4096), ceil(zeros / 4096);
 *   C[sigma + 1]                as for wt_build;
 *   lens[256] (u32), codes[256] code length and left-aligned canonical code
 *                               (bit 63 = code bit 0) per symbol, 0 if absent;
 *   nd[h_cap]                   level sizes;
 *   tables                      tables_bytes, 16-byte aligned, opaque.
 * *h_out (host) receives the height.  Returns WT_ERR_RANGE when the height
 * exceeds h_cap (nothing past the code construction is then enqueued),
 * WT_ERR_RANGE for sym_bytes != 1, sigma > 256 or n >= 2^32, WT_ERR_ARG for
 * missing outputs or misaligned pointers, WT_ERR_SCRATCH for a short
 * scratch.  A symbol >= sigma is reported by wt_status_get; the level passes
 * are then skipped and the outputs are unspecified. */
typedef struct {
    uint64_t *bits;        /* [h_cap][W] */
    uint64_t *C;           /* [sigma+1] */
    uint64_t *rank;        /* [h_cap][rank_len] */
    uint64_t *sel1, *sel0; /* [h_cap][sel_cap] */
    uint64_t *sel_counts;  /* [2 h_cap] */
    uint32_t *lens;        /* [256] */
    uint64_t *codes;       /* [256] */
    uint64_t *nd;          /* [h_cap] */
    void *tables;          /* tables_bytes */
} wt_huffman_outputs;

int wt_huffman_plan(uint64_t n, uint64_t sigma, uint32_t h_cap, uint32_t *h_bound, uint64_t *scratch_bytes,
                    uint64_t *tables_bytes);
int wt_build_huffman(const void *d_seq, uint64_t n, uint64_t sigma, const wt_huffman_outputs *out, uint32_t h_cap,
                     uint32_t *h_out, void *d_scratch, uint64_t scratch_bytes, void *stream);

/* Queries on a Huffman-shaped tree; conventions as for wt_access / wt_rank
 * / wt_select (a symbol that does not occur has rank 0 and select -1).  A
 * query walks the code of its symbol (access: the bits it reads) from the
 * root: at depth d, node q starts at the node start the tables hold, the
 * position inside it comes from rank on level d's nd[d] bits, and the child
 * link gives the next node or the leaf.  The view holds the build's
 * device outputs and h (0 for a tree of one symbol or none). */
typedef struct {
    const uint64_t *bits, *rank, *sel1, *sel0;  /* device, strides as in wt_huffman_outputs */
    const void *tables;                          /* device */
    uint64_t n, sigma;
    uint32_t h;
} wt_huffman_view;

int wt_huffman_access(const wt_huffman_view *t, const uint64_t *d_i, uint64_t count, uint32_t *d_sym, void *stream);
int wt_huffman_rank(const wt_huffman_view *t, const uint32_t *d_c, const uint64_t *d_i, uint64_t count,
                    uint64_t *d_out, void *stream);
int wt_huffman_select(const wt_huffman_view *t, const uint32_t *d_c, const uint64_t *d_k, uint64_t count,
                      int64_t *d_out, void *stream);

/* ---------------------------------------------------------------------------
 * Batched construction: many sequences of uneven length and alphabet, each
 * built exactly as wt_build builds it (levelWT, Fig. 1), by one kernel that
 * takes work items from a per-level queue: histogram tiles of every job,
 * then each job's tables, then level 0 tiles of every job, level 1 tiles,
 * and so on.  A level's tiles start once that job's previous level is done.
 * The outputs of every job are identical to wt_build's for the same input.
 *
 * Use: wt_batch_plan (host only: sizes), allocate the scratch, then
 * wt_batch_prepare once (uploads the job and queue tables, synchronous), then
 * wt_batch_run as often as wanted (kernel launches only, no host work or
 * allocation: capturable in a HIP graph), then wt_batch_status.  A run
 * rebuilds every job from the current contents of its input. */

/* One sequence of a batch.  The output buffers are sized as wt_plan gives
 * for (n, sigma, sym_bytes); directories are required (all four pointers)
 * when L > 0. */
typedef struct {
    const void *seq;     /* device, n symbols of sym_bytes each, 16-byte aligned */
    uint64_t n;          /* < 2^32 */
    uint64_t sigma;      /* as for wt_build */
    uint32_t sym_bytes;  /* 1, 2 or 4 */
    uint32_t reserved;   /* 0 */
    wt_outputs out;
} wt_job;

#define WT_BATCH_PERSISTENT 0u /* one launch of the work kernel for the whole queue */
#define WT_BATCH_PER_PHASE 1u  /* one launch per phase (histograms, tables, level 0, 1, ...) */

/* Launch tunables of wt_batch_run; a zero field takes the default. */
typedef struct {
    uint32_t mode;          /* WT_BATCH_PERSISTENT (default) or WT_BATCH_PER_PHASE */
    uint32_t blocks_per_cu; /* resident work-kernel blocks per CU (default: as many as fit) */
    uint32_t chunk;         /* consecutive work items taken per queue access (default 1, at most 4096) */
    uint32_t spin_limit;    /* polls before a waiting block gives up (default 2^22, roughly seconds);
                               a give-up marks the job WT_ERR_TIMEOUT and leaves its outputs unspecified */
} wt_tune;

/* Sizes and queue shape of a batch: a pure function of the jobs' (n, sigma,
 * sym_bytes), in the given order. */
typedef struct {
    uint64_t scratch_bytes;   /* device scratch of wt_batch_prepare / wt_batch_run (256-byte aligned) */
    uint64_t clear_bytes;     /* leading scratch bytes every run clears */
    uint64_t off_jobs, off_segs, off_seg_of; /* offsets of the tables wt_batch_prepare writes */
    uint64_t off_list;        /* lists of live items that per-phase runs build on the device */
    uint32_t njobs;
    uint32_t nsegs;           /* queue segments: (job, phase) pairs with work */
    uint32_t items;           /* work items in the queue */
    uint32_t phases;          /* tile histograms, whole-job histograms, tables, then per level of the
                                 deepest job byte-symbol and wider tiles, then fused tail levels */
    uint32_t phase_first[72]; /* first item of each phase; phase_first[phases] = items */
    uint32_t phase_var[72];   /* level phases: the one tile variant of their items, 0 when mixed */
} wt_batch_layout;

/* Host only.  WT_ERR_ARG / WT_ERR_RANGE as wt_plan (and n >= 2^32). */
int wt_batch_plan(const wt_job *jobs, uint32_t njobs, wt_batch_layout *out);

/* Writes the job and queue tables into d_scratch (>= scratch_bytes, 256-byte
 * aligned) and waits for the copies.  `lay` must come from wt_batch_plan on
 * the same jobs.  The jobs' input and output pointers are recorded: they
 * must stay valid for every later wt_batch_run. */
int wt_batch_prepare(const wt_job *jobs, uint32_t njobs, const wt_batch_layout *lay, void *d_scratch,
                     uint64_t scratch_bytes, void *stream);

/* Builds every job (asynchronous on `stream`; tune may be NULL). */
int wt_batch_run(const wt_batch_layout *lay, const wt_tune *tune, void *d_scratch, void *stream);

/* Waits for `stream`; writes each job's code (WT_OK, WT_ERR_SYMBOL,
 * WT_ERR_TIMEOUT) to codes[0..njobs) when codes is not NULL and returns
 * WT_ERR_TIMEOUT if any job timed out, else the first error, else WT_OK. */
int wt_batch_status(const wt_batch_layout *lay, const void *d_scratch, int32_t *codes, void *stream);

/* Mixed queries over many built trees in one launch (the serving path:
 * a batch of queries spread over the resident trees).
 *   d_views: device array of ntrees wt_view (each as for wt_access).
 *   query j: tree d_tree[j], kind d_kind[j], arguments (d_a[j], d_b[j]):
 *     WT_Q_ACCESS  a = i            -> S[i], or 0xFFFFFFFF when i >= n
 *     WT_Q_RANK    a = c, b = i     -> occurrences of c in S[0, min(i, n)); 0 when c >= sigma
 *     WT_Q_SELECT  a = c, b = k     -> position of the k-th (1-based) c, or -1
 *   d_out[j] (int64): the answer, or WT_Q_BAD for a tree index >= ntrees, a
 *   view without C, or an unknown kind. */
#define WT_Q_ACCESS 0
#define WT_Q_RANK 1
#define WT_Q_SELECT 2
#define WT_Q_BAD (-2)
int wt_query_multi(const wt_view *d_views, uint32_t ntrees, const uint32_t *d_tree, const uint8_t *d_kind,
                   const uint64_t *d_a, const uint64_t *d_b, uint64_t m, int64_t *d_out, void *stream);

/* The wt_set_* settings below are per host thread: each applies to the later
 * launches made from the thread that set it, and other threads keep their
 * own values (defaults as stated). */

/* Fused tail levels (levels = 1 by default).  Once every node of a level
 * fits one block's segment, wt_build and wt_batch_run run that level and all
 * deeper ones on chip, one node-aligned segment per block (no sequence
 * traffic for those levels); outputs are identical whatever the setting.
 *   0       no fused levels;
 *   1       from the first level whose nodes fit;
 *   m >= 2  at most the last m levels (from level max(first fitting, L - m)).
 * WT_ERR_ARG for a negative value. */
int wt_set_fused_levels(int levels);

/* Wide-alphabet histogram (on by default).  For sigma > 8192, wt_build counts
 * symbols in 2^16-symbol slices of packed 16-bit LDS counters, one row of
 * counts per input chunk, summed by a second kernel (the rows use the
 * sequence ping-pong of the scratch, idle at that point).  Trees of more
 * than 16 levels over 32-bit symbols (2^20 <= n < 2^32) count in two
 * phases instead: the groups of the top L-16 bits before level 0 (all that
 * the levels above L-16 need), then, once S_{L-16} holds each group as a
 * contiguous segment, the low 16 bits segment by segment.  Inputs too short
 * for either use per-block LDS hashing with global atomics.  C and every
 * output are the same on all paths.  0 selects the hashing path for later
 * launches (for comparisons). */
int wt_set_sliced_histogram(int enable);

/* Two levels per pass (off by default).  When on, for byte symbols
 * (sym_bytes = 1, sigma <= 256) with n < 2^32 and no fused levels, wt_build
 * runs levels l and l+1 in one pass over S_l: both bit levels, both levels'
 * directory entries and S_{l+2} (a stable split of every node by two bits at
 * once; see the levelWT construction, Fig. 1, and the sortWT view of its
 * levels).  It halves the sequence traffic, but on gfx950 the byte level pass
 * is bound by its ALU and LDS work rather than by HBM, and the two splits of
 * a pair cost more than two single passes, so one level per pass is the
 * default.  Outputs are identical either way.  Returns the previous setting
 * (0 or 1); applies to later launches. */
int wt_set_level_pairs(int enable);

/* Look-back tuning and testing hook.  Tiles of a level pass find their
 * prefix by looking back at earlier tiles; a tile whose predecessor has not
 * published after `polls` polls reduces that predecessor's input itself
 * (results are identical either way).  0 forces that path for every
 * predecessor found unpublished.  Default 8.  Applies to later launches. */
int wt_set_lookback_spin_limit(int polls);

/* Kernel timing for measurement tools.  While enabled, every level-pass
 * launch of wt_build (and of the matrix and Huffman builds) carries a start
 * and a stop HIP event in its own dispatch on its stream (hipExtLaunchKernel),
 * so each pair times that kernel.
 * wt_timing_collect waits for the recorded events, writes up to `cap`
 * durations in milliseconds (launch order) and returns how many launches
 * were recorded since the previous collect (or a negative wt_status). */
int wt_timing_enable(int enable);
int wt_timing_collect(float *ms, int cap);

#ifdef __cplusplus
}
#endif

#endif /* WT_H */
