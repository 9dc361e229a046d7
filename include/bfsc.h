/*
 * bfsc -- lossless compression of BFS frontiers on one MI355X (gfx950).
 *
 * C-ABI of libbfsc.so.  The operations follow the BFS-with-compression
 * algorithm of Romera, "Optimizing Communication by Compression for Multi-GPU
 * Scalable Breadth-First Searches" (arXiv 1704.00513): each BFS level expands
 * the frontier (the SpMV step of the "Our Baseline algorithm" section), the
 * newly reached vertices are split by owning rank (the row exchange,
 * ALLTOALLV), and every outgoing sorted vertex list is compressed before the
 * exchange and decompressed after it ("Communication before and after
 * compression" section and its detailed integration algorithm).  Nothing here
 * sends data between GPUs: one GPU processes its share, segment by segment.
 *
 * Conventions (all entry points):
 *  - Pointers named *_dev or documented as "device" are device memory of the
 *    context's GPU, allocated and owned by the caller.  Host pointers are
 *    documented as such.  The library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call only enqueues work on `stream` and returns; nothing waits for
 *    the GPU except bfsc_sync_status and the functions documented as
 *    synchronous.
 *  - Return value: BFSC_OK, or an error detected on the host before anything
 *    was enqueued (BFSC_E_INVAL for bad arguments, BFSC_E_HIP when a HIP call
 *    fails).  Errors found by kernels (damaged stream, output capacity,
 *    unsorted input) are latched in the context and reported by
 *    bfsc_sync_status; output contents are then unspecified.
 *  - Calls on one context must be serialised by the caller (one stream at a
 *    time).  Workspaces are per call unless documented otherwise.
 *  - Sizes of device arrays that a kernel reads from device memory (frontier
 *    lengths, segment offsets) are never read back by the host, so every
 *    entry point can be captured into a HIP graph.
 *
 * Stream format of one segment of n IDs (little-endian 32-bit words).  Its
 * form depends on n and the context's compression threshold T (the least
 * sequence length that is compressed; shorter ones are sent as they are, the
 * "Usage of compression thresholds" section):
 *   n = 0       empty: no bytes
 *   0 < n < T   raw: the n IDs, 4 n bytes
 *   n >= T      compressed:
 *     header    16 B : n (IDs), hi, lo (the segment's ID range [lo, hi)), magic 0x31434642
 *     directory 8 B per block of 128 IDs: first (= v0 - lo), class u8, param u8, aux u16
 *     group tab 4 B per 16 blocks: payload word offset of block 16g in this segment
 *     payloads  a whole number of words per block, in block order
 * The decoder needs no T: a segment of L bytes is empty if L = 0, raw if
 * L < 16 or its words 1 and 2 increase (strictly increasing IDs), compressed
 * if they decrease (hi > lo).
 * Block classes: 0 = dense bitmap of the span after v0 (param 0, aux = span,
 * span <= 4096); 1..33 = delta bit-packing at width class-1 (param = width,
 * the binary packing of the compression-techniques section, delta coding with
 * eq. (6)/(7) widths); 34 = PFOR, patched coding with exceptions (eqs. (8),
 * (9); param = b, aux = E | h << 8): low b bits of every delta, E exception
 * positions as bytes, then the E high parts at h bits.  Bit i of a packed
 * field stream is bit (i mod 32) of word i/32.  Segments of a batch are
 * concatenated, word aligned; their byte offsets are kept out of band.
 */
#ifndef BFSC_H
#define BFSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfsc_ctx bfsc_ctx;

enum {
    BFSC_OK = 0,
    BFSC_E_INVAL = 1,        /* bad argument, or (from the GPU) unsorted / out-of-range IDs */
    BFSC_E_CAPACITY = 2,     /* output buffer too small */
    BFSC_E_CORRUPT = 3,      /* damaged compressed stream */
    BFSC_E_HIP = 4,          /* a HIP runtime call failed */
    BFSC_E_UNIMPLEMENTED = 5
};

/* Codec choice per block. */
enum {
    BFSC_SEL_DEFAULT = -1,   /* the context's configured choice (bfsc_config.selector) */
    BFSC_SEL_PLAIN_BP = 0,   /* bit-packing at the minimal width (the paper's S4-BP128-like plain method) */
    BFSC_SEL_EXHAUSTIVE = 1, /* fewest payload words among bitmap / all widths / PFOR */
    BFSC_SEL_LEARNED = 2     /* MLP prediction, resolved to a valid class (exhaustive fallback) */
};

/* Operations for bfsc_workspace_size. */
enum {
    BFSC_OP_BFS = 0,
    BFSC_OP_SELECT = 1,
    BFSC_OP_ENCODE = 2,
    BFSC_OP_DECODE = 3,
    BFSC_OP_FEATURES = 4,
    BFSC_OP_MLP = 5,
    BFSC_OP_ENCODE_PLACE = 6, /* timing only: the encoder's placement pass */
    BFSC_OP_PIPELINE = 7,     /* timing only: one bfsc_pipeline_step */
    BFSC_OP_BITMAP_ENCODE = 8,
    BFSC_OP_BITMAP_DECODE = 9
};

/* One GPU's CSR partition: a row range with global column IDs; on one GPU
 * the whole graph (the replicated-CSR layout of the baseline algorithm).
 * row_ptr u64[n_vertices+1] and col_idx u32[n_arcs] are device pointers;
 * each row's neighbours need not be sorted. */
typedef struct {
    uint32_t n_vertices;
    uint64_t n_arcs;
    const uint64_t *row_ptr;
    const uint32_t *col_idx;
} bfsc_csr;

/* A batch of segments to compress (device pointers):
 *   ids       u32[max_ids]     the segments' IDs back to back; each segment
 *                              strictly increasing and inside [seg_lo, seg_hi)
 *   seg_off   u64[nseg+1]      segment r is ids[seg_off[r] .. seg_off[r+1])
 *   seg_lo/hi u32[nseg]        each segment's vertex-ID range (its destination)
 *   seg_level i32[nseg] / NULL BFS level of each segment (a selector feature)
 * max_ids (host value) bounds seg_off[nseg]; it sizes grids and workspaces. */
typedef struct {
    const uint32_t *ids;
    const uint64_t *seg_off;
    const uint32_t *seg_lo;
    const uint32_t *seg_hi;
    const int32_t *seg_level;
    uint32_t nseg;
    uint64_t max_ids;
} bfsc_batch;

/* Adam settings for the selector's training step. */
typedef struct {
    float lr, beta1, beta2, eps;
} bfsc_adam;

/* Launch shapes of the codec kernels (chosen by bfsc_autotune or set). */
typedef struct {
    uint32_t enc_waves;      /* waves per workgroup, encode (1..16) */
    uint32_t enc_wg_per_cu;  /* workgroups per CU for the persistent grid (capped at
                                the kernel's occupancy limit) */
    uint32_t dec_waves;
    uint32_t dec_wg_per_cu;
    uint32_t enc_pack;       /* bit 0: prefix-sum packing instead of LDS atomic ORs;
                                bit 1: IDs loaded block by block instead of a whole unit
                                (8 blocks) staged in LDS at once;
                                bit 2: units taken every NW-th by a wave instead of in one
                                contiguous run per wave */
    uint32_t dec_mode;       /* bit 0: payload loaded block by block instead of a whole
                                unit staged in LDS at once;
                                bit 1: units taken every NW-th instead of in one contiguous
                                run per wave;
                                bit 2: full units decoded one block per 16-lane row, the
                                next unit's payload loaded straight into LDS while the
                                current one decodes (bit 0 is then ignored) */
} bfsc_tune;

/* Context settings, fixed at bfsc_create.
 *   selector        codec choice of calls given BFSC_SEL_DEFAULT (default
 *                   BFSC_SEL_EXHAUSTIVE)
 *   raw_below       compression threshold T: segments of 1 .. T-1 IDs are
 *                   written raw (the "Usage of compression thresholds"
 *                   section: compressing a short sequence costs more than it
 *                   saves).  0 or 1: every non-empty segment is compressed.
 *                   Default 32; at most 2048
 *   resolve_literal how the learned choice turns a predicted bit-pack width
 *                   into a class: 0 (default) the block's minimal width;
 *                   1 the predicted width if it holds the block, else the
 *                   exhaustive class (a diagnostic of the network's widths)
 *   autotune        1: bfsc_create takes the launch shapes stored for this
 *                   device (architecture name and compute-unit count) in the
 *                   file tune_cache, if it has them, and bfsc_autotune
 *                   stores what it measures there; 0: fixed default shapes
 *   tune_cache      path of that text file (NULL: none; copied at create) */
typedef struct {
    int32_t selector;
    uint32_t raw_below;
    uint32_t resolve_literal;
    uint32_t autotune;
    const char *tune_cache;
} bfsc_config;

/* Fills *cfg with the defaults above. */
void bfsc_config_default(bfsc_config *cfg);

/* Creates a context on HIP device `device` with settings cfg (NULL: the
 * defaults): queries the device, allocates the error word and the
 * selector's parameters (device memory owned by the context).  Synchronous.
 * BFSC_E_INVAL for settings out of range.  *out is NULL on failure. */
int bfsc_create(bfsc_ctx **out, int device, const bfsc_config *cfg);
int bfsc_destroy(bfsc_ctx *ctx);
/* The context's settings (tune_cache points at the context's copy). */
int bfsc_get_config(const bfsc_ctx *ctx, bfsc_config *cfg);

/* Bytes of workspace an operation needs for a batch of at most max_ids IDs
 * in nseg segments (BFSC_OP_MLP: max_ids = samples per call; BFSC_OP_BFS is
 * sized by bfsc_bfs_workspace_size instead).  The caller
 * allocates it (any alignment of at least 256 B) and passes it as `ws`. */
int bfsc_workspace_size(const bfsc_ctx *ctx, int op, uint64_t max_ids, uint32_t nseg,
                        size_t *bytes);

/* Bytes of BFS workspace for graph g (visited, next-level and frontier
 * bitmaps, the compaction counters, the queue of high-degree adjacency
 * chunks and the direction state). */
int bfsc_bfs_workspace_size(const bfsc_csr *g, size_t *bytes);

/* Initialises a traversal from `root`: level[] = -1 and parent[] = -1 except
 * level[root] = 0, parent[root] = root; frontier[0] = root and
 * *frontier_len_dev = 1; clears the visited state kept in `ws`.  The same
 * `ws` (bfsc_bfs_workspace_size bytes) must be passed to every bfsc_bfs_level call of the
 * traversal. */
int bfsc_bfs_init(bfsc_ctx *ctx, const bfsc_csr *g, uint32_t root, int32_t *level,
                  int32_t *parent, uint32_t *frontier, uint32_t *frontier_len_dev,
                  void *ws, void *stream);

/* One top-down BFS level (the SpMV step t = A (x) f, then t masked by the
 * visited list, of the baseline algorithm): every unvisited neighbour w of
 * the frontier gets level[w] = cur_level + 1 and a parent u in the frontier
 * with (u, w) an arc (any such u may win).  Writes the new frontier
 * next[0 .. *next_len_dev) sorted ascending (capacity n_vertices).
 * frontier (u32, length *frontier_len_dev on the device) must be the previous
 * level's output. */
int bfsc_bfs_level(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *frontier,
                   const uint32_t *frontier_len_dev, int32_t *level, int32_t *parent,
                   uint32_t *next, uint32_t *next_len_dev, void *ws, void *stream);

/* Direction-optimizing levels (the paper's related work, "Direction
 * optimization": a level may run bottom-up, each unvisited vertex searching
 * its own neighbours for one on the frontier; Beamer, Asanovic & Patterson,
 * SC 2012, for the switching rule).  With m_f the frontier's arcs and m_u the
 * arcs of the unvisited vertices, bfsc_bfs_level runs bottom-up from the
 * first level where m_f > m_u / alpha while the frontier grows, and top-down
 * again once the frontier holds fewer than n_vertices / beta vertices while
 * it shrinks; the choice is made on the device (levels stay capturable).
 * Levels and frontiers are the same as top-down; parents are any frontier
 * neighbour.  alpha = 0 (the default): top-down only.  Set it before
 * bfsc_bfs_init of a traversal.  Returns BFSC_E_INVAL for alpha < 0, or for
 * alpha > 0 with beta <= 0 (Beamer's values: alpha 14, beta 24). */
int bfsc_bfs_set_direction(bfsc_ctx *ctx, float alpha, float beta);

/* Splits a sorted frontier ids[0 .. *n_dev) by destination vertex range:
 * seg_off[r] = number of IDs below bounds[r] for r < nseg, seg_off[nseg] =
 * *n_dev.  bounds u32[nseg+1] non-decreasing.  No data is copied (the row
 * split of the ALLTOALLV exchange).  All pointers device. */
int bfsc_partition(const uint32_t *ids, const uint32_t *n_dev, const uint32_t *bounds,
                   uint32_t nseg, uint64_t *seg_off, void *stream);

/* ---- Candidate exchange (the paper's algorithm "Integration of
 * compression": the candidate vector t = A x f is compressed, sent to its
 * owners by ALLTOALLV and decompressed there, and only then multiplied
 * element-wise by the complement of the visited list), on one GPU.
 *
 * The vertex range [0, n_vertices) is split by bounds u32[nseg+1] (device;
 * bounds[0] = 0, bounds[nseg] = n_vertices, non-decreasing, else the call
 * reports BFSC_E_INVAL through the error word) into nseg owners.  Owner p
 * holds the frontier vertices in [bounds[p], bounds[p+1]); its candidate set
 * T_p is every neighbour of them, visited or not.  T_p restricted to owner
 * d's range is segment p*nseg + d of a batch (sorted, without repeats), so a
 * vertex that several owners reach is sent once by each: the exchanged
 * volume.  Requires nseg <= 65535 and nseg * ceil(n_vertices / 32) below
 * 2^32 - 2^16 (the owners' bitmaps are indexed by 32-bit word numbers): at
 * scale 26 up to 2047 owners.
 *
 * Workspace: bfsc_exchange_workspace_size bytes (nseg + 1 bitmaps of
 * n_vertices bits, a queue of high-degree vertices, counters), caller-owned, cleared once by
 * bfsc_exchange_init before the first bfsc_candidates / bfsc_merge_filter
 * of a traversal; the calls leave it clear again. */
int bfsc_exchange_workspace_size(const bfsc_csr *g, uint32_t nseg, size_t *bytes);
int bfsc_exchange_init(bfsc_ctx *ctx, const bfsc_csr *g, uint32_t nseg, void *ws, void *stream);

/* The senders' side.  frontier u32[*frontier_len_dev] (device, sorted, as
 * bfsc_bfs_level writes it).  Writes the nseg*nseg segments back to back:
 * ids u32[cap] (the candidates; more than cap sets BFSC_E_CAPACITY and the
 * batch keeps the first cap), seg_off u64[nseg*nseg + 1], seg_lo / seg_hi
 * u32[nseg*nseg] (bounds[d], bounds[d+1] of segment p*nseg + d): a batch
 * for bfsc_encode.  All pointers device; asynchronous. */
int bfsc_candidates(bfsc_ctx *ctx, const bfsc_csr *g, const uint32_t *frontier,
                    const uint32_t *frontier_len_dev, const uint32_t *bounds, uint32_t nseg,
                    uint32_t *ids, uint64_t cap, uint64_t *seg_off, uint32_t *seg_lo,
                    uint32_t *seg_hi, void *ws, void *stream);

/* The receivers' side.  ids u32[*n_dev] (device; every owner's decoded
 * segments, as bfsc_decode writes them, in any order, repeats allowed) are
 * merged into one set; the vertices in it that are not yet visited (the
 * visited list of the BFS workspace bfs_ws, as bfsc_bfs_init /
 * bfsc_bfs_level keep it) become visited, get level[w] = cur_level + 1, and
 * form the next frontier next[0 .. *next_len_dev), sorted ascending
 * (capacity n_vertices).  parent[] is not written: the exchanged candidates
 * carry no predecessor.  IDs >= n_vertices are ignored. */
int bfsc_merge_filter(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *ids,
                      const uint64_t *n_dev, int32_t *level, uint32_t *next, uint32_t *next_len_dev,
                      void *bfs_ws, void *ws, void *stream);

/* Chooses a class per block (0 bitmap, 1..33 bit-pack width 0..32, 34 PFOR)
 * for every 128-ID block of every segment, in segment order (raw and empty
 * segments included): classes u8, capacity ceil(max_ids/128) + nseg.  The
 * candidates are the compression techniques' options for a sorted block:
 * delta coding with binary packing at a width of eqs. (6)-(7), patched
 * coding with exceptions (eqs. (8)-(9)), and a bitmap index.  The
 * "Experimental performance comparison" subsection sums up which family
 * suits which data: frame of reference plus delta coding for sequences with
 * small gaps, bitmap indexes for low cardinality (dense sets); this choice
 * is made per block instead of once for all data.
 * BFSC_SEL_PLAIN_BP takes the minimal width (the paper's single fixed
 * codec); BFSC_SEL_EXHAUSTIVE the fewest payload words (ties: bit-pack with
 * the smallest width, then bitmap, then PFOR); BFSC_SEL_LEARNED resolves the
 * MLP's prediction to a valid class (bitmap -> exhaustive if the span is too
 * wide; a width -> the minimal width, or with resolve_literal the predicted
 * width if it holds the block, else exhaustive; PFOR kept); blocks that fell
 * back are counted in *fallbacks_dev (u64, device, may be NULL; added to). */
int bfsc_select(bfsc_ctx *ctx, const bfsc_batch *b, int mode, uint8_t *classes,
                uint64_t *fallbacks_dev, void *ws, void *stream);

/* Upper bound of the compressed size of any batch of n_ids IDs in nseg
 * segments (host arithmetic). */
int bfsc_encode_bound(uint64_t n_ids, uint32_t nseg, size_t *bytes);

/* Compresses a batch (the compress step before each exchange of the
 * BFS-with-compression algorithm).  classes: u8 per block as produced by
 * bfsc_select, or NULL to choose with `mode` inside the encoder; with
 * BFSC_SEL_LEARNED and NULL classes the network runs inside the pack pass
 * (on the matrix cores, per unit of 8 blocks) and the stream equals the one
 * that bfsc_select + bfsc_encode produce (fallbacks are not counted; with
 * resolve_literal the selection runs as a separate pass into the workspace
 * first).  The batch's seg_level is then a feature and must be given.
 * Segments shorter than the context's threshold are written raw, empty ones
 * as no bytes (their classes, if given, are skipped).  Writes the
 * segments back to back into out (capacity out_cap bytes) and
 * seg_byte_off u64[nseg+1] (device): segment r occupies
 * out[seg_byte_off[r] .. seg_byte_off[r+1]).  Overflow latches
 * BFSC_E_CAPACITY; unsorted or out-of-range IDs latch BFSC_E_INVAL. */
int bfsc_encode(bfsc_ctx *ctx, const bfsc_batch *b, const uint8_t *classes, int mode,
                uint8_t *out, size_t out_cap, uint64_t *seg_byte_off, void *ws, void *stream);

/* Decompresses nseg segments (the decompress step after each exchange).
 * in: the compressed bytes; seg_byte_off u64[nseg+1] their boundaries.
 * Writes the IDs back to back into out_ids (capacity out_cap IDs) and
 * out_off u64[nseg+1] (segment r -> out_ids[out_off[r] .. out_off[r+1])).
 * Validates while decoding; a damaged stream latches BFSC_E_CORRUPT and never
 * reads or writes outside the given buffers.  max_ids bounds the total: a
 * stream that holds more IDs than max_ids or out_cap latches
 * BFSC_E_CAPACITY.  The workspace (bfsc_workspace_size with BFSC_OP_DECODE)
 * holds the per-segment plan and the segment of every tile. */
int bfsc_decode(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                uint64_t max_ids, uint32_t *out_ids, uint64_t out_cap, uint64_t *out_off,
                void *ws, void *stream);

/* bfsc_decode without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, output and error
 * behaviour as bfsc_decode.  The decoder's per-segment plan lives in a
 * fixed array of the library (about 0.8 MB per GPU, held until the process
 * ends), so nseg is limited to BFSC_DECODE_NOALLOC_MAX_SEGS (BFSC_E_INVAL
 * beyond it); the per-tile map is not kept there, and each tile's segment
 * is found by search instead.  The call allocates nothing and records no timing events.
 * All calls on one GPU share that array: calls that overlap on one GPU (two
 * streams, or two contexts of the same device) race and must be serialised
 * by the caller. */
#define BFSC_DECODE_NOALLOC_MAX_SEGS 65536u
int bfsc_decode_noalloc(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                        uint64_t max_ids, uint32_t *out_ids, uint64_t out_cap, uint64_t *out_off,
                        void *stream);

/* ---- Bitmap codec: one owner's share of a vertex bitmap (the visited
 * list, or a frontier kept as a bitmap).  The paper leaves the compression
 * of the visited bitmap as future work ("Future work" chapter), after the
 * work of Huiwei et al. that it reviews (related work: the BFS's sparse
 * vectors as bitmaps, compressed with a bitmap index); its guidance on
 * compression techniques names bitmap indexes for low-cardinality data.
 *
 * A batch: bitmap words bits u32 (device), segment r = words
 * [seg_w[r], seg_w[r+1]) (u64[nseg+1], device, non-decreasing,
 * seg_w[nseg] <= max_words, fewer than 2^27 words per segment).  Bit i of a
 * segment is bit (i mod 32) of its word i / 32.  Stream of a segment of nw
 * words (little-endian 32-bit words):
 *   nw = 0      no bytes
 *   otherwise   header 16 B: nw, pop (set bits), nb = ceil(nw / 128), magic 0x31434D42
 *               directory 12 B per block of 128 words: off (payload word
 *                 offset of the block in the segment's payload area),
 *                 count u16 | first u16 << 16, class u8 | width u8 << 8
 *                 (upper 16 bits zero)
 *               payloads, whole words per block, in block order
 * Block classes: 0 ZERO (every bit clear) and 1 ONES (every bit set), no
 * payload; 2 SET / 3 CLEAR: the positions p_0 < ... of the set / clear
 * bits, count of them, first = p_0, the gaps p_j - p_{j-1} bit-packed at
 * width = bitlen(largest gap) (field j-1 at stream bits [(j-1) w, j w),
 * LSB first); 4 LITERAL: the block's words.  The encoder takes ZERO or ONES
 * when they apply, else the fewest payload words among SET, CLEAR, LITERAL
 * (ties in that order).  Segments are back to back, word aligned, their
 * byte offsets out of band (seg_byte_off u64[nseg+1], device).
 * Workspace: bfsc_workspace_size(BFSC_OP_BITMAP_ENCODE / _DECODE, max_words,
 * nseg).  Errors latch as for the frontier codec: bad segments or sizes
 * BFSC_E_INVAL, output overflow BFSC_E_CAPACITY, a damaged stream
 * BFSC_E_CORRUPT (nothing is read or written outside the buffers). */
int bfsc_bitmap_encode_bound(uint64_t n_words, uint32_t nseg, size_t *bytes);
int bfsc_bitmap_encode(bfsc_ctx *ctx, const uint32_t *bits, const uint64_t *seg_w, uint32_t nseg, uint64_t max_words,
                       uint8_t *out, size_t out_cap, uint64_t *seg_byte_off, void *ws, void *stream);
/* Writes segment r's words to out[out_off[r] .. out_off[r+1]) (out_off
 * u64[nseg+1], device; out capacity out_cap words); max_words bounds the
 * total. */
int bfsc_bitmap_decode(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                       uint64_t max_words, uint32_t *out, uint64_t out_cap, uint64_t *out_off, void *ws,
                       void *stream);

/* Selector features: 8 fp16 values per block (bit patterns as u16, row
 * major [block][8]): n/128, bitlen(min delta)/32, bitlen(max delta)/32,
 * bitlen(floor(span/m))/32, bitlen(span)/32, fp16(fp32(n)/fp32(span+1)),
 * min(level,63)/64, bitlen(segment length)/32.  They are the data
 * properties that the "Experimental performance comparison" subsection
 * chooses a codec family by: the size of the gaps (eq. (6)'s width of
 * max - min, here of the deltas), outliers that favour patched coding
 * (eq. (8)), cardinality / density for bitmap indexes, and the length of
 * the sequence; bitlen(x) = ceil(log2(x + 1)) is eq. (6)'s width. */
int bfsc_features(bfsc_ctx *ctx, const bfsc_batch *b, uint16_t *feat, void *ws, void *stream);

/* Selector network 8 -> 64 -> 64 -> 35 (ReLU), fp32 master parameters in the
 * order W1[64][8] b1[64] W2[64][64] b2[64] W3[35][64] b3[35] (7,011 floats).
 * set/get copy host <-> context and are synchronous; set resets Adam state. */
int bfsc_mlp_param_count(void);
/* He-uniform initial parameters: weight i of layer l (0..2) is
 * lim * (2 u - 1) with lim = sqrt(6 / fan_in) and u = (x >> 40) * 2^-24,
 * x = mix(mix(seed + G (100 + l + 1)) + G (i + 1)) (G = 0x9E3779B97F4A7C15,
 * mix the SplitMix64 finaliser of Steele, Lea & Flood, OOPSLA 2014);
 * biases 0.  Resets Adam state.  Synchronous. */
int bfsc_mlp_init(bfsc_ctx *ctx, uint64_t seed);
int bfsc_mlp_set_weights(bfsc_ctx *ctx, const float *host_params);
int bfsc_mlp_get_weights(bfsc_ctx *ctx, float *host_params);

/* Logits f32[n][35] for fp16 features X u16[n][8] (device): weights rounded
 * to fp16, hidden layers fp16(relu(W h + b)), fp32 accumulation. */
int bfsc_mlp_forward(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, void *ws,
                     void *stream);

/* The same network evaluated on the matrix cores (v_mfma_f32_16x16x16_f16,
 * 16 features at a time; fp16 weights and activations, fp32 accumulation and
 * biases): the inference used by the learned selector.  Writes logits
 * f32[n][35] and/or the predicted class u8[n] (largest logit, lowest class
 * on ties, 255 if any logit is NaN); either output may be NULL.  Only the
 * order of the fp32 additions differs from bfsc_mlp_forward.  The selector
 * definition (8 -> 64 ReLU -> 64 ReLU -> 35 over per-block features) follows
 * the learned-codec configuration; the paper's own codec choice was a fixed
 * table ("Compression techniques" section). */
int bfsc_mlp_infer(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, uint8_t *classes,
                   void *stream);

/* Gradient f32[7011] (device) of the mean softmax cross-entropy over
 * (X u16[n][8], y u8[n]), straight-through at the fp16 rounding points;
 * *loss_dev (f32, device, may be NULL) receives the loss. */
int bfsc_mlp_grad(bfsc_ctx *ctx, const uint16_t *X, const uint8_t *y, uint32_t n, float *grads,
                  float *loss_dev, void *ws, void *stream);

/* One Adam step on the context's parameters from the gradient of a batch. */
int bfsc_mlp_train_step(bfsc_ctx *ctx, const uint16_t *X, const uint8_t *y, uint32_t n,
                        const bfsc_adam *opt, float *loss_dev, void *ws, void *stream);

/* Launch shapes: read, set, or measure on a sample batch (synchronous; the
 * sample must be valid input; ws sized for BFSC_OP_ENCODE of the sample). */
int bfsc_get_tune(const bfsc_ctx *ctx, bfsc_tune *out);
int bfsc_set_tune(bfsc_ctx *ctx, const bfsc_tune *t);
int bfsc_autotune(bfsc_ctx *ctx, const bfsc_batch *sample, void *ws, void *stream);

/* Per-kernel timing.  While enabled, every launch of an operation's main
 * kernel (BFSC_OP_ENCODE: the encoder, BFSC_OP_DECODE: the decoder,
 * BFSC_OP_SELECT / BFSC_OP_FEATURES: the selector, BFSC_OP_BFS: the whole
 * level) is bracketed by a HIP event pair on the caller's stream (at most
 * 4096 pairs are kept).  bfsc_timing_read waits for the events of `op`,
 * returns their summed milliseconds and count, and forgets them.  Enabling
 * clears all recorded pairs. */
int bfsc_timing_enable(bfsc_ctx *ctx, int enable);
int bfsc_timing_read(bfsc_ctx *ctx, int op, double *total_ms, uint64_t *count);

/* Per-level pipeline: the level loop of the BFS-with-compression algorithm
 * on one GPU.  One step takes the current frontier F_L, splits it into the
 * nseg destination ranges given by bounds_host (u32[nseg+1], host,
 * non-decreasing), chooses a codec per block with `mode`, encodes, decodes
 * (the exchange itself is left out), and expands F_L into F_{L+1}.  The
 * pipeline owns its device buffers (allocated at create, freed at destroy).
 * use_graph != 0 captures the step into two HIP graphs (even / odd level,
 * ping-pong frontier buffers; the level number lives on the device) that
 * every step replays; use_graph == 0 launches the same kernels one by one.
 * create is synchronous; start and step enqueue on `stream`; step with a
 * non-NULL next_len_host also waits and returns the length of F_{L+1}. */
typedef struct bfsc_pipeline bfsc_pipeline;

/* Device buffers of a pipeline (valid until destroy).  After a step,
 * prev_frontier holds the frontier that step compressed, seg_off its
 * segments, stream / seg_byte_off its compressed form and decoded /
 * decoded_off the decompressed IDs; frontier holds the next frontier. */
typedef struct {
    uint32_t *frontier;
    uint32_t *frontier_len;
    uint32_t *prev_frontier;
    uint32_t *prev_frontier_len;
    int32_t *level;
    int32_t *parent;
    uint64_t *seg_off;
    uint8_t *stream;
    size_t stream_cap;
    uint64_t *seg_byte_off;
    uint32_t *decoded;
    uint64_t *decoded_off;
    uint8_t *classes;
} bfsc_pipeline_bufs;

int bfsc_pipeline_create(bfsc_ctx *ctx, const bfsc_csr *g, const uint32_t *bounds_host, uint32_t nseg,
                         int mode, int use_graph, bfsc_pipeline **out);
int bfsc_pipeline_start(bfsc_pipeline *p, uint32_t root, void *stream);
int bfsc_pipeline_step(bfsc_pipeline *p, void *stream, uint32_t *next_len_host);
int bfsc_pipeline_buffers(const bfsc_pipeline *p, bfsc_pipeline_bufs *bufs);
int bfsc_pipeline_destroy(bfsc_pipeline *p);

/* Synchronous copy of `bytes` between any two pointers the HIP runtime
 * knows (host or device), for reading pipeline buffers. */
int bfsc_memcpy(void *dst, const void *src, size_t bytes);

/* Waits for `stream`, reads and clears the latched kernel error word:
 * returns BFSC_OK or the first error class found (CORRUPT > CAPACITY > INVAL). */
int bfsc_sync_status(bfsc_ctx *ctx, void *stream);

/* Static string for a status code. */
const char *bfsc_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* BFSC_H */
