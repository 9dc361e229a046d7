/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously-correct reference for everything the GPU path
 * computes: a textbook FIFO-queue BFS, the BFS invariant checker, the
 * frontier partitioner, the block codec (stream writer and validating
 * reader), the codec selectors, the selector features and the resolve rules.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header or table with the HIP
 * library; the two meet only in the byte format and the arrays they exchange.
 *
 * Where the paper fixes a definition it is cited by section / equation /
 * algorithm of Romera, "Optimizing Communication by Compression for
 * Multi-GPU Scalable Breadth-First Searches" (arXiv 1704.00513).  The byte
 * format itself is this project's own reading (the paper used third-party
 * codec libraries and prints no format): see the format notes below.
 *
 * Stream format of one segment of n IDs (little-endian 32-bit words).  The
 * form depends on n and the compression threshold T, the least sequence
 * length that is compressed (the "Usage of compression thresholds" section:
 * shorter sequences are sent as they are):
 *   n = 0       empty form: no bytes at all
 *   0 < n < T   raw form: the n IDs, 4 n bytes
 *   n >= T      compressed form:
 *     header    16 B : n, hi, lo, magic 0x31434642
 *     directory 8 B per 128-ID block: first (= v0 - lo), class u8, param u8, aux u16
 *     group tab 4 B per 16 blocks: payload word offset of block 16g
 *     payloads  whole words per block, in block order
 * The reader tells the forms apart by the segment's byte length L and its
 * words 1 and 2: L = 0 is empty; L < 16, or word 1 < word 2 (IDs strictly
 * increase), is raw; word 1 > word 2 (hi > lo in the header) is compressed.
 * It needs no T.  Block classes: 0 = dense bitmap, 1..33 = bit-packed deltas
 * of width class-1, 34 = patched frame of reference (PFOR) with exceptions.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BLK 128u
#define GRP 16u
#define MAGIC 0x31434642u
#define CLS_BITMAP 0
#define CLS_PFOR 34
#define BITMAP_MAX_SPAN 4096u

enum { ST_OK = 0, ST_INVAL = 1, ST_CAPACITY = 2, ST_CORRUPT = 3 };
enum { SEL_PLAIN_BP = 0, SEL_EXHAUSTIVE = 1 };

/* ------------------------------------------------------------------ */
/* BFS                                                                 */
/* ------------------------------------------------------------------ */

/* Textbook breadth-first search from `root` with a FIFO queue (the level
 * structure of the paper's BFS algorithms in the "Our Baseline algorithm"
 * section: each level's frontier is the set of newly reached vertices).
 * level[v] = hop distance or -1; parent[v] = the vertex that first reached
 * v (the root is its own parent), -1 if unreached.  Returns the depth. */
int32_t ref_bfs(uint32_t V, const uint64_t *row_ptr, const uint32_t *col_idx,
                uint32_t root, int32_t *level, int32_t *parent)
{
    for (uint32_t v = 0; v < V; ++v) { level[v] = -1; parent[v] = -1; }
    uint32_t *queue = (uint32_t *)malloc((size_t)V * sizeof(uint32_t));
    if (!queue) return -2;
    uint64_t head = 0, tail = 0;
    level[root] = 0;
    parent[root] = (int32_t)root;
    queue[tail++] = root;
    int32_t depth = 0;
    while (head < tail) {
        uint32_t u = queue[head++];
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint32_t w = col_idx[e];
            if (level[w] == -1) {
                level[w] = level[u] + 1;
                parent[w] = (int32_t)u;
                if (level[w] > depth) depth = level[w];
                queue[tail++] = w;
            }
        }
    }
    free(queue);
    return depth;
}

static int has_arc(const uint64_t *row_ptr, const uint32_t *col_idx, uint32_t u, uint32_t w)
{
    for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
        if (col_idx[e] == w) return 1;
    return 0;
}

/* BFS result checker.  Returns 0 if valid, else the number of the first rule
 * broken:
 *  1 root has level 0 and is its own parent
 *  2 unreached vertices have parent -1
 *  3 a reached non-root vertex's parent is a vertex one level closer
 *  4 the parent arc exists in the graph
 *  5 every arc joins two reached or two unreached vertices, whose levels
 *    differ by at most one.
 * Rules 1, 3 and 5 together force level = hop distance. */
int ref_bfs_check(uint32_t V, const uint64_t *row_ptr, const uint32_t *col_idx,
                  uint32_t root, const int32_t *level, const int32_t *parent)
{
    if (level[root] != 0 || parent[root] != (int32_t)root) return 1;
    for (uint32_t v = 0; v < V; ++v) {
        if (level[v] < 0) {
            if (level[v] != -1 || parent[v] != -1) return 2;
            continue;
        }
        if (v == root) continue;
        int32_t p = parent[v];
        if (p < 0 || (uint32_t)p >= V || level[p] != level[v] - 1) return 3;
        if (!has_arc(row_ptr, col_idx, (uint32_t)p, v)) return 4;
    }
    for (uint32_t u = 0; u < V; ++u) {
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint32_t w = col_idx[e];
            int a = level[u], b = level[w];
            if ((a < 0) != (b < 0)) return 5;
            if (a >= 0 && (a - b > 1 || b - a > 1)) return 5;
        }
    }
    return 0;
}

/* Frontier of level L: all v with level[v] == L, ascending. Returns count. */
uint64_t ref_frontier(uint32_t V, const int32_t *level, int32_t L, uint32_t *out)
{
    uint64_t k = 0;
    for (uint32_t v = 0; v < V; ++v)
        if (level[v] == L) out[k++] = v;
    return k;
}

/* Split a sorted frontier by vertex-ID range: seg_off[r] = number of IDs
 * below bounds[r] (rows of the ALLTOALLV in the paper's BFS-with-compression
 * algorithm go to the rank owning each range). */
void ref_partition(const uint32_t *ids, uint64_t n, const uint32_t *bounds, uint32_t nseg,
                   uint64_t *seg_off)
{
    for (uint32_t r = 0; r <= nseg; ++r) {
        uint64_t k = 0;
        while (k < n && ids[k] < bounds[r]) ++k;
        seg_off[r] = k;
    }
    seg_off[nseg] = n;
}

/* ------------------------------------------------------------------ */
/* Codec arithmetic                                                    */
/* ------------------------------------------------------------------ */

/* Bits needed for x: ceil(log2(x + 1)), the frame-of-reference width of
 * eq. (6) applied to a range [0, x]. */
uint32_t ref_bitlen(uint64_t x)
{
    uint32_t b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

typedef struct {
    uint32_t n;     /* IDs in the block */
    uint32_t m;     /* deltas = n - 1 */
    uint32_t v0;
    uint32_t span;  /* v_last - v0 */
    uint32_t dmin, dmax;
    uint32_t wmin;  /* bitlen(dmax), 0 if m == 0 */
    uint32_t d[BLK];/* d[j] for j = 1..m (d[0] unused) */
} blockinfo;

/* Delta coding ("Delta compression" item of the compression-techniques
 * section): keep the first value, store successive differences. */
static void block_stats(const uint32_t *v, uint32_t n, blockinfo *b)
{
    b->n = n;
    b->m = n - 1;
    b->v0 = v[0];
    b->span = v[n - 1] - v[0];
    b->dmin = 0xFFFFFFFFu;
    b->dmax = 0;
    for (uint32_t j = 1; j < n; ++j) {
        b->d[j] = v[j] - v[j - 1];
        if (b->d[j] < b->dmin) b->dmin = b->d[j];
        if (b->d[j] > b->dmax) b->dmax = b->d[j];
    }
    if (n == 1) b->dmin = 0;
    b->wmin = ref_bitlen(b->dmax);
}

/* Number of deltas that do not fit in b bits (the exceptions of patched
 * coding, eqs. (8)-(9)). */
static uint32_t exceptions(const blockinfo *b, uint32_t bits)
{
    uint32_t e = 0;
    for (uint32_t j = 1; j <= b->m; ++j)
        if (bits < 32 && ((uint64_t)b->d[j] >> bits) != 0) ++e;
    return e;
}

static uint64_t pfor_words(const blockinfo *b, uint32_t bits)
{
    uint32_t E = exceptions(b, bits);
    uint32_t h = E ? b->wmin - bits : 0;
    return ceil_div((uint64_t)b->m * bits, 32) + ceil_div(E, 4) + ceil_div((uint64_t)E * h, 32);
}

/* PFOR exception width: the b in [0, wmin] with 10*E <= m and the fewest
 * payload words; ties go to the larger b.  b = wmin has E = 0, so a choice
 * always exists. */
static uint32_t pfor_best_b(const blockinfo *b)
{
    uint32_t best = b->wmin;
    uint64_t bestw = pfor_words(b, best);
    for (int bits = (int)b->wmin - 1; bits >= 0; --bits) {
        uint32_t E = exceptions(b, (uint32_t)bits);
        if ((uint64_t)10 * E > b->m) continue;
        uint64_t w = pfor_words(b, (uint32_t)bits);
        if (w < bestw) { bestw = w; best = (uint32_t)bits; }
    }
    return best;
}

static int class_valid(const blockinfo *b, uint32_t cls)
{
    if (cls == CLS_BITMAP) return b->span <= BITMAP_MAX_SPAN;
    if (cls >= 1 && cls <= 33) return cls - 1 >= b->wmin;
    return cls == CLS_PFOR;
}

/* Payload words of a block under a class (closed form). */
static uint64_t class_words(const blockinfo *b, uint32_t cls)
{
    if (cls == CLS_BITMAP) return ceil_div(b->span, 32);
    if (cls >= 1 && cls <= 33) return ceil_div((uint64_t)b->m * (cls - 1), 32);
    return pfor_words(b, pfor_best_b(b));
}

/* Exhaustive choice: the fewest payload words among the valid classes;
 * ties prefer bit-packing (smallest width), then bitmap, then PFOR. */
static uint32_t select_exhaustive(const blockinfo *b)
{
    uint32_t best = 0;
    uint64_t bestw = UINT64_MAX;
    for (uint32_t w = 0; w <= 32; ++w) {
        if (!class_valid(b, 1 + w)) continue;
        uint64_t c = class_words(b, 1 + w);
        if (c < bestw) { bestw = c; best = 1 + w; }
    }
    if (class_valid(b, CLS_BITMAP)) {
        uint64_t c = class_words(b, CLS_BITMAP);
        if (c < bestw) { bestw = c; best = CLS_BITMAP; }
    }
    {
        uint64_t c = class_words(b, CLS_PFOR);
        if (c < bestw) { bestw = c; best = CLS_PFOR; }
    }
    return best;
}

static uint32_t select_mode(const blockinfo *b, int mode)
{
    if (mode == SEL_PLAIN_BP) return 1 + b->wmin;
    return select_exhaustive(b);
}

/* ------------------------------------------------------------------ */
/* Bit writer / reader: stream bit i is bit (i mod 32) of word i / 32.   */
/* ------------------------------------------------------------------ */

static void put_bits(uint32_t *words, uint64_t pos, uint32_t nbits, uint64_t value)
{
    for (uint32_t t = 0; t < nbits; ++t) {
        uint64_t bit = pos + t;
        if ((value >> t) & 1u) words[bit / 32] |= 1u << (bit % 32);
    }
}

static uint64_t get_bits(const uint32_t *words, uint64_t pos, uint32_t nbits)
{
    uint64_t v = 0;
    for (uint32_t t = 0; t < nbits; ++t) {
        uint64_t bit = pos + t;
        if ((words[bit / 32] >> (bit % 32)) & 1u) v |= (uint64_t)1 << t;
    }
    return v;
}

/* Writes the payload of one block; returns its word count. */
static uint64_t write_payload(const blockinfo *b, uint32_t cls, uint32_t *out,
                              uint8_t *param, uint16_t *aux)
{
    uint64_t words = class_words(b, cls);
    memset(out, 0, words * 4);
    if (cls == CLS_BITMAP) {
        /* dense bitmap: bit (i-1) set iff v0 + i is in the block */
        uint32_t off = 0;
        for (uint32_t j = 1; j <= b->m; ++j) {
            off += b->d[j];
            put_bits(out, off - 1, 1, 1);
        }
        *param = 0;
        *aux = (uint16_t)b->span;
    } else if (cls <= 33) {
        /* binary packing of the deltas at width w (eq. (7) item) */
        uint32_t w = cls - 1;
        for (uint32_t j = 1; j <= b->m; ++j)
            put_bits(out, (uint64_t)(j - 1) * w, w, b->d[j]);
        *param = (uint8_t)w;
        *aux = 0;
    } else {
        /* patched coding: low b bits of every delta, then exception
         * positions (one byte each), then the high parts at h bits */
        uint32_t bb = pfor_best_b(b);
        uint32_t E = exceptions(b, bb);
        uint32_t h = E ? b->wmin - bb : 0;
        uint64_t lowwords = ceil_div((uint64_t)b->m * bb, 32);
        uint64_t poswords = ceil_div(E, 4);
        uint32_t *pos = out + lowwords;
        uint32_t *high = pos + poswords;
        uint32_t e = 0;
        for (uint32_t j = 1; j <= b->m; ++j) {
            uint64_t d = b->d[j];
            uint64_t low = bb >= 32 ? d : (d & (((uint64_t)1 << bb) - 1));
            put_bits(out, (uint64_t)(j - 1) * bb, bb, low);
            if (bb < 32 && (d >> bb) != 0) {
                put_bits(pos, (uint64_t)e * 8, 8, j - 1);
                put_bits(high, (uint64_t)e * h, h, d >> bb);
                ++e;
            }
        }
        *param = (uint8_t)bb;
        *aux = (uint16_t)(E | (h << 8));
    }
    return words;
}

static void put_u32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static uint32_t get_u32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }

static uint64_t seg_nblocks(uint64_t n) { return ceil_div(n, BLK); }

/* Checks that a segment's IDs are strictly increasing and inside [lo, hi). */
static int seg_ids_ok(const uint32_t *ids, uint64_t n, uint32_t lo, uint32_t hi)
{
    for (uint64_t i = 0; i < n; ++i) {
        if (ids[i] < lo || ids[i] >= hi) return 0;
        if (i && ids[i] <= ids[i - 1]) return 0;
    }
    return 1;
}

/* Upper bound of the encoded size of a batch. */
uint64_t ref_encode_bound(uint64_t n_ids, uint32_t nseg)
{
    uint64_t nb = ceil_div(n_ids, BLK) + nseg;
    return 16ull * nseg + nb * (8 + 512) + 4 * (ceil_div(n_ids, BLK * GRP) + nseg);
}

/* Per-block class choice for a batch (no stream written).
 * mode: 0 = plain bit-packing at the minimal width, 1 = exhaustive. */
int ref_select(const uint32_t *ids, const uint64_t *seg_off, const uint32_t *seg_lo,
               const uint32_t *seg_hi, uint32_t nseg, int mode, uint8_t *classes)
{
    blockinfo *b = (blockinfo *)malloc(sizeof(blockinfo));
    uint64_t k = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        uint64_t n = seg_off[r + 1] - seg_off[r];
        const uint32_t *v = ids + seg_off[r];
        if (!seg_ids_ok(v, n, seg_lo[r], seg_hi[r])) { free(b); return ST_INVAL; }
        for (uint64_t s = 0; s < n; s += BLK) {
            uint32_t nk = (uint32_t)((n - s) < BLK ? (n - s) : BLK);
            block_stats(v + s, nk, b);
            classes[k++] = (uint8_t)select_mode(b, mode);
        }
    }
    free(b);
    return ST_OK;
}

/* Block details for a batch: class, payload words, min width, span, PFOR b
 * and exception count (for tests and reporting).  classes may be NULL
 * (exhaustive choice). */
int ref_block_details(const uint32_t *ids, const uint64_t *seg_off, uint32_t nseg,
                      const uint8_t *classes, uint32_t *words, uint32_t *wmin,
                      uint32_t *span, uint32_t *pfor_b, uint32_t *pfor_e)
{
    blockinfo *b = (blockinfo *)malloc(sizeof(blockinfo));
    uint64_t k = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        uint64_t n = seg_off[r + 1] - seg_off[r];
        const uint32_t *v = ids + seg_off[r];
        for (uint64_t s = 0; s < n; s += BLK) {
            uint32_t nk = (uint32_t)((n - s) < BLK ? (n - s) : BLK);
            block_stats(v + s, nk, b);
            uint32_t cls = classes ? classes[k] : select_exhaustive(b);
            words[k] = class_valid(b, cls) ? (uint32_t)class_words(b, cls) : 0xFFFFFFFFu;
            wmin[k] = b->wmin;
            span[k] = b->span;
            pfor_b[k] = pfor_best_b(b);
            pfor_e[k] = exceptions(b, pfor_b[k]);
            ++k;
        }
    }
    free(b);
    return ST_OK;
}

/* Encodes a batch of segments into one buffer (segments back to back,
 * word aligned).  classes == NULL: choose with `mode`.  seg_byte_off[nseg+1]
 * receives the segment start offsets and the total.  The paper's
 * BFS-with-compression algorithm compresses each outgoing sequence before the
 * exchange; here one segment = one destination's sequence. */
int ref_encode(const uint32_t *ids, const uint64_t *seg_off, const uint32_t *seg_lo,
               const uint32_t *seg_hi, uint32_t nseg, const uint8_t *classes, int mode,
               uint32_t raw_below, uint8_t *out, uint64_t out_cap, uint64_t *seg_byte_off)
{
    blockinfo *b = (blockinfo *)malloc(sizeof(blockinfo));
    uint32_t *payload = (uint32_t *)malloc(BLK * 4 * 2);
    uint64_t pos = 0, k = 0;
    int st = ST_OK;
    for (uint32_t r = 0; r < nseg && st == ST_OK; ++r) {
        uint64_t n = seg_off[r + 1] - seg_off[r];
        const uint32_t *v = ids + seg_off[r];
        uint32_t lo = seg_lo[r], hi = seg_hi[r];
        if (n > 0xFFFFFFFFull || lo > hi || !seg_ids_ok(v, n, lo, hi)) { st = ST_INVAL; break; }
        uint64_t nb = seg_nblocks(n), ng = ceil_div(nb, GRP);
        seg_byte_off[r] = pos;
        if (n == 0) continue;  /* empty form */
        if (n < raw_below) {
            /* raw form: below the threshold the IDs go as they are; their
             * classes (if given) are skipped */
            if (pos + 4 * n > out_cap) { st = ST_CAPACITY; break; }
            for (uint64_t i = 0; i < n; ++i) put_u32(out + pos + 4 * i, v[i]);
            pos += 4 * n;
            k += nb;
            continue;
        }
        uint64_t meta = 16 + 8 * nb + 4 * ng;
        if (pos + meta > out_cap) { st = ST_CAPACITY; break; }
        uint8_t *seg = out + pos;
        put_u32(seg + 0, (uint32_t)n);
        put_u32(seg + 4, hi);
        put_u32(seg + 8, lo);
        put_u32(seg + 12, MAGIC);
        uint64_t pw = 0; /* payload words so far in this segment */
        for (uint64_t blk = 0; blk < nb; ++blk, ++k) {
            uint64_t s = blk * BLK;
            uint32_t nk = (uint32_t)((n - s) < BLK ? (n - s) : BLK);
            block_stats(v + s, nk, b);
            uint32_t cls = classes ? classes[k] : select_mode(b, mode);
            if (cls > 34 || !class_valid(b, cls)) { st = ST_INVAL; break; }
            uint8_t param = 0;
            uint16_t aux = 0;
            uint64_t words = write_payload(b, cls, payload, &param, &aux);
            if (blk % GRP == 0) put_u32(seg + 16 + 8 * nb + 4 * (blk / GRP), (uint32_t)pw);
            if (pos + meta + 4 * (pw + words) > out_cap) { st = ST_CAPACITY; break; }
            uint8_t *de = seg + 16 + 8 * blk;
            put_u32(de, b->v0 - lo);
            de[4] = (uint8_t)cls;
            de[5] = param;
            memcpy(de + 6, &aux, 2);
            memcpy(seg + meta + 4 * pw, payload, words * 4);
            pw += words;
        }
        pos += meta + 4 * pw;
    }
    if (st == ST_OK) seg_byte_off[nseg] = pos;
    free(payload);
    free(b);
    return st;
}

/* Encoded size of a batch from the closed-form size model (no stream):
 * 16 + 8 nb + 4 ceil(nb/16) + 4 sum(words) per compressed segment, 4 n per
 * raw one, 0 per empty one. */
uint64_t ref_encoded_size(const uint32_t *ids, const uint64_t *seg_off, uint32_t nseg,
                          const uint8_t *classes, int mode, uint32_t raw_below)
{
    blockinfo *b = (blockinfo *)malloc(sizeof(blockinfo));
    uint64_t total = 0, k = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        uint64_t n = seg_off[r + 1] - seg_off[r];
        const uint32_t *v = ids + seg_off[r];
        uint64_t nb = seg_nblocks(n);
        if (n == 0) continue;
        if (n < raw_below) { total += 4 * n; k += nb; continue; }
        total += 16 + 8 * nb + 4 * ceil_div(nb, GRP);
        for (uint64_t s = 0; s < n; s += BLK, ++k) {
            uint32_t nk = (uint32_t)((n - s) < BLK ? (n - s) : BLK);
            block_stats(v + s, nk, b);
            uint32_t cls = classes ? classes[k] : select_mode(b, mode);
            total += 4 * class_words(b, cls);
        }
    }
    free(b);
    return total;
}

static uint32_t popcount32(uint32_t x)
{
    uint32_t c = 0;
    while (x) { c += x & 1u; x >>= 1; }
    return c;
}

/* Form of a segment of `bytes` bytes: 0 empty, 1 raw, 2 compressed, -1 neither
 * (see the format notes at the top). */
static int segment_form(const uint8_t *seg, uint64_t bytes)
{
    if (bytes == 0) return 0;
    if (bytes % 4) return -1;
    if (bytes < 16) return 1;
    uint32_t w1 = get_u32(seg + 4), w2 = get_u32(seg + 8);
    if (w1 < w2) return 1;
    if (w1 > w2) return 2;
    return -1;
}

/* Reads a raw segment: its words are the IDs, strictly increasing. */
static int decode_raw(const uint8_t *seg, uint64_t bytes, uint32_t *out, uint64_t *n_out)
{
    uint64_t n = bytes / 4;
    *n_out = n;
    for (uint64_t i = 1; i < n; ++i)
        if (get_u32(seg + 4 * i) <= get_u32(seg + 4 * (i - 1))) return ST_CORRUPT;
    if (out)
        for (uint64_t i = 0; i < n; ++i) out[i] = get_u32(seg + 4 * i);
    return ST_OK;
}

/* Reads one compressed segment; returns ST_OK or ST_CORRUPT.  Values go to
 * out (if not NULL).  *n_out receives the header count. */
static int decode_segment(const uint8_t *seg, uint64_t bytes, uint32_t *out, uint64_t *n_out)
{
    if (bytes < 16) return ST_CORRUPT;
    uint32_t n = get_u32(seg), hi = get_u32(seg + 4), lo = get_u32(seg + 8);
    /* the compressed form is only used for non-empty segments */
    if (get_u32(seg + 12) != MAGIC || lo > hi || n == 0 || n > hi - lo) return ST_CORRUPT;
    *n_out = n;
    uint64_t nb = seg_nblocks(n), ng = ceil_div(nb, GRP);
    uint64_t meta = 16 + 8 * nb + 4 * ng;
    if (meta > bytes) return ST_CORRUPT;
    const uint32_t *words = (const uint32_t *)(seg + meta); /* meta is a multiple of 4 */
    uint64_t avail = (bytes - meta) / 4;
    if ((bytes - meta) % 4) return ST_CORRUPT;
    uint64_t pw = 0;
    uint64_t prev_last = 0;
    for (uint64_t blk = 0; blk < nb; ++blk) {
        if (blk % GRP == 0 && get_u32(seg + 16 + 8 * nb + 4 * (blk / GRP)) != pw) return ST_CORRUPT;
        const uint8_t *de = seg + 16 + 8 * blk;
        uint32_t first = get_u32(de);
        uint32_t cls = de[4], param = de[5];
        uint16_t aux;
        memcpy(&aux, de + 6, 2);
        uint32_t nk = (uint32_t)((n - blk * BLK) < BLK ? (n - blk * BLK) : BLK);
        uint32_t m = nk - 1;
        uint64_t vals[BLK];
        vals[0] = (uint64_t)lo + first;
        uint64_t wc;
        if (cls == CLS_BITMAP) {
            if (param != 0 || aux > BITMAP_MAX_SPAN) return ST_CORRUPT;
            wc = ceil_div(aux, 32);
            if (pw + wc > avail) return ST_CORRUPT;
            const uint32_t *bm = words + pw;
            uint32_t cnt = 0;
            for (uint64_t q = 0; q < wc; ++q) cnt += popcount32(bm[q]);
            if (cnt != m) return ST_CORRUPT;
            if (aux % 32 && (bm[wc - 1] >> (aux % 32)) != 0) return ST_CORRUPT;
            uint32_t j = 1;
            for (uint32_t i = 1; i <= aux; ++i)
                if (get_bits(bm, i - 1, 1)) vals[j++] = vals[0] + i;
        } else if (cls <= 33) {
            uint32_t w = cls - 1;
            if (param != w || aux != 0) return ST_CORRUPT;
            wc = ceil_div((uint64_t)m * w, 32);
            if (pw + wc > avail) return ST_CORRUPT;
            for (uint32_t j = 1; j <= m; ++j)
                vals[j] = vals[j - 1] + get_bits(words + pw, (uint64_t)(j - 1) * w, w);
        } else if (cls == CLS_PFOR) {
            uint32_t bb = param, E = aux & 0xFFu, h = aux >> 8;
            if (bb > 32 || bb + h > 32 || (uint64_t)10 * E > m) return ST_CORRUPT;
            uint64_t lw = ceil_div((uint64_t)m * bb, 32), qw = ceil_div(E, 4);
            wc = lw + qw + ceil_div((uint64_t)E * h, 32);
            /* no block payload is larger than the block's raw 128 words */
            if (wc > BLK || pw + wc > avail) return ST_CORRUPT;
            uint64_t d[BLK];
            for (uint32_t j = 1; j <= m; ++j) d[j] = get_bits(words + pw, (uint64_t)(j - 1) * bb, bb);
            int64_t last = -1;
            for (uint32_t e = 0; e < E; ++e) {
                uint64_t p = get_bits(words + pw + lw, (uint64_t)e * 8, 8);
                if ((int64_t)p <= last || p >= m) return ST_CORRUPT;
                last = (int64_t)p;
                d[p + 1] |= get_bits(words + pw + lw + qw, (uint64_t)e * h, h) << bb;
            }
            for (uint32_t j = 1; j <= m; ++j) vals[j] = vals[j - 1] + d[j];
        } else {
            return ST_CORRUPT;
        }
        for (uint32_t j = 0; j < nk; ++j) {
            if (vals[j] >= hi) return ST_CORRUPT;
            if (j > 0 && vals[j] <= vals[j - 1]) return ST_CORRUPT;
        }
        if (blk > 0 && vals[0] <= prev_last) return ST_CORRUPT;
        prev_last = vals[nk - 1];
        if (out)
            for (uint32_t j = 0; j < nk; ++j) out[blk * BLK + j] = (uint32_t)vals[j];
        pw += wc;
    }
    if (pw != avail) return ST_CORRUPT;
    return ST_OK;
}

/* Reads a batch: out_off[nseg+1] receives output offsets; out_ids the IDs
 * (capacity out_cap IDs).  Returns ST_OK, ST_CORRUPT or ST_CAPACITY. */
int ref_decode(const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
               uint32_t *out_ids, uint64_t out_cap, uint64_t *out_off)
{
    uint64_t acc = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        if (seg_byte_off[r + 1] < seg_byte_off[r]) return ST_CORRUPT;
        uint64_t bytes = seg_byte_off[r + 1] - seg_byte_off[r];
        const uint8_t *seg = in + seg_byte_off[r];
        uint64_t n = 0;
        out_off[r] = acc;
        int form = segment_form(seg, bytes), st = ST_OK;
        if (form < 0) return ST_CORRUPT;
        if (form == 1) {
            if (acc + bytes / 4 > out_cap) return ST_CAPACITY;
            st = decode_raw(seg, bytes, out_ids + acc, &n);
        } else if (form == 2) {
            n = get_u32(seg);
            uint64_t nb = seg_nblocks(n);
            /* a count the segment cannot hold is damage, not a capacity problem */
            if (16 + 8 * nb + 4 * ceil_div(nb, GRP) <= bytes && acc + n > out_cap)
                return ST_CAPACITY;
            st = decode_segment(seg, bytes, out_ids + acc, &n);
        }
        if (st != ST_OK) return st;
        acc += n;
    }
    out_off[nseg] = acc;
    return ST_OK;
}

/* ------------------------------------------------------------------ */
/* Selector features and resolve rules                                 */
/* ------------------------------------------------------------------ */

/* fp32 -> fp16 bit pattern, round to nearest even (IEEE 754 binary16). */
uint16_t ref_f32_to_f16(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    uint32_t sign = (x >> 16) & 0x8000u;
    uint32_t ex = (x >> 23) & 0xFFu;
    uint32_t man = x & 0x7FFFFFu;
    if (ex == 0xFF) return (uint16_t)(sign | 0x7C00u | (man ? 0x200u | (man >> 13) : 0));
    int32_t e = (int32_t)ex - 127 + 15; /* binary16 biased exponent */
    if (e >= 31) return (uint16_t)(sign | 0x7C00u);
    uint32_t full; /* significand with hidden bit, 24 bits */
    int32_t shift;  /* right shift to reach the binary16 field */
    if (e <= 0) {
        if (ex == 0) return (uint16_t)sign; /* fp32 zero / subnormal is far below half's range */
        full = man | 0x800000u;
        shift = 13 + (1 - e);
        if (shift > 24) return (uint16_t)sign;
    } else {
        full = man | 0x800000u;
        shift = 13;
    }
    uint32_t q = full >> shift;
    uint32_t rem = full & ((1u << shift) - 1u);
    uint32_t half = 1u << (shift - 1);
    if (rem > half || (rem == half && (q & 1u))) q += 1;
    uint32_t out;
    if (e <= 0) {
        out = q; /* subnormal (q may carry into the smallest normal) */
    } else {
        /* q includes the hidden bit at position 10 */
        out = ((uint32_t)e << 10) + (q - 0x400u);
        if (q == 0x800u) out = ((uint32_t)(e + 1) << 10); /* carry */
        if (out >= 0x7C00u) out = 0x7C00u;
    }
    return (uint16_t)(sign | out);
}

/* Eight per-block features, as fp16 bit patterns (8 per block):
 *  f0 = n_k/128, f1 = bitlen(min delta)/32, f2 = bitlen(max delta)/32,
 *  f3 = bitlen(floor(span/m))/32, f4 = bitlen(span)/32,
 *  f5 = fp16(fp32(n_k) / fp32(span + 1)), f6 = min(level, 63)/64,
 *  f7 = bitlen(segment length)/32.
 * f1 = f2 = f3 = 0 for one-ID blocks.  seg_level may be NULL (level 0). */
int ref_features(const uint32_t *ids, const uint64_t *seg_off, uint32_t nseg,
                 const int32_t *seg_level, uint16_t *feat)
{
    blockinfo *b = (blockinfo *)malloc(sizeof(blockinfo));
    uint64_t k = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        uint64_t n = seg_off[r + 1] - seg_off[r];
        const uint32_t *v = ids + seg_off[r];
        int32_t L = seg_level ? seg_level[r] : 0;
        if (L < 0) L = 0;
        if (L > 63) L = 63;
        for (uint64_t s = 0; s < n; s += BLK, ++k) {
            uint32_t nk = (uint32_t)((n - s) < BLK ? (n - s) : BLK);
            block_stats(v + s, nk, b);
            float f[8];
            f[0] = (float)nk / 128.0f;
            f[1] = b->m ? (float)ref_bitlen(b->dmin) / 32.0f : 0.0f;
            f[2] = b->m ? (float)b->wmin / 32.0f : 0.0f;
            f[3] = b->m ? (float)ref_bitlen(b->span / b->m) / 32.0f : 0.0f;
            f[4] = (float)ref_bitlen(b->span) / 32.0f;
            f[5] = (float)nk / (float)((uint64_t)b->span + 1u);
            f[6] = (float)L / 64.0f;
            f[7] = (float)ref_bitlen(n) / 32.0f;
            for (int q = 0; q < 8; ++q) feat[k * 8 + q] = ref_f32_to_f16(f[q]);
        }
    }
    free(b);
    return ST_OK;
}

/* Turns a predicted class per block into a valid one.  Bitmap: kept if the
 * block's span allows, else the exhaustive class.  Bit-packing: snap
 * (literal == 0) -> minimal width; literal -> kept if wide enough, else
 * exhaustive.  PFOR: kept.  Classes > 34 -> exhaustive.  Returns the number
 * of blocks that fell back to the exhaustive class. */
uint64_t ref_resolve(const uint32_t *ids, const uint64_t *seg_off, uint32_t nseg,
                     const uint8_t *pred, int literal, uint8_t *out)
{
    blockinfo *b = (blockinfo *)malloc(sizeof(blockinfo));
    uint64_t k = 0, fallbacks = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        uint64_t n = seg_off[r + 1] - seg_off[r];
        const uint32_t *v = ids + seg_off[r];
        for (uint64_t s = 0; s < n; s += BLK, ++k) {
            uint32_t nk = (uint32_t)((n - s) < BLK ? (n - s) : BLK);
            block_stats(v + s, nk, b);
            uint32_t c = pred[k];
            uint32_t res;
            if (c == CLS_BITMAP) {
                res = class_valid(b, c) ? c : 0xFFu;
            } else if (c >= 1 && c <= 33) {
                if (!literal) res = 1 + b->wmin;
                else res = class_valid(b, c) ? c : 0xFFu;
            } else if (c == CLS_PFOR) {
                res = c;
            } else {
                res = 0xFFu;
            }
            if (res == 0xFFu) { res = select_exhaustive(b); ++fallbacks; }
            out[k] = (uint8_t)res;
        }
    }
    free(b);
    return fallbacks;
}
