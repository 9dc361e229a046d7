/*
 * CPU ORACLE -- test infrastructure only (built into liboracle.so beside
 * oracle.c; shares nothing with the HIP library).
 *
 * Codec for one owner's share of a vertex bitmap (the visited list, or a
 * frontier kept as a bitmap).  The paper leaves it as future work: compress
 * the visited-neighbourhood bitmap, after the work of Huiwei et al. that it
 * reviews (related work: sparse vectors treated as bitmaps and compressed
 * with a bitmap-index codec, WAH), and its compression-techniques guidance
 * names bitmap indexes for low-cardinality data.  It prints no format; the
 * one below is this project's own, written block by block so that every
 * block is coded and decoded on its own.
 *
 * A batch: bitmap words `bits`, segment r = words [seg_w[r], seg_w[r+1]).
 * Stream of one segment of nw words (little-endian 32-bit words):
 *   nw = 0      no bytes
 *   otherwise   header 16 B : nw, pop (set bits of the segment), nb, magic 0x31434D42
 *               directory 12 B per block: off (payload word offset of the
 *                 block in the segment's payload area), count u16,
 *                 first u16, class u8, width u8, reserved u16 = 0
 *               payloads, a whole number of words per block, in block order
 * Block k holds words [128 k, min(128 k + 128, nw)): nbits = 32 x its words;
 * bit i of a block is bit (i mod 32) of its word i / 32.
 * Classes (count / first / width are 0 unless stated):
 *   0 ZERO     every bit clear; no payload
 *   1 ONES     every bit set; no payload
 *   2 SET      the positions p_0 < ... < p_{c-1} of the set bits (c = count
 *              >= 1, first = p_0): the c - 1 gaps p_j - p_{j-1} packed at
 *              `width` = bitlen(largest gap) bits each (0 when c = 1),
 *              field j - 1 at stream bits [(j-1) w, j w), LSB first
 *   3 CLEAR    the same list for the clear bits
 *   4 LITERAL  the block's words as they are
 * Choice: ZERO or ONES when they apply, else the fewest payload words among
 * SET, CLEAR and LITERAL, ties in that order.
 */
#include <stdint.h>
#include <string.h>

#define BMC_BLOCK_WORDS 128u
#define BMC_MAGIC 0x31434D42u
#define BMC_DIR_BYTES 12u

enum { BMC_ZERO = 0, BMC_ONES = 1, BMC_SET = 2, BMC_CLEAR = 3, BMC_LITERAL = 4 };
enum { BST_OK = 0, BST_INVAL = 1, BST_CAPACITY = 2, BST_CORRUPT = 3 };

static uint64_t bdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

static uint32_t blen(uint64_t x)
{
    uint32_t n = 0;
    while (x) { ++n; x >>= 1; }
    return n;
}

static int bit_of(const uint32_t *w, uint32_t i) { return (int)((w[i / 32] >> (i % 32)) & 1u); }

static void put32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static uint32_t get32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static void put16(uint8_t *p, uint16_t v) { memcpy(p, &v, 2); }
static uint16_t get16(const uint8_t *p) { uint16_t v; memcpy(&v, p, 2); return v; }

/* The list of positions whose bit equals `want`, the first of them and the
 * width of their gaps. */
typedef struct {
    uint32_t count, first, width;
} bmc_list;

static bmc_list list_of(const uint32_t *w, uint32_t nbits, int want)
{
    bmc_list L = {0, 0, 0};
    uint32_t prev = 0, gmax = 0;
    for (uint32_t i = 0; i < nbits; ++i) {
        if (bit_of(w, i) != want) continue;
        if (L.count == 0) L.first = i;
        else if (i - prev > gmax) gmax = i - prev;
        prev = i;
        ++L.count;
    }
    L.width = blen(gmax);
    return L;
}

static uint64_t list_words(bmc_list L)
{
    return L.count ? bdiv((uint64_t)(L.count - 1) * L.width, 32) : 0;
}

/* The class of a block of nw32 words and its directory fields. */
typedef struct {
    uint32_t cls, count, first, width, words;
} bmc_block;

static bmc_block choose_block(const uint32_t *w, uint32_t nw32)
{
    const uint32_t nbits = 32 * nw32;
    bmc_list S = list_of(w, nbits, 1), C = list_of(w, nbits, 0);
    bmc_block b = {BMC_LITERAL, 0, 0, 0, nw32};
    if (S.count == 0) { b.cls = BMC_ZERO; b.words = 0; return b; }
    if (C.count == 0) { b.cls = BMC_ONES; b.words = 0; return b; }
    uint64_t ws = list_words(S), wc = list_words(C);
    /* ties: SET, then CLEAR, then LITERAL */
    if (ws <= wc && ws <= nw32) {
        b.cls = BMC_SET; b.count = S.count; b.first = S.first; b.width = S.width; b.words = (uint32_t)ws;
    } else if (wc <= nw32) {
        b.cls = BMC_CLEAR; b.count = C.count; b.first = C.first; b.width = C.width; b.words = (uint32_t)wc;
    }
    return b;
}

static void put_field(uint32_t *out, uint64_t pos, uint32_t nb, uint32_t v)
{
    for (uint32_t k = 0; k < nb; ++k)
        if ((v >> k) & 1u) out[(pos + k) / 32] |= 1u << ((pos + k) % 32);
}

static uint32_t get_field(const uint32_t *in, uint64_t pos, uint32_t nb)
{
    uint32_t v = 0;
    for (uint32_t k = 0; k < nb; ++k)
        v |= (uint32_t)((in[(pos + k) / 32] >> ((pos + k) % 32)) & 1u) << k;
    return v;
}

/* Writes block b's payload (b.words words, zeroed first). */
static void write_block(const uint32_t *w, uint32_t nw32, bmc_block b, uint32_t *pay)
{
    memset(pay, 0, (size_t)b.words * 4);
    if (b.cls == BMC_LITERAL) {
        memcpy(pay, w, (size_t)nw32 * 4);
        return;
    }
    if (b.cls != BMC_SET && b.cls != BMC_CLEAR) return;
    const int want = b.cls == BMC_SET ? 1 : 0;
    uint32_t j = 0, prev = 0;
    for (uint32_t i = 0; i < 32 * nw32; ++i) {
        if (bit_of(w, i) != want) continue;
        if (j > 0) put_field(pay, (uint64_t)(j - 1) * b.width, b.width, i - prev);
        prev = i;
        ++j;
    }
}

uint64_t ref_bmc_bound(uint64_t n_words, uint32_t nseg)
{
    /* header and directory of every segment, literal payloads at most */
    return 16ull * nseg + BMC_DIR_BYTES * (bdiv(n_words, BMC_BLOCK_WORDS) + nseg) + 4ull * n_words;
}

/* Block classes of a batch (class per block, segment order); returns the
 * number of blocks written to cls. */
uint64_t ref_bmc_classes(const uint32_t *bits, const uint64_t *seg_w, uint32_t nseg, uint8_t *cls)
{
    uint64_t k = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        uint64_t nw = seg_w[r + 1] - seg_w[r];
        for (uint64_t q = 0; q < nw; q += BMC_BLOCK_WORDS) {
            uint32_t n32 = (uint32_t)(nw - q < BMC_BLOCK_WORDS ? nw - q : BMC_BLOCK_WORDS);
            cls[k++] = (uint8_t)choose_block(bits + seg_w[r] + q, n32).cls;
        }
    }
    return k;
}

int ref_bmc_encode(const uint32_t *bits, const uint64_t *seg_w, uint32_t nseg, uint8_t *out, uint64_t cap,
                   uint64_t *seg_byte_off)
{
    uint64_t at = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        if (seg_w[r + 1] < seg_w[r]) return BST_INVAL;
        uint64_t nw = seg_w[r + 1] - seg_w[r];
        seg_byte_off[r] = at;
        if (nw == 0) continue;
        if (nw > 0xFFFFFFFFull) return BST_INVAL;
        const uint32_t *w = bits + seg_w[r];
        uint64_t nb = bdiv(nw, BMC_BLOCK_WORDS), pop = 0;
        for (uint64_t i = 0; i < nw; ++i)
            for (uint32_t k = 0; k < 32; ++k) pop += (w[i] >> k) & 1u;
        uint64_t meta = 16 + BMC_DIR_BYTES * nb;
        if (at + meta > cap) return BST_CAPACITY;
        uint8_t *seg = out + at;
        put32(seg, (uint32_t)nw);
        put32(seg + 4, (uint32_t)pop);
        put32(seg + 8, (uint32_t)nb);
        put32(seg + 12, BMC_MAGIC);
        uint64_t pw = 0;
        for (uint64_t k = 0; k < nb; ++k) {
            uint32_t n32 = (uint32_t)(nw - k * BMC_BLOCK_WORDS < BMC_BLOCK_WORDS ? nw - k * BMC_BLOCK_WORDS
                                                                                : BMC_BLOCK_WORDS);
            bmc_block b = choose_block(w + k * BMC_BLOCK_WORDS, n32);
            uint8_t *de = seg + 16 + BMC_DIR_BYTES * k;
            put32(de, (uint32_t)pw);
            put16(de + 4, (uint16_t)b.count);
            put16(de + 6, (uint16_t)b.first);
            de[8] = (uint8_t)b.cls;
            de[9] = (uint8_t)b.width;
            put16(de + 10, 0);
            if (at + meta + 4 * (pw + b.words) > cap) return BST_CAPACITY;
            uint32_t pay[BMC_BLOCK_WORDS];
            write_block(w + k * BMC_BLOCK_WORDS, n32, b, pay);
            memcpy(seg + meta + 4 * pw, pay, (size_t)b.words * 4);
            pw += b.words;
        }
        at += meta + 4 * pw;
    }
    seg_byte_off[nseg] = at;
    return BST_OK;
}

/* Reads one segment (bytes > 0) into out (nw words); checks everything the
 * format fixes.  *nw_out: the header's word count. */
static int decode_bmc_segment(const uint8_t *seg, uint64_t bytes, uint32_t *out, uint64_t out_room,
                              uint64_t *nw_out)
{
    if (bytes < 16 || bytes % 4) return BST_CORRUPT;
    uint32_t nw = get32(seg), pop = get32(seg + 4), nb = get32(seg + 8);
    if (get32(seg + 12) != BMC_MAGIC || nw == 0 || nb != bdiv(nw, BMC_BLOCK_WORDS)) return BST_CORRUPT;
    uint64_t meta = 16 + (uint64_t)BMC_DIR_BYTES * nb;
    if (meta > bytes) return BST_CORRUPT;
    *nw_out = nw;
    if (nw > out_room) return BST_CAPACITY;
    const uint32_t *pay = (const uint32_t *)(seg + meta);
    uint64_t avail = (bytes - meta) / 4, pw = 0, seen = 0;
    for (uint32_t k = 0; k < nb; ++k) {
        const uint8_t *de = seg + 16 + BMC_DIR_BYTES * k;
        uint32_t off = get32(de), count = get16(de + 4), first = get16(de + 6);
        uint32_t cls = de[8], width = de[9];
        if (get16(de + 10) != 0 || off != pw) return BST_CORRUPT;
        uint32_t n32 = nw - k * BMC_BLOCK_WORDS < BMC_BLOCK_WORDS ? nw - k * BMC_BLOCK_WORDS : BMC_BLOCK_WORDS;
        uint32_t nbits = 32 * n32;
        uint32_t *w = out + (uint64_t)k * BMC_BLOCK_WORDS;
        uint64_t words;
        if (cls == BMC_ZERO || cls == BMC_ONES || cls == BMC_LITERAL) {
            if (count || first || width) return BST_CORRUPT;
            words = cls == BMC_LITERAL ? n32 : 0;
            if (pw + words > avail) return BST_CORRUPT;
            for (uint32_t i = 0; i < n32; ++i)
                w[i] = cls == BMC_ZERO ? 0u : cls == BMC_ONES ? 0xFFFFFFFFu : pay[pw + i];
        } else if (cls == BMC_SET || cls == BMC_CLEAR) {
            if (count == 0 || count > nbits || width > 32 || first >= nbits) return BST_CORRUPT;
            words = bdiv((uint64_t)(count - 1) * width, 32);
            if (words > n32 || pw + words > avail) return BST_CORRUPT;
            const uint32_t fill = cls == BMC_SET ? 0u : 0xFFFFFFFFu;
            for (uint32_t i = 0; i < n32; ++i) w[i] = fill;
            uint64_t p = first;
            for (uint32_t j = 0; j < count; ++j) {
                if (j > 0) {
                    uint32_t d = get_field(pay + pw, (uint64_t)(j - 1) * width, width);
                    if (d == 0) return BST_CORRUPT;
                    p += d;
                }
                if (p >= nbits) return BST_CORRUPT;
                w[p / 32] ^= 1u << (p % 32);
            }
        } else {
            return BST_CORRUPT;
        }
        for (uint32_t i = 0; i < n32; ++i)
            for (uint32_t b = 0; b < 32; ++b) seen += (w[i] >> b) & 1u;
        pw += words;
    }
    if (pw != avail || seen != pop) return BST_CORRUPT;
    return BST_OK;
}

int ref_bmc_decode(const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg, uint32_t *out,
                   uint64_t out_cap, uint64_t *out_off)
{
    uint64_t acc = 0;
    for (uint32_t r = 0; r < nseg; ++r) {
        if (seg_byte_off[r + 1] < seg_byte_off[r]) return BST_CORRUPT;
        uint64_t bytes = seg_byte_off[r + 1] - seg_byte_off[r];
        out_off[r] = acc;
        if (bytes == 0) continue;
        uint64_t nw = 0;
        int st = decode_bmc_segment(in + seg_byte_off[r], bytes, out + acc, out_cap - acc, &nw);
        if (st != BST_OK) return st;
        acc += nw;
    }
    out_off[nseg] = acc;
    return BST_OK;
}
