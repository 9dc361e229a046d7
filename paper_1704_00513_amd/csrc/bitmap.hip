// Codec for one owner's share of a vertex bitmap: the visited list, or a
// frontier kept as a bitmap.  The paper leaves this as future work, after the
// work of Huiwei et al. it reviews (related work: the sparse vectors of a BFS
// treated as bitmaps and compressed with a bitmap index, WAH), and its
// guidance on compression techniques names bitmap indexes for
// low-cardinality data.  The format is this project's own, block by block
// (128 words, 4096 bits) so that one wave codes one block with no scan over
// the segment: ZERO and ONES blocks cost only their directory entry, sparse
// blocks carry the gaps between their set bits (SET) or clear bits (CLEAR),
// bit-packed at the width of the largest gap, and the rest go as they are
// (LITERAL).  See include/bfsc.h for the byte layout.
//
// Encode: a plan pass over the segments (blocks and non-empty segments
// before each one), a size pass (one wave per block: popcount, the two
// lists' first position and largest gap, the class), a scan of the payload
// sizes, the segment offsets (a linear function of those counts), and a
// pack pass (one wave per block; SET / CLEAR fields ORed into LDS).
// Decode: a plan pass over the headers, one wave per block (directory entry
// checked against the next one, lists expanded by a prefix sum of the gaps
// and an XOR into an LDS bitmap), and a final check of every segment's
// popcount against its header.
#include "common.hpp"

namespace bfsc {

constexpr uint32_t kBmBlk = 128;  // words per block
constexpr uint32_t kBmMagic = 0x31434D42u;
enum : uint32_t { kBmZero = 0, kBmOnes = 1, kBmSet = 2, kBmClear = 3, kBmLit = 4 };
constexpr uint32_t kBmScan = 4096;  // entries per workgroup of the payload scan
constexpr uint64_t kBmMaxSegWords = 1ull << 27;  // 2^32 bits: the header's popcount fits

__host__ __device__ constexpr uint64_t bm_max_blocks(uint64_t max_words, uint32_t nseg) {
    return max_words / kBmBlk + nseg + 1;
}

struct BmWs {
    uint32_t *blk_base;  // [nseg+1] first block of each segment
    uint32_t *ne_base;   // [nseg+1] non-empty segments before each one
    uint32_t *seg_pop;   // [nseg+1] set bits per segment (encode)
    uint64_t *out_off;   // [nseg+1] decode: output word offset of each segment (caller's array)
    uint32_t *carry;     // [4 x prep chunks] per chunk of segments: blocks, non-empty
                         // segments (encode) / blocks, words low, words high (decode)
    uint32_t *info;      // [2 x max blocks] class | width << 8 | count << 16, first
    uint32_t *pw;        // [max blocks + 1] payload words -> their exclusive prefix
    uint32_t *pw_chunk;  // [scan chunks]
    uint32_t *bpop;      // [max blocks] set bits per block (encode: of the input, decode: of the output)
    uint32_t max_blocks;
};

__host__ __device__ inline size_t bm_ws_layout(void *ws, uint64_t max_words, uint32_t nseg, BmWs *w) {
    char *b = (char *)ws;
    size_t off = 0;
    const size_t n1 = (size_t)nseg + 1;
    const uint64_t mb = bm_max_blocks(max_words, nseg);
    if (w) w->blk_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (w) w->ne_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (w) w->seg_pop = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (w) w->carry = (uint32_t *)(b + off);
    off = align256(off + (size_t)prep_chunks(nseg) * 16);
    if (w) w->info = (uint32_t *)(b + off);
    off = align256(off + mb * 8);
    if (w) w->pw = (uint32_t *)(b + off);
    off = align256(off + (mb + 1) * 4);
    if (w) w->pw_chunk = (uint32_t *)(b + off);
    off = align256(off + ((mb + 1 + kBmScan - 1) / kBmScan) * 4);
    if (w) w->bpop = (uint32_t *)(b + off);
    off = align256(off + mb * 4);
    if (w) {
        w->max_blocks = (uint32_t)mb;
        w->out_off = nullptr;
    }
    return off;
}

struct BmArgs {
    const uint32_t *bits;
    const uint64_t *seg_w;
    const uint8_t *in;             // decode input
    const uint64_t *seg_byte_off;  // decode input
    uint64_t *seg_byte_off_out;    // encode output
    uint32_t *out_words;           // decode output
    uint8_t *out;                  // encode output
    uint64_t out_cap;              // bytes (encode) or words (decode)
    uint32_t nseg;
    uint64_t max_words;
    BmWs w;
    uint32_t *err;
};

// ------------------------------------------------------------------ lists

__device__ __forceinline__ uint32_t ffbl(uint32_t x) { return (uint32_t)__builtin_ctz(x); }

// Largest distance between consecutive set bits of one word (0 if it has
// fewer than two): one more than the longest run of clear bits strictly
// between its lowest and highest set bit.  The run is found in five steps
// with no data-dependent loop: p_k marks the bits that start a run of at
// least k (p_1 = z, p_2k = p_k & p_k >> k), and the length is built from the
// largest step down, keeping a step when some run still reaches that far.
__device__ __forceinline__ uint32_t inner_gap(uint32_t x) {
    if (__popc(x) < 2) return 0u;
    const uint32_t lo = ffbl(x), hi = 31u - (uint32_t)__clz(x);
    const uint32_t z = ~x & ((1u << hi) - 1u) & ~((2u << lo) - 1u);
    const uint32_t p1 = z, p2 = p1 & (p1 >> 1), p4 = p2 & (p2 >> 2), p8 = p4 & (p4 >> 4), p16 = p8 & (p8 >> 8);
    // q: bits starting a run of at least `run` (all bits for run = 0)
    uint32_t q = 0xFFFFFFFFu, run = 0;
    uint32_t t = q & p16;  // run >= 16 (z has at most 29 bits, so at most one step of 16)
    if (t) { q = t; run = 16; }
    t = q & (p8 >> run);
    if (t) { q = t; run += 8; }
    t = q & (p4 >> run);
    if (t) { q = t; run += 4; }
    t = q & (p2 >> run);
    if (t) { q = t; run += 2; }
    t = q & (p1 >> run);
    if (t) { run += 1; }
    return run + 1u;
}

// One list of a block (its positions are the set bits of xa = word lane and
// xb = word 64 + lane): count, first position, largest gap, and per lane the
// list's last position + 1 before each of the lane's two words (0: none).
struct BmList {
    uint32_t count, first, gmax;
    uint32_t preva, prevb;   // last position + 1 before word lane / word 64 + lane
    uint32_t ranka, rankb;   // list entries before word lane / word 64 + lane
};

__device__ __forceinline__ BmList bm_list(uint32_t xa, uint32_t xb, uint32_t lane) {
    BmList L;
    const uint32_t ca = __popc(xa), cb = __popc(xb);
    const uint32_t ia = wave_incl_scan(ca);
    const uint32_t ta = readlane(ia, 63);
    const uint32_t ib = wave_incl_scan(cb);
    L.count = ta + readlane(ib, 63);
    L.ranka = ia - ca;
    L.rankb = ta + ib - cb;
    const uint32_t fa = xa ? 32u * lane + ffbl(xa) : 0xFFFFFFFFu;
    const uint32_t fb = xb ? 32u * (64u + lane) + ffbl(xb) : 0xFFFFFFFFu;
    L.first = wave_min(min(fa, fb));
    const uint32_t la = xa ? 32u * lane + 32u - (uint32_t)__clz(xa) : 0u;
    const uint32_t lb = xb ? 32u * (64u + lane) + 32u - (uint32_t)__clz(xb) : 0u;
    const uint32_t ma = wave_incl_max(la);
    const uint32_t tm = readlane(ma, 63);
    const uint32_t mb = max(wave_incl_max(lb), tm);
    L.preva = lane_prev(ma, 0u);
    L.prevb = lane_prev(mb, tm);
    uint32_t g = max(inner_gap(xa), inner_gap(xb));
    if (xa && L.preva) g = max(g, fa + 1u - L.preva);
    if (xb && L.prevb) g = max(g, fb + 1u - L.prevb);
    L.gmax = wave_max(g);
    return L;
}

__device__ __forceinline__ uint32_t list_words(uint32_t count, uint32_t width) {
    return count ? (uint32_t)(((uint64_t)(count - 1) * width + 31) / 32) : 0u;
}

// The block's class and directory fields (as the format's choice rule says).
struct BmChoice {
    uint32_t cls, width, count, first, words;
};

__device__ __forceinline__ BmChoice bm_choose(uint32_t wa, uint32_t wb, uint32_t n32, uint32_t lane,
                                              uint32_t *pop_out) {
    const uint32_t va = lane < n32 ? 0xFFFFFFFFu : 0u, vb = lane + 64 < n32 ? 0xFFFFFFFFu : 0u;
    const BmList S = bm_list(wa, wb, lane);
    const BmList C = bm_list(~wa & va, ~wb & vb, lane);
    *pop_out = S.count;
    BmChoice ch = {kBmLit, 0u, 0u, 0u, n32};
    if (S.count == 0) return BmChoice{kBmZero, 0u, 0u, 0u, 0u};
    if (C.count == 0) return BmChoice{kBmOnes, 0u, 0u, 0u, 0u};
    const uint32_t ws = bitlen32(S.gmax), wc = bitlen32(C.gmax);
    const uint32_t ns = list_words(S.count, ws), nc = list_words(C.count, wc);
    if (ns <= nc && ns <= n32)
        ch = BmChoice{kBmSet, ws, S.count, S.first, ns};
    else if (nc <= n32)
        ch = BmChoice{kBmClear, wc, C.count, C.first, nc};
    return ch;
}

// ------------------------------------------------------------------ encode plan

// The encode plan's totals at index nseg (blocks, non-empty segments); more
// blocks than max_words allows: no block runs.
__device__ __forceinline__ void bm_plan_end(const BmArgs &a, uint32_t tb, uint32_t te) {
    const bool over = tb > a.w.max_blocks;
    if (over) raise_err(a.err, kErrInval);
    a.w.blk_base[a.nseg] = over ? 0u : tb;
    a.w.ne_base[a.nseg] = te;
}

// Pass 1, one workgroup per chunk of segments; a batch of one chunk is then
// complete (its pass 2 is not launched).
__global__ __launch_bounds__(1024) void k_bm_plan_local(BmArgs a) {
    __shared__ uint32_t s_tmp[17];
    const uint32_t tid = threadIdx.x, c = blockIdx.x, r = c * kPrepChunk + tid;
    uint32_t nb = 0, ne = 0;
    if (r < a.nseg) {
        const uint64_t s = a.seg_w[r], e = a.seg_w[r + 1];
        const bool bad = e < s || e > a.max_words || e - s >= kBmMaxSegWords;
        if (bad) raise_err(a.err, kErrInval);
        const uint64_t nw = bad ? 0ull : e - s;
        nb = (uint32_t)((nw + kBmBlk - 1) / kBmBlk);
        ne = nw ? 1u : 0u;
    }
    uint32_t tb, te;
    const uint32_t xb = wg_excl_scan(nb, s_tmp, &tb);
    const uint32_t xe = wg_excl_scan(ne, s_tmp, &te);
    if (r < a.nseg) {
        a.w.blk_base[r] = xb;
        a.w.ne_base[r] = xe;
    }
    if (tid == 0) *(uint2 *)(a.w.carry + 4 * c) = make_uint2(tb, te);
    if (gridDim.x == 1 && tid == 0) bm_plan_end(a, tb, te);
}

__global__ __launch_bounds__(1024) void k_bm_plan_fix(BmArgs a) {
    __shared__ uint2 s_red[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6, c = blockIdx.x;
    uint32_t qb = 0, qe = 0;
    for (uint32_t i = tid; i < c; i += blockDim.x) {
        const uint2 x = *(const uint2 *)(a.w.carry + 4 * i);
        qb += x.x;
        qe += x.y;
    }
    qb = wave_sum(qb);
    qe = wave_sum(qe);
    if (lane == 0) s_red[w] = make_uint2(qb, qe);
    __syncthreads();
    uint32_t pb = 0, pe = 0;
    for (uint32_t i = 0; i < (blockDim.x >> 6); ++i) {
        pb += s_red[i].x;
        pe += s_red[i].y;
    }
    const uint32_t r = c * kPrepChunk + tid;
    if (r < a.nseg) {
        a.w.blk_base[r] += pb;
        a.w.ne_base[r] += pe;
    }
    if (c + 1 == gridDim.x && tid == 0) {
        const uint2 own = *(const uint2 *)(a.w.carry + 4 * c);
        bm_plan_end(a, pb + own.x, pe + own.y);
    }
}

// ------------------------------------------------------------------ encode passes

// The block of global index k: its segment r, index kk in the segment, word
// count n32 and first word.
struct BmBlock {
    uint32_t r, kk, n32;
    uint64_t w0;
};

__device__ __forceinline__ BmBlock bm_block(const BmArgs &a, uint32_t k, uint32_t lane) {
    BmBlock B;
    B.r = wave_find(a.w.blk_base, a.nseg, k, lane);
    B.kk = k - readfirst(a.w.blk_base[B.r]);
    const uint64_t s = readfirst64(a.seg_w[B.r]), e = readfirst64(a.seg_w[B.r + 1]);
    const uint64_t rem = e - s - (uint64_t)B.kk * kBmBlk;
    B.n32 = (uint32_t)(rem < kBmBlk ? rem : kBmBlk);
    B.w0 = s + (uint64_t)B.kk * kBmBlk;
    return B;
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_bm_size(BmArgs a) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t total = readfirst(a.w.blk_base[a.nseg]);
    const uint32_t W = blockIdx.x * WAVES + (threadIdx.x >> 6), NW = gridDim.x * WAVES;
    for (uint32_t k = W; k < total; k += NW) {
        const BmBlock B = bm_block(a, k, lane);
        const uint32_t *src = a.bits + B.w0;
        const uint32_t wa = lane < B.n32 ? src[lane] : 0u, wb = lane + 64 < B.n32 ? src[64 + lane] : 0u;
        uint32_t pop;
        const BmChoice ch = bm_choose(wa, wb, B.n32, lane, &pop);
        if (lane == 0) {
            *(uint2 *)(a.w.info + 2 * (uint64_t)k) = make_uint2(ch.cls | ch.width << 8 | ch.count << 16, ch.first);
            a.w.pw[k] = ch.words;
            a.w.bpop[k] = pop;
        }
    }
}

// Exclusive scan of pw[0 .. total) in chunks of kBmScan (4 per thread):
// chunk-local prefixes and chunk totals, then the carries.
__global__ __launch_bounds__(1024) void k_bm_scan_local(BmArgs a) {
    __shared__ uint32_t s_tmp[17];
    const uint32_t total = a.w.blk_base[a.nseg];
    const uint32_t tid = threadIdx.x, c = blockIdx.x;
    const uint64_t i0 = (uint64_t)c * kBmScan + 4ull * tid;
    uint32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = i0 + q < total ? a.w.pw[i0 + q] : 0u;
    const uint32_t s = v[0] + v[1] + v[2] + v[3];
    uint32_t tt;
    uint32_t x = wg_excl_scan(s, s_tmp, &tt);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (i0 + q < total) a.w.pw[i0 + q] = x;
        x += v[q];
    }
    if (tid == 0) a.w.pw_chunk[c] = tt;
}

__global__ __launch_bounds__(1024) void k_bm_scan_fix(BmArgs a) {
    __shared__ uint32_t s_red[16];
    const uint32_t total = a.w.blk_base[a.nseg];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6, c = blockIdx.x;
    uint32_t q = 0;
    for (uint32_t i = tid; i < c; i += blockDim.x) q += a.w.pw_chunk[i];
    q = wave_sum(q);
    if (lane == 0) s_red[w] = q;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t i = 0; i < (blockDim.x >> 6); ++i) pre += s_red[i];
    const uint64_t i0 = (uint64_t)c * kBmScan + 4ull * tid;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i0 + k < total) a.w.pw[i0 + k] += pre;
    // the grand total at pw[total], by the chunk that holds index total
    if (tid == 0 && (uint64_t)total / kBmScan == c) a.w.pw[total] = pre + a.w.pw_chunk[c];
}

// Byte offset of segment r: 16 bytes per non-empty segment, 12 per block and
// 4 per payload word before it.  The segment's set bits (its header field)
// are the sum of its blocks' counts, taken by one wave per segment: counted
// block by block into one word per segment, all of a segment's blocks would
// have hit the same address.
__device__ __forceinline__ uint64_t bm_seg_start(const BmArgs &a, uint32_t r) {
    const uint32_t b = min(a.w.blk_base[r], a.w.max_blocks);
    return 16ull * a.w.ne_base[r] + 12ull * b + 4ull * a.w.pw[b];
}

__global__ __launch_bounds__(256) void k_bm_offsets(BmArgs a) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t r = readfirst(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (r > a.nseg) return;
    if (lane == 0) {
        const uint64_t S = bm_seg_start(a, r);
        a.seg_byte_off_out[r] = S;
        if (r == a.nseg && S > a.out_cap) raise_err(a.err, kErrCapacity);
    }
    if (r == a.nseg) return;
    const uint32_t b0 = min(readfirst(a.w.blk_base[r]), a.w.max_blocks);
    const uint32_t b1 = min(readfirst(a.w.blk_base[r + 1]), a.w.max_blocks);
    uint32_t sum = 0;
    for (uint32_t k = b0 + lane; k < b1; k += 64) sum += a.w.bpop[k];
    sum = wave_sum(sum);
    if (lane == 0) a.w.seg_pop[r] = sum;
}

__device__ __forceinline__ void or_word(uint32_t *buf, uint32_t pos, uint32_t v) {
    const uint64_t x = (uint64_t)v << (pos & 31);
    atomicOr(buf + (pos >> 5), (uint32_t)x);
    if ((uint32_t)(x >> 32)) atomicOr(buf + (pos >> 5) + 1, (uint32_t)(x >> 32));
}

// A lane's list entries in one word x (positions base32 + bit), the first of
// them having rank `rank` and the list's previous position + 1 `prev1`: gap
// fields (rank j >= 1: field j - 1 at bit (j - 1) w) ORed into buf.
__device__ __forceinline__ void bm_put_word(uint32_t *buf, uint32_t x, uint32_t base32, uint32_t rank,
                                            uint32_t prev1, uint32_t w) {
    uint32_t prev = prev1 ? prev1 - 1u : 0u;
    bool have = prev1 != 0;
    while (x) {
        const uint32_t p = base32 + ffbl(x);
        x &= x - 1u;
        if (have && w) or_word(buf, (rank - 1u) * w, p - prev);
        prev = p;
        have = true;
        ++rank;
    }
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_bm_pack(BmArgs a) {
    __shared__ uint32_t s_buf[WAVES][kBmBlk + 2];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *buf = s_buf[wv];
    const uint32_t total = readfirst(a.w.blk_base[a.nseg]);
    const uint32_t W = blockIdx.x * WAVES + wv, NW = gridDim.x * WAVES;
    for (uint32_t k = W; k < total; k += NW) {
        const BmBlock B = bm_block(a, k, lane);
        const uint32_t *src = a.bits + B.w0;
        const uint32_t wa = lane < B.n32 ? src[lane] : 0u, wb = lane + 64 < B.n32 ? src[64 + lane] : 0u;
        const uint2 inf = *(const uint2 *)(a.w.info + 2 * (uint64_t)k);
        const uint32_t cls = readfirst(inf.x & 0xFFu), width = readfirst((inf.x >> 8) & 0xFFu);
        const uint32_t count = readfirst(inf.x >> 16), first = readfirst(inf.y);
        const uint32_t b0 = readfirst(a.w.blk_base[B.r]), nb = readfirst(a.w.blk_base[B.r + 1]) - b0;
        const uint32_t poff = readfirst(a.w.pw[k]) - readfirst(a.w.pw[b0]);
        const uint32_t words = readfirst(a.w.pw[k + 1]) - readfirst(a.w.pw[k]);
        const uint64_t S = bm_seg_start(a, B.r);
        const uint64_t meta = 16ull + 12ull * nb;
        const uint64_t pay = S + meta + 4ull * poff;
        if (pay + 4ull * words > a.out_cap || S + meta > a.out_cap) continue;  // reported by k_bm_offsets
        uint32_t *seg = (uint32_t *)(a.out + S);
        if (B.kk == 0 && lane < 4) {
            const uint64_t nw = readfirst64(a.seg_w[B.r + 1]) - readfirst64(a.seg_w[B.r]);
            const uint32_t h = lane == 0 ? (uint32_t)nw : lane == 1 ? a.w.seg_pop[B.r] : lane == 2 ? nb : kBmMagic;
            seg[lane] = h;
        }
        if (lane < 3) {
            const uint32_t d = lane == 0 ? poff : lane == 1 ? (count | first << 16) : (cls | width << 8);
            seg[4 + 3 * B.kk + lane] = d;
        }
        uint32_t *dst = (uint32_t *)(a.out + pay);
        if (cls == kBmLit) {
            if (lane < B.n32) dst[lane] = wa;
            if (lane + 64 < B.n32) dst[64 + lane] = wb;
        } else if (cls == kBmSet || cls == kBmClear) {
            buf[lane] = 0u;
            buf[lane + 64] = 0u;
            if (lane < 2) buf[kBmBlk + lane] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const uint32_t va = lane < B.n32 ? 0xFFFFFFFFu : 0u, vb = lane + 64 < B.n32 ? 0xFFFFFFFFu : 0u;
            const uint32_t xa = cls == kBmSet ? wa : ~wa & va, xb = cls == kBmSet ? wb : ~wb & vb;
            const BmList L = bm_list(xa, xb, lane);
            bm_put_word(buf, xa, 32u * lane, L.ranka, L.preva, width);
            bm_put_word(buf, xb, 32u * (64u + lane), L.rankb, L.prevb, width);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane < words) dst[lane] = buf[lane];
            if (lane + 64 < words) dst[64 + lane] = buf[lane + 64];
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// ------------------------------------------------------------------ decode

// The decode plan's totals at index nseg (blocks, output words) and their
// checks.
__device__ __forceinline__ void bmd_plan_end(const BmArgs &a, uint32_t tb, uint64_t co) {
    const bool over = tb > a.w.max_blocks;
    if (over) raise_err(a.err, kErrCorrupt);
    a.w.blk_base[a.nseg] = over ? 0u : tb;
    a.w.out_off[a.nseg] = co;
    if (co > a.out_cap) raise_err(a.err, kErrCapacity);
}

// Plan pass 1 over the headers: form (empty, or compressed when the header
// checks), words and blocks per segment, their scans inside the chunk.
__global__ __launch_bounds__(1024) void k_bmd_plan_local(BmArgs a) {
    __shared__ uint32_t s_tmp[17];
    __shared__ unsigned long long s_w[16];
    __shared__ unsigned long long s_c;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, c = blockIdx.x;
    const uint32_t r = c * kPrepChunk + tid;
    uint32_t nw = 0, nb = 0;
    if (r < a.nseg) {
        const uint64_t s = a.seg_byte_off[r], e = a.seg_byte_off[r + 1];
        bool bad = e < s || (s & 3) || (e & 3);
        if (!bad && e > s) {
            const uint64_t L = e - s;
            const uint32_t *h = (const uint32_t *)(a.in + s);
            if (L < 16) {
                bad = true;
            } else {
                const uint32_t hn = h[0], hb = h[2], mg = h[3];
                bad = mg != kBmMagic || hn == 0 || (uint64_t)hn >= kBmMaxSegWords ||
                      hb != (hn + kBmBlk - 1) / kBmBlk || 16ull + 12ull * hb > L;
                nw = hn;
                nb = hb;
            }
        }
        if (bad) {
            raise_err(a.err, kErrCorrupt);
            nw = 0;
            nb = 0;
        }
    }
    uint32_t tb;
    const uint32_t xb = wg_excl_scan(nb, s_tmp, &tb);
    uint64_t incl = nw;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t l2 = shfl_up((uint32_t)incl, d), h2 = shfl_up((uint32_t)(incl >> 32), d);
        if (lane >= (uint32_t)d) incl += ((uint64_t)h2 << 32) | l2;
    }
    if (lane == 63) s_w[wv] = incl;
    __syncthreads();
    if (tid == 0) {
        unsigned long long acc = 0;
        for (uint32_t i = 0; i < (blockDim.x >> 6); ++i) {
            const unsigned long long x = s_w[i];
            s_w[i] = acc;
            acc += x;
        }
        s_c = acc;
    }
    __syncthreads();
    if (r < a.nseg) {
        a.w.blk_base[r] = xb;
        a.w.out_off[r] = s_w[wv] + incl - nw;
    }
    if (tid == 0) {
        a.w.carry[4 * c] = tb;
        a.w.carry[4 * c + 1] = (uint32_t)s_c;
        a.w.carry[4 * c + 2] = (uint32_t)(s_c >> 32);
        if (gridDim.x == 1) bmd_plan_end(a, tb, s_c);  // one chunk: complete, no pass 2
    }
}

__global__ __launch_bounds__(1024) void k_bmd_plan_fix(BmArgs a) {
    __shared__ unsigned long long s_n[16];
    __shared__ uint32_t s_b[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, c = blockIdx.x;
    uint64_t qn = 0;
    uint32_t qb = 0;
    for (uint32_t i = tid; i < c; i += blockDim.x) {
        qn += (uint64_t)a.w.carry[4 * i + 1] | (uint64_t)a.w.carry[4 * i + 2] << 32;
        qb += a.w.carry[4 * i];
    }
    qn = wave_sum64(qn);
    qb = wave_sum(qb);
    if (lane == 0) {
        s_n[wv] = qn;
        s_b[wv] = qb;
    }
    __syncthreads();
    uint64_t pn = 0;
    uint32_t pb = 0;
    for (uint32_t i = 0; i < (blockDim.x >> 6); ++i) {
        pn += s_n[i];
        pb += s_b[i];
    }
    const uint32_t r = c * kPrepChunk + tid;
    if (r < a.nseg) {
        a.w.blk_base[r] += pb;
        a.w.out_off[r] += pn;
    }
    if (c + 1 == gridDim.x && tid == 0) {
        const uint64_t own = (uint64_t)a.w.carry[4 * c + 1] | (uint64_t)a.w.carry[4 * c + 2] << 32;
        bmd_plan_end(a, pb + a.w.carry[4 * c], pn + own);
    }
}

// w-bit field at bit pos of LDS words (w <= 32).
__device__ __forceinline__ uint32_t bm_field(const uint32_t *buf, uint32_t pos, uint32_t w) {
    const uint32_t wi = pos >> 5, sh = pos & 31;
    const uint32_t v = __builtin_amdgcn_alignbit(buf[wi + 1], buf[wi], sh);
    return w >= 32 ? v : (v & ((1u << w) - 1u));
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_bmd_blocks(BmArgs a) {
    __shared__ uint32_t s_pay[WAVES][kBmBlk + 2];
    __shared__ uint32_t s_bm[WAVES][kBmBlk];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t *pay = s_pay[wv], *bm = s_bm[wv];
    const uint32_t total = readfirst(a.w.blk_base[a.nseg]);
    const uint32_t W = blockIdx.x * WAVES + wv, NW = gridDim.x * WAVES;
    for (uint32_t k = W; k < total; k += NW) {
        const uint32_t r = wave_find(a.w.blk_base, a.nseg, k, lane);
        const uint32_t kk = k - readfirst(a.w.blk_base[r]);
        const uint64_t S = readfirst64(a.seg_byte_off[r]), E = readfirst64(a.seg_byte_off[r + 1]);
        const uint32_t *seg = (const uint32_t *)(a.in + S);
        const uint32_t nw = readfirst(seg[0]), nb = readfirst(seg[2]);
        const uint64_t meta = 16ull + 12ull * nb;
        const uint64_t avail = (E - S - meta) / 4;
        const uint32_t n32 = min(kBmBlk, nw - kk * kBmBlk), nbits = 32u * n32;
        const uint32_t *de = seg + 4 + 3 * kk;
        const uint32_t off = readfirst(de[0]), cf = readfirst(de[1]), cw = readfirst(de[2]);
        const uint64_t next = kk + 1 < nb ? (uint64_t)readfirst(de[3]) : avail;
        const uint32_t count = cf & 0xFFFFu, first = cf >> 16, cls = cw & 0xFFu, width = (cw >> 8) & 0xFFu;
        bool bad = (cw >> 16) != 0u || (E - S - meta) % 4 != 0;
        if (kk == 0) bad |= off != 0u;
        uint32_t words = 0;
        if (cls == kBmZero || cls == kBmOnes || cls == kBmLit) {
            bad |= count != 0u || first != 0u || width != 0u;
            words = cls == kBmLit ? n32 : 0u;
        } else if (cls == kBmSet || cls == kBmClear) {
            bad |= count == 0u || count > nbits || width > 32u || first >= nbits;
            words = list_words(count, width);
            bad |= words > n32;
        } else {
            bad = true;
        }
        bad |= (uint64_t)off + words != next || (uint64_t)off + words > avail;
        if (bad) {
            if (lane == 0) raise_err(a.err, kErrCorrupt);
            continue;
        }
        const uint32_t *src = seg + meta / 4 + off;
        uint32_t xa = 0, xb = 0;
        if (cls == kBmOnes) {
            xa = 0xFFFFFFFFu;
            xb = 0xFFFFFFFFu;
        } else if (cls == kBmLit) {
            xa = lane < n32 ? src[lane] : 0u;
            xb = lane + 64 < n32 ? src[64 + lane] : 0u;
        } else if (cls != kBmZero) {
            // the gap fields into LDS, then 64 gaps per step: prefix sum,
            // checks, and an XOR of each position into the block's bitmap
            pay[lane] = lane < words ? src[lane] : 0u;
            pay[lane + 64] = lane + 64 < words ? src[64 + lane] : 0u;
            if (lane < 2) pay[kBmBlk + lane] = 0u;
            bm[lane] = 0u;
            bm[lane + 64] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) atomicXor(bm + (first >> 5), 1u << (first & 31));
            uint32_t pos = first;  // the last position placed
            bool ok = true;
            for (uint32_t j0 = 1; j0 < count && ok; j0 += 64) {
                const uint32_t j = j0 + lane;
                const bool in = j < count;
                const uint32_t d = in && width ? bm_field(pay, (j - 1) * width, width) : 0u;
                const bool zero = in && d == 0u;
                // gaps past the block end the block anyway: clamped so the
                // 64-lane sum cannot wrap
                const uint32_t incl = wave_incl_scan(min(d, 8192u));
                const uint32_t p = pos + incl;
                const bool out = in && p >= nbits;
                ok = ballot(zero || out) == 0ull;
                if (ok && in) atomicXor(bm + (p >> 5), 1u << (p & 31));
                pos += readlane(incl, 63);
            }
            if (!ok) {
                if (lane == 0) raise_err(a.err, kErrCorrupt);
                continue;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const uint32_t inv = cls == kBmClear ? 0xFFFFFFFFu : 0u;
            xa = bm[lane] ^ inv;
            xb = bm[lane + 64] ^ inv;
            __builtin_amdgcn_wave_barrier();
        }
        if (lane >= n32) xa = 0u;
        if (lane + 64 >= n32) xb = 0u;
        const uint64_t o = readfirst64(a.w.out_off[r]) + (uint64_t)kk * kBmBlk;
        if (lane < n32 && o + lane < a.out_cap) a.out_words[o + lane] = xa;
        if (lane + 64 < n32 && o + 64 + lane < a.out_cap) a.out_words[o + 64 + lane] = xb;
        const uint32_t seen = wave_sum(__popc(xa) + __popc(xb));
        if (lane == 0) a.w.bpop[k] = seen;
    }
}

// Every compressed segment's popcount against its header: one wave per
// segment adds up its blocks' counts.  (A block found damaged has left its
// count unwritten, but it has reported the stream already.)
__global__ __launch_bounds__(256) void k_bmd_final(BmArgs a) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t r = readfirst(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (r >= a.nseg) return;
    const uint64_t s = readfirst64(a.seg_byte_off[r]), e = readfirst64(a.seg_byte_off[r + 1]);
    const uint32_t b0 = min(readfirst(a.w.blk_base[r]), a.w.max_blocks);
    const uint32_t b1 = min(readfirst(a.w.blk_base[r + 1]), a.w.max_blocks);
    if (e <= s || b1 <= b0) return;
    uint32_t sum = 0;
    for (uint32_t k = b0 + lane; k < b1; k += 64) sum += a.w.bpop[k];
    sum = wave_sum(sum);
    const uint32_t *h = (const uint32_t *)(a.in + s);
    if (lane == 0 && h[1] != sum) raise_err(a.err, kErrCorrupt);
}

// ------------------------------------------------------------------ launchers

size_t bitmap_ws_bytes(uint64_t max_words, uint32_t nseg) { return bm_ws_layout(nullptr, max_words, nseg, nullptr); }

uint64_t bitmap_encode_bound(uint64_t n_words, uint32_t nseg) {
    return 16ull * nseg + 12ull * ((n_words + kBmBlk - 1) / kBmBlk + nseg) + 4ull * n_words;
}

static uint32_t bm_grid(const bfsc_ctx *ctx, uint64_t blocks) {
    uint64_t g = (uint64_t)ctx->n_cu * 8;
    const uint64_t need = (blocks + 3) / 4;
    if (g > need) g = need;
    return (uint32_t)(g ? g : 1);
}

int launch_bitmap_encode(bfsc_ctx *ctx, const uint32_t *bits, const uint64_t *seg_w, uint32_t nseg, uint64_t max_words,
                         uint8_t *out, uint64_t out_cap, uint64_t *seg_byte_off, void *ws, hipStream_t s) {
    BmArgs a{};
    a.bits = bits;
    a.seg_w = seg_w;
    a.nseg = nseg;
    a.max_words = max_words;
    a.out = out;
    a.out_cap = out_cap;
    a.seg_byte_off_out = seg_byte_off;
    a.err = ctx->err;
    bm_ws_layout(ws, max_words, nseg, &a.w);
    const uint32_t chunks = prep_chunks(nseg);
    hipLaunchKernelGGL(k_bm_plan_local, dim3(chunks), dim3(kPrepChunk), 0, s, a);
    if (chunks > 1) hipLaunchKernelGGL(k_bm_plan_fix, dim3(chunks), dim3(kPrepChunk), 0, s, a);
    const uint32_t grid = bm_grid(ctx, a.w.max_blocks);
    hipLaunchKernelGGL(k_bm_size<4>, dim3(grid), dim3(256), 0, s, a);
    const uint32_t sc = (uint32_t)((a.w.max_blocks + 1ull + kBmScan - 1) / kBmScan);
    hipLaunchKernelGGL(k_bm_scan_local, dim3(sc), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_bm_scan_fix, dim3(sc), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_bm_offsets, dim3((nseg + 1 + 3) / 4), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bm_pack<4>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_bitmap_decode(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                         uint64_t max_words, uint32_t *out, uint64_t out_cap, uint64_t *out_off, void *ws,
                         hipStream_t s) {
    BmArgs a{};
    a.in = in;
    a.seg_byte_off = seg_byte_off;
    a.nseg = nseg;
    a.max_words = max_words;
    a.out_words = out;
    a.out_cap = out_cap;
    a.err = ctx->err;
    bm_ws_layout(ws, max_words, nseg, &a.w);
    a.w.out_off = out_off;
    const uint32_t chunks = prep_chunks(nseg);
    hipLaunchKernelGGL(k_bmd_plan_local, dim3(chunks), dim3(kPrepChunk), 0, s, a);
    if (chunks > 1) hipLaunchKernelGGL(k_bmd_plan_fix, dim3(chunks), dim3(kPrepChunk), 0, s, a);
    hipLaunchKernelGGL(k_bmd_blocks<4>, dim3(bm_grid(ctx, a.w.max_blocks)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_bmd_final, dim3((nseg + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

}  // namespace bfsc
