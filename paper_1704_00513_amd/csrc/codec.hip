// Frontier codec kernels for gfx950: batch planning, per-block codec choice,
// encode and validating decode.  The block formats follow the compression
// techniques of Romera, arXiv 1704.00513 (delta coding + binary packing in
// blocks of 128, eqs. (6)-(7); patched coding with exceptions, eqs. (8)-(9);
// bitmap indexes for dense sets), in this project's own byte layout
// (described in bfsc.h).
//
// Work decomposition: a tile is one group of <= 16 blocks of one segment.
// One wave handles one 128-ID block at a time, two IDs per lane (lane l holds
// IDs l and 64+l, so loads and stores are fully coalesced); cross-lane steps
// use DPP.  Encode = plan passes (per-segment counts and offsets, and every
// tile's segment) + pack pass (every tile into a private slot) + offset scan
// + place pass.  Decode = plan passes (the same from the stream's headers) +
// one decoding pass: the group table gives every tile its payload offset.
#include "common.hpp"
#include "mlp_mfma.hpp"

namespace bfsc {

// ------------------------------------------------------------------ scans

// ------------------------------------------------------------------ plan

struct PlanArgs {
    const uint64_t *seg_off;
    const uint32_t *seg_lo;
    const uint32_t *seg_hi;
    uint32_t nseg;
    uint64_t max_ids;
    Plan p;
    uint32_t *err;
};

// Per-segment block / group / tile / fixed-word counts.  A segment of n IDs
// is empty (n = 0: no bytes), raw (n below the compression threshold: its n
// IDs) or compressed (16-byte header, 8 bytes of directory per block, the
// group table and the payloads).  Pass 1, one workgroup per kPrepChunk
// segments: the counts, their exclusive scans inside the chunk, and the
// chunk's totals.
// The batch totals at index nseg (blocks, groups, fixed words, tiles) from
// the totals cb, cg, cf, ct of all chunks.  Inconsistent offsets (totals
// beyond what max_ids allows) disable the batch: no tile runs, so nothing is
// indexed past the workspace.
__device__ __forceinline__ void plan_end(const PlanArgs &a, uint32_t cb, uint32_t cg, uint32_t ct, uint32_t cf) {
    const uint64_t max_blocks = (a.max_ids + kBlock - 1) / kBlock + a.nseg;
    const bool over = ct > a.p.max_tiles || cb > max_blocks;
    if (over) raise_err(a.err, kErrInval);
    a.p.blk_base[a.nseg] = cb;
    a.p.grp_base[a.nseg] = cg;
    a.p.fix_base[a.nseg] = cf;
    a.p.tile_base[a.nseg] = over ? 0u : ct;
    a.p.counter[0] = 0;
}

// Groups of a segment of n IDs (none for a raw one, n below the threshold
// T), and its tiles: one per group, or one for a segment without groups.
__device__ __forceinline__ uint32_t plan_seg_groups(uint32_t n, uint32_t T) {
    const uint32_t nb = (n >> 7) + ((n & 127u) != 0u);
    return n < T ? 0u : (nb >> 4) + ((nb & 15u) != 0u);
}
__device__ __forceinline__ uint32_t plan_seg_tiles(uint32_t n, uint32_t T) { return max(1u, plan_seg_groups(n, T)); }

// Every tile's segment and that segment's first tile: tile_seg[tb + q] =
// (r, tb) for q < nt.  A segment of up to 64 tiles is written by its own
// lane; longer ones by the whole wave, one after another, their tiles
// across the lanes.  Nothing is written at or past max_tiles (plan_end then
// refuses the batch).  Only the encoder's plan keeps the map (tile_seg is
// NULL in the selection pass's).
__device__ __forceinline__ void plan_tile_map(const PlanArgs &a, uint32_t r, uint32_t tb, uint32_t nt,
                                              uint32_t lane) {
    const bool own = nt <= 64u;
    if (own)
        for (uint32_t q = 0; q < nt && (uint64_t)tb + q < a.p.max_tiles; ++q) a.p.tile_seg[tb + q] = make_uint2(r, tb);
    uint64_t m = ballot(!own);
    while (m) {
        const uint32_t j = (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        const uint32_t rj = readlane(r, j), tj = readlane(tb, j), nj = readlane(nt, j);
        for (uint32_t q = lane; q < nj && (uint64_t)tj + q < a.p.max_tiles; q += 64)
            a.p.tile_seg[tj + q] = make_uint2(rj, tj);
    }
}

// Pass 1, one workgroup per chunk of kPrepChunk segments: the chunk-local
// exclusive scans and the chunk's totals.  A batch of one chunk is then
// complete (its pass 2 is not launched) and the pass writes the tile map.
__global__ __launch_bounds__(1024) void k_plan_local(PlanArgs a) {
    const uint32_t tid = threadIdx.x, c = blockIdx.x;
    __shared__ uint32_t s_tmp[17];
    const uint32_t T = a.p.raw_below;
    const uint32_t r = c * kPrepChunk + tid;
    uint32_t nb = 0, ng = 0, nt = 0, nf = 0;
    if (r < a.nseg) {
        const uint64_t s = a.seg_off[r], e = a.seg_off[r + 1];
        const uint32_t lo = a.seg_lo[r], hi = a.seg_hi[r];
        const bool bad = e < s || e > a.max_ids || lo > hi || (e - s) > (uint64_t)(hi - lo);
        const uint32_t n = bad ? 0u : (uint32_t)(e - s);
        if (bad) raise_err(a.err, kErrInval);
        a.p.seg_n[r] = n;
        const bool raw = n < T;  // (an empty segment too: no groups)
        nb = (n >> 7) + ((n & 127u) != 0u);
        ng = plan_seg_groups(n, T);
        nt = plan_seg_tiles(n, T);
        nf = raw ? n : 4u + 2u * nb;
        if (n == 0) nf = 0;
    }
    uint32_t tb, tg, tt, tf;
    const uint32_t xb = wg_excl_scan(nb, s_tmp, &tb);
    const uint32_t xg = wg_excl_scan(ng, s_tmp, &tg);
    const uint32_t xt = wg_excl_scan(nt, s_tmp, &tt);
    const uint32_t xf = wg_excl_scan(nf, s_tmp, &tf);
    if (r < a.nseg) {
        a.p.blk_base[r] = xb;
        a.p.grp_base[r] = xg;
        a.p.tile_base[r] = xt;
        a.p.fix_base[r] = xf;
    }
    if (tid == 0) *(uint4 *)(a.p.chunk_sums + 4 * c) = make_uint4(tb, tg, tt, tf);
    if (gridDim.x == 1 && tid == 0) plan_end(a, tb, tg, tt, tf);
    if (gridDim.x == 1 && a.p.tile_seg) plan_tile_map(a, r, xt, nt, tid & 63);
}

// Sum over workgroup threads of four values (up to 1024 threads).
__device__ __forceinline__ uint4 wg_sum4(uint4 v, uint4 *s_red /*[16]*/) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    v.z = wave_sum(v.z);
    v.w = wave_sum(v.w);
    if (lane == 0) s_red[w] = v;
    __syncthreads();
    uint4 t = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t i = 0; i < (blockDim.x >> 6); ++i) {
        const uint4 x = s_red[i];
        t.x += x.x, t.y += x.y, t.z += x.z, t.w += x.w;
    }
    return t;
}

// Pass 2, one workgroup per chunk: adds the totals of the chunks before it
// and writes the tile map; the last workgroup writes the batch totals at
// index nseg.
__global__ __launch_bounds__(1024) void k_plan_fix(PlanArgs a) {
    const uint32_t tid = threadIdx.x, c = blockIdx.x;
    __shared__ uint4 s_red[16];
    uint4 q = make_uint4(0u, 0u, 0u, 0u);
    const uint4 *cs = (const uint4 *)a.p.chunk_sums;
    for (uint32_t i = tid; i < c; i += blockDim.x) {
        const uint4 x = cs[i];
        q.x += x.x, q.y += x.y, q.z += x.z, q.w += x.w;
    }
    const uint4 pre = wg_sum4(q, s_red);
    const uint32_t r = c * kPrepChunk + tid;
    uint32_t tb = 0, nt = 0;
    if (r < a.nseg) {
        a.p.blk_base[r] += pre.x;
        a.p.grp_base[r] += pre.y;
        tb = a.p.tile_base[r] + pre.z;
        a.p.tile_base[r] = tb;
        a.p.fix_base[r] += pre.w;
        nt = plan_seg_tiles(a.p.seg_n[r], a.p.raw_below);
    }
    if (c + 1 == gridDim.x && tid == 0) {
        const uint4 own = cs[c];
        plan_end(a, pre.x + own.x, pre.y + own.y, pre.z + own.z, pre.w + own.w);
    }
    if (a.p.tile_seg) plan_tile_map(a, r, tb, nt, tid & 63);
}

// ------------------------------------------------------------------ block analysis

struct BlockInfo {
    uint32_t cls, param, aux, words, first;
};

// Deltas of one block, held by one wave: lane l holds value index l (a) and
// 64+l (b); delta index j of value j is v_j - v_{j-1}.
struct BlockRegs {
    uint32_t da, db;   // deltas (0 where there is none)
    uint32_t oa, ob;   // value - v0
    bool hasa, hasb;   // lane carries delta j = lane / 64+lane
};

struct BlockStats {
    uint32_t nk, m, v0, span, dmin, dmax, wmin;
};

__device__ __forceinline__ void fetch_block(const uint32_t *ids, uint32_t nk, uint32_t lane,
                                            uint32_t &va, uint32_t &vb) {
    if (nk == kBlock) {  // uniform: no per-lane masks for a full block
        va = ids[lane];
        vb = ids[64 + lane];
    } else {
        va = lane < nk ? ids[lane] : 0u;
        vb = lane + 64 < nk ? ids[64 + lane] : 0u;
    }
}

__device__ __forceinline__ void analyze_block(uint32_t va, uint32_t vb, uint32_t nk, uint32_t lo,
                                              uint32_t hi, uint32_t lane, bool want_min,
                                              BlockRegs &R, BlockStats &S, uint32_t *err) {
    const bool ina = lane < nk, inb = lane + 64 < nk;
    const uint32_t a63 = readlane(va, 63);
    const uint32_t pa = lane_prev(va, 0u);
    const uint32_t pb = lane_prev(vb, a63);
    R.hasa = ina && lane >= 1;
    R.hasb = inb;
    R.da = R.hasa ? va - pa : 0u;
    R.db = R.hasb ? vb - pb : 0u;
    // bitwise, not short-circuit: straight-line selects instead of branches
    const bool bad = (R.hasa & (va <= pa)) | (R.hasb & (vb <= pb)) |
                     (ina & ((va < lo) | (va >= hi))) | (inb & ((vb < lo) | (vb >= hi)));
    if (ballot(bad) != 0ull && lane == 0) raise_err(err, kErrInval);
    S.nk = nk;
    S.m = nk - 1;
    S.v0 = readlane(va, 0);
    const uint32_t vlast = nk <= 64 ? readlane(va, nk - 1) : readlane(vb, nk - 65);
    S.span = vlast - S.v0;
    S.dmax = wave_max(max(R.da, R.db));
    if (want_min) {
        uint32_t mn = 0xFFFFFFFFu;
        if (R.hasa) mn = R.da;
        if (R.hasb) mn = min(mn, R.db);
        S.dmin = S.m ? wave_min(mn) : 0u;
    } else {
        S.dmin = 0;
    }
    S.wmin = bitlen32(S.dmax);
    R.oa = va - S.v0;
    R.ob = vb - S.v0;
}

// Best PFOR exception width: fewest payload words with 10 E <= m; ties go
// to the larger b.  b = wmin (no exceptions) is always allowed.  E only
// grows as b shrinks, so the search stops at the first b with too many.
__device__ __forceinline__ void pfor_best(const BlockRegs &R, const BlockStats &S, uint32_t &bb,
                                          uint32_t &E, uint32_t &words) {
    bb = S.wmin;
    E = 0;
    words = cdiv32(S.m * S.wmin, 32);
    for (int b = (int)S.wmin - 1; b >= 0; --b) {
        // deltas of lanes without one are 0, so they never count
        const uint32_t thr = (1u << b) - 1u;
        const uint32_t e = popc64(ballot(R.da > thr)) + popc64(ballot(R.db > thr));
        if (10u * e > S.m) break;
        const uint32_t h = e ? S.wmin - (uint32_t)b : 0u;
        const uint32_t w = cdiv32(S.m * (uint32_t)b, 32) + cdiv32(e, 4) + cdiv32(e * h, 32);
        if (w < words) {
            words = w;
            bb = (uint32_t)b;
            E = e;
        }
    }
}

__device__ __forceinline__ bool class_valid(const BlockStats &S, uint32_t c) {
    if (c == kClsBitmap) return S.span <= kBitmapMaxSpan;
    if (c >= 1 && c <= 33) return c - 1 >= S.wmin;
    return c == kClsPfor;
}

// Class and payload size of a block.  given >= 0: that class (checked);
// otherwise plain minimal-width packing or the exhaustive choice (fewest
// payload words; ties: bit-pack < bitmap < PFOR).
__device__ __forceinline__ BlockInfo choose(const BlockRegs &R, const BlockStats &S, int mode,
                                            int given, uint32_t *err) {
    BlockInfo I;
    I.first = 0;
    uint32_t c;
    if (given >= 0) {
        c = (uint32_t)given;
        if (!class_valid(S, c)) {
            if (lane_id() == 0) raise_err(err, kErrInval);
            c = 0xFFu;
        }
    } else {
        c = mode == BFSC_SEL_PLAIN_BP ? 1u + S.wmin : 0xFFu;
    }
    uint32_t pb = 0, pe = 0, pw = 0;
    if (c == 0xFFu || c == kClsPfor) pfor_best(R, S, pb, pe, pw);
    if (c == 0xFFu) {
        uint32_t best = 1u + S.wmin, bw = cdiv32(S.m * S.wmin, 32);
        if (S.span <= kBitmapMaxSpan) {
            const uint32_t w = cdiv32(S.span, 32);
            if (w < bw) { bw = w; best = kClsBitmap; }
        }
        if (pw < bw) best = kClsPfor;
        c = best;
    }
    I.cls = c;
    if (c == kClsBitmap) {
        I.param = 0;
        I.aux = S.span;
        I.words = cdiv32(S.span, 32);
    } else if (c <= 33) {
        I.param = c - 1;
        I.aux = 0;
        I.words = cdiv32(S.m * (c - 1), 32);
    } else {
        I.param = pb;
        const uint32_t h = pe ? S.wmin - pb : 0u;
        I.aux = pe | (h << 8);
        I.words = pw;
    }
    return I;
}

// ------------------------------------------------------------------ packing

__device__ __forceinline__ void put_bits(uint32_t *buf, uint32_t pos, uint32_t w, uint32_t v) {
    if (w == 0) return;
    const uint32_t wi = pos >> 5, sh = pos & 31;
    atomicOr(&buf[wi], v << sh);
    if (sh + w > 32) atomicOr(&buf[wi + 1], v >> (32 - sh));
}

// floor(x / w) for x < 2^13 and 1 <= w <= 32: multiply by ceil(2^32 / w)
// and keep the high word (the error term is below 2^-19, far from the next
// integer because frac(x / w) <= 1 - 1/w).
__device__ __forceinline__ uint32_t div_small(uint32_t x, uint32_t w, uint32_t recip) {
    return w == 1 ? x : __umulhi(x, recip);
}

// Packs the deltas of one block at width w (w >= 1) into words [0,
// ceil(m w / 32)) of buf without atomics.  Field t = j - 1 starts at bit t w.
// Fields that start in the same word occupy disjoint bits, so an inclusive
// prefix sum of the shifted fields gives each word as a difference of two
// prefixes; the field that straddles into the word adds its spilled high bits.
// pj / dj are per-wave LDS scratch of 128 words each.
__device__ __forceinline__ void pack_fields(uint32_t *buf, uint32_t *pj, uint32_t *dj, uint32_t da,
                                            uint32_t db, bool hasa, bool hasb, uint32_t m,
                                            uint32_t w, uint32_t lane) {
    const uint32_t ja = lane, jb = 64 + lane;
    const uint32_t loa = hasa ? da << (((ja - 1) * w) & 31) : 0u;
    const uint32_t lob = hasb ? db << (((jb - 1) * w) & 31) : 0u;
    const uint32_t pa = wave_incl_scan(loa);
    const uint32_t pb = wave_incl_scan(lob) + readlane(pa, 63);
    pj[ja] = pa;  // pj[j] = sum of fields 0 .. j-1; pj[0] = 0
    pj[jb] = pb;
    dj[ja] = da;
    dj[jb] = db;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t words = cdiv32(m * w, 32);
    const uint32_t recip = w > 1 ? 0xFFFFFFFFu / w + 1u : 0u;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t q = lane + 64u * h;
        if (q < words) {
            const uint32_t x0 = 32 * q;
            const uint32_t tA = div_small(x0 + w - 1, w, recip);   // first field starting here
            const uint32_t tB = min(div_small(x0 + 31, w, recip), m - 1);
            uint32_t v = tA <= tB ? pj[tB + 1] - pj[tA] : 0u;
            if (tA >= 1 && tA * w != x0) v += dj[tA] >> (x0 - (tA - 1) * w);
            buf[q] = v;
        }
    }
}

// Builds one block's payload in the wave's LDS buffer (128 words) without
// atomics for the packed fields (bit-pack, PFOR low bits); bitmap bits and
// PFOR exceptions use LDS atomics.
__device__ __forceinline__ void pack_block_scan(uint32_t *buf, uint32_t *pj, uint32_t *dj,
                                                const BlockInfo &I, const BlockRegs &R,
                                                const BlockStats &S, uint32_t lane) {
    if (I.cls == kClsBitmap) {
        buf[lane] = 0;
        buf[lane + 64] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (R.hasa && R.oa >= 1 && R.oa <= S.span) atomicOr(&buf[(R.oa - 1) >> 5], 1u << ((R.oa - 1) & 31));
        if (R.hasb && R.ob >= 1 && R.ob <= S.span) atomicOr(&buf[(R.ob - 1) >> 5], 1u << ((R.ob - 1) & 31));
    } else if (I.cls <= 33) {
        pack_fields(buf, pj, dj, R.da, R.db, R.hasa, R.hasb, S.m, I.param, lane);
    } else {
        const uint32_t b = I.param, E = I.aux & 0xFFu, h = I.aux >> 8;
        const uint32_t lw = cdiv32(S.m * b, 32), qw = cdiv32(E, 4), hw = cdiv32(E * h, 32);
        if (b) {
            const uint32_t mask = b >= 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
            pack_fields(buf, pj, dj, R.da & mask, R.db & mask, R.hasa, R.hasb, S.m, b, lane);
        }
        if (lane < qw + hw) buf[lw + lane] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (E) {
            const bool xa = R.hasa && b < 32 && (R.da >> b) != 0u;
            const bool xb = R.hasb && b < 32 && (R.db >> b) != 0u;
            const uint64_t ma = ballot(xa), mb = ballot(xb);
            if (xa) {
                const uint32_t e = mbcnt64(ma);
                put_bits(buf, lw * 32 + e * 8, 8, lane - 1);
                put_bits(buf, (lw + qw) * 32 + e * h, h, R.da >> b);
            }
            if (xb) {
                const uint32_t e = popc64(ma) + mbcnt64(mb);
                put_bits(buf, lw * 32 + e * 8, 8, 63 + lane);
                put_bits(buf, (lw + qw) * 32 + e * h, h, R.db >> b);
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Builds one block's payload in the wave's LDS buffer (128 words).
__device__ __forceinline__ void pack_block(uint32_t *buf, const BlockInfo &I, const BlockRegs &R,
                                           const BlockStats &S, uint32_t lane) {
    buf[lane] = 0;
    buf[lane + 64] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t ja = lane, jb = 64 + lane;  // delta indices
    if (I.cls == kClsBitmap) {
        if (R.hasa && R.oa >= 1 && R.oa <= S.span) atomicOr(&buf[(R.oa - 1) >> 5], 1u << ((R.oa - 1) & 31));
        if (R.hasb && R.ob >= 1 && R.ob <= S.span) atomicOr(&buf[(R.ob - 1) >> 5], 1u << ((R.ob - 1) & 31));
    } else if (I.cls <= 33) {
        const uint32_t w = I.param;
        if (R.hasa) put_bits(buf, (ja - 1) * w, w, R.da);
        if (R.hasb) put_bits(buf, (jb - 1) * w, w, R.db);
    } else {
        const uint32_t b = I.param, E = I.aux & 0xFFu, h = I.aux >> 8;
        const uint32_t mask = b >= 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
        if (R.hasa) put_bits(buf, (ja - 1) * b, b, R.da & mask);
        if (R.hasb) put_bits(buf, (jb - 1) * b, b, R.db & mask);
        if (E) {
            const uint32_t lw = cdiv32(S.m * b, 32), qw = cdiv32(E, 4);
            const bool xa = R.hasa && b < 32 && (R.da >> b) != 0u;
            const bool xb = R.hasb && b < 32 && (R.db >> b) != 0u;
            const uint64_t ma = ballot(xa), mb = ballot(xb);
            if (xa) {
                const uint32_t e = mbcnt64(ma);
                put_bits(buf, lw * 32 + e * 8, 8, ja - 1);
                put_bits(buf, (lw + qw) * 32 + e * h, h, R.da >> b);
            }
            if (xb) {
                const uint32_t e = popc64(ma) + mbcnt64(mb);
                put_bits(buf, lw * 32 + e * 8, 8, jb - 1);
                put_bits(buf, (lw + qw) * 32 + e * h, h, R.db >> b);
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------ encode

struct EncArgs {
    const uint32_t *ids;
    const uint64_t *seg_off;
    const uint32_t *seg_lo;
    const uint32_t *seg_hi;
    const uint8_t *classes;
    int mode;
    uint32_t nseg;
    uint32_t *out;          // word view of the output
    uint64_t out_cap;       // bytes
    uint64_t *seg_byte_off;
    Plan p;
    uint32_t *err;
    uint32_t strided;       // unit order of the staged pack pass (else contiguous per wave)
    const int32_t *seg_level;  // BFS level per segment (learned choice: a feature)
    const MlpMfma *w;          // the network in MFMA operand order (learned choice)
};

// Segment and metadata of one encoder tile.
struct EncTile {
    uint64_t id_base;
    uint32_t n, nb, lo, hi, bb, g;
    int32_t level;
};
constexpr uint32_t kMetaChunk = 64;  // tiles resolved per pre-pass of a workgroup

__device__ __forceinline__ EncTile enc_tile_meta(const Plan &p, const uint64_t *seg_off,
                                                 const uint32_t *seg_lo, const uint32_t *seg_hi,
                                                 uint32_t nseg, uint32_t t,
                                                 const int32_t *seg_level = nullptr) {
    const uint32_t r = upper_bound_m1(p.tile_base, nseg, t);
    EncTile m;
    m.g = t - p.tile_base[r];
    m.bb = p.blk_base[r];
    m.nb = p.blk_base[r + 1] - m.bb;
    m.n = p.seg_n[r];
    m.lo = seg_lo[r];
    m.hi = seg_hi[r];
    m.id_base = seg_off[r];
    m.level = seg_level ? seg_level[r] : 0;
    return m;
}

__device__ __forceinline__ uint16_t f16bits(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(uint16_t, h);
}

// Eight selector features of a block (identical arithmetic to the spec in bfsc.h).
__device__ __forceinline__ void block_features(const BlockStats &S, uint32_t seg_n, int32_t level,
                                               float f[8]) {
    const int32_t L = level < 0 ? 0 : (level > 63 ? 63 : level);
    f[0] = (float)S.nk / 128.0f;
    f[1] = S.m ? (float)bitlen32(S.dmin) / 32.0f : 0.0f;
    f[2] = S.m ? (float)S.wmin / 32.0f : 0.0f;
    f[3] = S.m ? (float)bitlen32(S.span / S.m) / 32.0f : 0.0f;
    f[4] = (float)bitlen32(S.span) / 32.0f;
    f[5] = __fdiv_rn((float)S.nk, (float)((uint64_t)S.span + 1ull));
    f[6] = (float)L / 64.0f;
    f[7] = (float)bitlen32(seg_n) / 32.0f;
}

// ORs a field (v < 2^32, at most 32 bits) into the LDS words at bit pos, the
// spilled high part into the next word unconditionally (it is 0 when the
// field does not cross a word boundary): no branches.
__device__ __forceinline__ void or_field(uint32_t *buf, uint32_t pos, uint32_t v) {
    const uint32_t wi = pos >> 5, sh = pos & 31;
    atomicOr(&buf[wi], v << sh);
    atomicOr(&buf[wi + 1], sh ? v >> (32 - sh) : 0u);
}

// PFOR payload of a full block into zeroed LDS words: the low b bits of every
// delta as a bit-pack at width b, then the E exception positions (bytes,
// j - 1, ascending) and their high parts (h bits each).  Only the lanes that
// hold an exception (at most 12) write the last two parts.
__device__ __forceinline__ void pack_pfor_full(uint32_t *buf, uint32_t da, uint32_t db, uint32_t b,
                                               uint32_t E, uint32_t h, uint32_t lane) {
    constexpr uint32_t m = kBlock - 1;
    const uint32_t mask = b >= 32 ? 0xFFFFFFFFu : (1u << b) - 1u;
    or_field(buf, (lane ? lane - 1 : 0u) * b, da & mask);
    or_field(buf, (63 + lane) * b, db & mask);
    if (E) {
        const uint32_t lw = (m * b + 31) >> 5, qw = (E + 3) >> 2;
        const bool xa = da > mask, xb = db > mask;
        const uint64_t ma = ballot(xa), mb = ballot(xb);
        if (xa) {
            const uint32_t e = mbcnt64(ma);
            or_field(buf, lw * 32 + e * 8, lane - 1);
            or_field(buf, (lw + qw) * 32 + e * h, da >> b);
        }
        if (xb) {
            const uint32_t e = popc64(ma) + mbcnt64(mb);
            or_field(buf, lw * 32 + e * 8, 63 + lane);
            or_field(buf, (lw + qw) * 32 + e * h, db >> b);
        }
    }
}

// What enc_full encodes a block as: the plain minimal width, the exhaustive
// choice, or (a resolved learned choice) the bitmap or PFOR with its best b.
enum FullSel : int { kSelPlain = 0, kSelExhaustive = 1, kSelBitmap = 2, kSelPfor = 3 };

// Full block (128 IDs) whose class the encoder picks itself or is handed:
// the same choice as choose(), computed with scalar selects, and bit-pack /
// bitmap payloads packed without branches.  PFOR payloads are packed by the
// general routine.  kSelBitmap requires span <= 4096.
// wmin_known: the block's minimal width when the caller has it already, else
// a negative value.
// The block's two directory words are returned in d0 / d1 (the caller
// collects a unit's entries in a register and stores them once).
__device__ __forceinline__ uint32_t enc_full(uint32_t va, uint32_t vb, uint32_t lo, uint32_t hi,
                                             int sel, uint32_t &d0, uint32_t &d1, uint32_t *dst,
                                             uint32_t *buf, uint32_t lane, uint32_t *err,
                                             int wmin_known = -1) {
    constexpr uint32_t m = kBlock - 1;
    const uint32_t a63 = readlane(va, 63);
    const uint32_t pa = lane_prev(va, 0u);
    const uint32_t pb = lane_prev(vb, a63);
    const uint32_t da = lane ? va - pa : 0u;
    const uint32_t db = vb - pb;
    const uint32_t v0 = readlane(va, 0), vlast = readlane(vb, 63);
    // strictly increasing, then first >= lo and last < hi bound every value
    const uint64_t bad = ballot((lane != 0) & (va <= pa)) | ballot(vb <= pb);
    if ((bad != 0ull) | (v0 < lo) | (vlast >= hi)) {
        if (lane == 0) raise_err(err, kErrInval);
    }
    const uint32_t wmin = wmin_known >= 0 ? (uint32_t)wmin_known : bitlen32(wave_max(max(da, db)));
    const uint32_t span = vlast - v0;
    const uint32_t bpw = (m * wmin + 31) >> 5;
    uint32_t cls = 1 + wmin, param = wmin, aux = 0, words = bpw;
    uint32_t pfb = wmin, pfe = 0;
    if (sel == kSelBitmap) {
        cls = kClsBitmap;
        param = 0;
        aux = span;
        words = (span + 31) >> 5;
    } else if (sel >= kSelExhaustive) {
        const uint32_t bmw = (span + 31) >> 5;
        if ((sel == kSelExhaustive) & (span <= kBitmapMaxSpan) & (bmw < words)) {
            cls = kClsBitmap;
            param = 0;
            aux = span;
            words = bmw;
        }
        // PFOR: fewest words with 10 E <= m (E <= 12), ties to the larger b.
        // A width b < wmin has E >= 1, so it costs at least ceil(m b / 32) + 2
        // words: widths whose bound reaches the best so far cannot be chosen
        // and are skipped (b <= (32 (words - 3)) / m is the largest candidate).
        uint32_t best = bpw;
        const uint32_t bcap = sel == kSelPfor ? wmin : words >= 3 ? min(wmin, (32 * (words - 3)) / m + 1) : 0u;
        uint32_t low = m * bcap, h = wmin - bcap;
        for (uint32_t b = bcap; b-- > 0;) {
            low -= m;
            ++h;
            const uint32_t thr = (1u << b) - 1u;
            const uint32_t e = popc64(ballot(da > thr)) + popc64(ballot(db > thr));
            if (e > m / 10) break;
            const uint32_t wd = ((low + 31) >> 5) + ((e + 3) >> 2) + ((e * h + 31) >> 5);
            if (wd < best) {
                best = wd;
                pfb = b;
                pfe = e;
            }
        }
        if ((best < words) | (sel == kSelPfor)) {
            cls = kClsPfor;
            param = pfb;
            aux = pfe | (pfe ? (wmin - pfb) << 8 : 0u);
            words = best;
        }
    }
    d0 = v0 - lo;
    d1 = cls | (param << 8) | (aux << 16);
    buf[lane] = 0u;
    buf[lane + 64] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (cls == kClsPfor) {
        pack_pfor_full(buf, da, db, param, aux & 0xFFu, aux >> 8, lane);
    } else if (cls == kClsBitmap) {
        // bit o-1 for offset o = v - v0 >= 1 (the first value is implied); the
        // word index is kept inside the buffer even for unsorted input,
        // which has already been flagged as invalid
        const uint32_t oa = va - v0, ob = vb - v0;
        const uint32_t qa = oa ? oa - 1 : 0u, qb = ob - 1;
        atomicOr(&buf[(qa >> 5) & 127], oa ? 1u << (qa & 31) : 0u);
        atomicOr(&buf[(qb >> 5) & 127], 1u << (qb & 31));
    } else {
        // field of delta j at bit (j-1) w: lane l carries deltas l (none for
        // l = 0, whose delta is 0) and 64+l
        or_field(buf, (lane ? lane - 1 : 0u) * param, da);
        or_field(buf, (63 + lane) * param, db);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t wa = buf[lane], wb = buf[lane + 64];
    if (lane < words) dst[lane] = wa;
    if (lane + 64 < words) dst[lane + 64] = wb;
    return words;
}

// Analyses, chooses and packs one block held by the wave (value index l in
// va, 64+l in vb of lane l); writes its directory entry to dir[0..1] and its
// payload words to dst; returns the payload words.  FULL: a block of exactly
// 128 IDs (all but the last block of a segment), where every per-lane
// validity test folds away at compile time.
template <bool FULL, bool SCANPACK>
__device__ __forceinline__ uint32_t enc_block(uint32_t va, uint32_t vb, uint32_t nk, uint32_t lo,
                                              uint32_t hi, int mode, int given, uint32_t &d0, uint32_t &d1,
                                              uint32_t *dst, uint32_t *buf, uint32_t *pj, uint32_t *dj,
                                              uint32_t lane, uint32_t *err) {
    if constexpr (FULL) {
        if (given < 0 && !SCANPACK)
            return enc_full(va, vb, lo, hi, mode == BFSC_SEL_PLAIN_BP ? kSelPlain : kSelExhaustive, d0, d1, dst,
                            buf, lane, err);
        nk = kBlock;
    } else {
        nk = readfirst(nk);
    }
    BlockRegs R;
    BlockStats S;
    analyze_block(va, vb, nk, lo, hi, lane, false, R, S, err);
    const BlockInfo I = choose(R, S, mode, given, err);
    d0 = S.v0 - lo;
    d1 = I.cls | (I.param << 8) | (I.aux << 16);
    if (I.words) {
        if constexpr (SCANPACK)
            pack_block_scan(buf, pj, dj, I, R, S, lane);
        else
            pack_block(buf, I, R, S, lane);
        if (lane < I.words) dst[lane] = buf[lane];
        if (lane + 64 < I.words) dst[lane + 64] = buf[lane + 64];
        __builtin_amdgcn_wave_barrier();
    }
    return I.words;
}

// A DPP move whose result only some lanes select must still run with every
// lane of the wave active: were the compiler to move it under the select's
// exec mask, lanes would read disabled neighbours (and get `old`).  The
// empty asm consumes the value where it is computed, which pins it.
__device__ __forceinline__ uint32_t pin(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ void pin64(uint64_t &x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    asm volatile("" : "+v"(lo), "+v"(hi));
    x = ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------------------------ 16-lane rows

// Lanes 16r .. 16r+15 of a wave form row r (ri = lane & 15), the unit of the
// GFX9 DPP row operations: row_shr:n (0x110+n), row_mirror (0x140),
// row_half_mirror (0x141), the quad permutations 0x4E / 0xB1, and
// row_newbcast:n (0x150+n, lane n of the row to all of it).  The helpers
// combine values inside every row at once; a row is either wholly active or
// wholly inactive wherever they are used.
__device__ __forceinline__ uint32_t row_max(uint32_t v) {
    v = max(v, dpp<0x140>(v, v));
    v = max(v, dpp<0x141>(v, v));
    v = max(v, dpp<0x4E>(v, v));
    v = max(v, dpp<0xB1>(v, v));
    return v;
}
__device__ __forceinline__ uint32_t row_min(uint32_t v) {
    v = min(v, dpp<0x140>(v, v));
    v = min(v, dpp<0x141>(v, v));
    v = min(v, dpp<0x4E>(v, v));
    v = min(v, dpp<0xB1>(v, v));
    return v;
}
__device__ __forceinline__ uint32_t row_sum(uint32_t v) {
    v += dpp<0x140>(v, v);
    v += dpp<0x141>(v, v);
    v += dpp<0x4E>(v, v);
    v += dpp<0xB1>(v, v);
    return v;
}
// Exclusive prefix sum inside the row (row shifts bring 0 in at its start).
__device__ __forceinline__ uint32_t row_excl_scan(uint32_t v) {
    uint32_t s = v;
    s += dpp<0x111>(0u, s);
    s += dpp<0x112>(0u, s);
    s += dpp<0x114>(0u, s);
    s += dpp<0x118>(0u, s);
    return s - v;
}

// LDS words a wave needs to assemble a full unit's payloads: 8 blocks of at
// most 128 words, one spill word, rounded to 16 bytes, then 2 x 64 words that
// take the atomics of lanes with nothing to write (one word per lane: were
// they aimed at the payload, up to 16 lanes would hit one address).
constexpr uint32_t kUnitPay = kHalf * kBlock + 4;
constexpr uint32_t kUnitStage = kUnitPay + 128;

// A full unit (8 blocks of 128 IDs, src 4-byte aligned; al16: 16-byte
// aligned) encoded by the wave in two passes of four blocks, one block per
// 16-lane row: lane i of row r holds IDs 8i .. 8i+7 of block 4p + r in pass
// p.  The per-block analysis is then a few row reductions shared by four
// blocks and the class choice is ordinary vector code, the same choice as
// enc_full for the selection kind (FullSel) of the block: selu for every
// block, or sel8[k] for block k when sel8 (LDS) is given.  The payloads are
// assembled back to back in the wave's LDS area st (kUnitStage words) and
// copied to pay (16-byte aligned); the 16 directory words go to dir.
// Returns the unit's payload words.
__device__ __forceinline__ uint32_t enc_unit_r(const uint32_t *src, bool al16, uint32_t lo, uint32_t hi,
                                               uint32_t selu, const uint8_t *sel8, uint32_t *pay, uint32_t *dir,
                                               uint32_t *st, uint32_t lane, uint32_t *err) {
    constexpr uint32_t m = kBlock - 1;
    const uint32_t ri = lane & 15, r = lane >> 4;
    const uint64_t all = ballot(true);
    uint32_t *const dmy0 = st + kUnitPay + lane, *const dmy1 = dmy0 + 64;
    // the previous unit's copy-out has read st before it is cleared
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) ((uint4 *)st)[lane + 64 * q] = make_uint4(0u, 0u, 0u, 0u);
    if (lane == 0) ((uint4 *)st)[256] = make_uint4(0u, 0u, 0u, 0u);
    uint32_t total = 0;
#pragma unroll 1
    for (uint32_t p = 0; p < 2; ++p) {
        uint32_t v[8];
        const uint32_t *ps = src + 512 * p + 8 * lane;
        if (al16) {
            const uint4 x = ((const uint4 *)ps)[0], y = ((const uint4 *)ps)[1];
            v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w;
            v[4] = y.x, v[5] = y.y, v[6] = y.z, v[7] = y.w;
        } else {
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) v[k] = ps[k];
        }
        // deltas: the row's first lane receives its own first ID (delta 0:
        // the first ID of a block is stored in the directory)
        const uint32_t pv = dpp<0x111>(v[0], v[7]);
#define BFSC_D(k) ((k) ? v[k] - v[(k) ? (k) - 1 : 0] : v[0] - pv)
        // strictly increasing inside the block, first >= lo, last < hi
        uint64_t okm = ballot(ri == 0 || v[0] > pv);
        uint32_t dm = BFSC_D(0);
#pragma unroll
        for (uint32_t k = 1; k < 8; ++k) {
            okm &= ballot(v[k] > v[k - 1]);
            dm = max(dm, BFSC_D(k));
        }
        const uint32_t v0 = dpp<0x150>(v[0], v[0]), vl = dpp<0x15F>(v[7], v[7]);
        okm &= ballot((v0 >= lo) & (vl < hi));
        if (okm != all) {
            if (lane == 0) raise_err(err, kErrInval);
        }
        const uint32_t wmin = bitlen32(row_max(dm));
        const uint32_t span = vl - v0;
        // the deltas are not kept from here on (recomputed where used)
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) v[k] = pin(v[k]);

        // choice, uniform inside each row
        const uint32_t sel = sel8 ? sel8[4 * p + r] : selu;
        const bool exh = sel == kSelExhaustive, pf = sel == kSelPfor;
        const uint32_t bpw = (m * wmin + 31) >> 5;
        uint32_t cls = 1 + wmin, param = wmin, aux = 0, words = bpw;
        const uint32_t bmw = (span + 31) >> 5;
        if ((sel == kSelBitmap) | (exh & (span <= kBitmapMaxSpan) & (bmw < words))) {
            cls = kClsBitmap;
            param = 0;
            aux = span;
            words = bmw;
        }
        if (ballot(exh | pf) != 0ull) {
            // PFOR: fewest words with 10 E <= m, ties to the larger b.  For
            // the exhaustive choice the same bound as enc_full prunes widths
            // that cannot win; a block resolved to PFOR tries every b < wmin
            // (and keeps b = wmin, no exceptions, if none is smaller)
            uint32_t best = bpw, pfb = wmin, pfe = 0;
            const uint32_t bcap = pf ? wmin : (exh & (words >= 3)) ? min(wmin, (32 * (words - 3)) / m + 1) : 0u;
            uint32_t b = bcap;
            bool live = b > 0;
            while (ballot(live) != 0ull) {
                if (live) {
                    --b;
                    const uint32_t thr = (1u << b) - 1u;
                    uint32_t c = 0;
#pragma unroll
                    for (uint32_t k = 0; k < 8; ++k) c += BFSC_D(k) > thr;
                    const uint32_t e = row_sum(c);
                    if (e > m / 10) {
                        live = false;
                    } else {
                        const uint32_t h = wmin - b;
                        const uint32_t wd = ((m * b + 31) >> 5) + ((e + 3) >> 2) + ((e * h + 31) >> 5);
                        if (wd < best) {
                            best = wd;
                            pfb = b;
                            pfe = e;
                        }
                        live = b > 0;
                    }
                }
            }
            if ((exh & (best < words)) | pf) {
                cls = kClsPfor;
                param = pfb;
                aux = pfe | (pfe ? (wmin - pfb) << 8 : 0u);
                words = best;
            }
        }

        // payload offsets: the pass's blocks back to back after the earlier
        // ones
        const uint32_t own = ri == 15 ? words : 0u;
        const uint32_t incl = wave_incl_scan(own);
        uint32_t *sg = st + total + (incl - own);
        total += readlane(incl, 63);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();

        // main fields.  A bitmap sets bit o-1 for offset o = v - v0 >= 1; a
        // bit-pack, or the low part of a PFOR, puts delta j at bit (j-1) w.
        // A lane's fields are gathered into a 64-bit window that starts at
        // the word of its first field and ORed into LDS with two atomics:
        // this holds the whole run of a bit-pack of width <= 4 (8 w + 31 <
        // 64 bits) and, mostly, of a bitmap; bitmap bits beyond the window
        // (sparse blocks, or unsorted input, which is flagged and kept inside
        // the block's words) and wider bit-packs are ORed field by field.
        const bool isbm = cls == kClsBitmap;
        const uint32_t pw = isbm ? 0u : param;
        const uint32_t mask = pw >= 32 ? 0xFFFFFFFFu : (1u << pw) - 1u;
        const bool narrow = isbm || pw <= 4;
        const uint32_t qmax = 32 * max(words, 1u) - 1, vb1 = v0 + 1;
        const uint32_t p0 = ri ? (8 * ri - 1) * pw : 0u;  // bit-pack: bit of the lane's first field
        const uint32_t b0 = ri == 0 ? 0u : isbm ? min(v[0] - vb1, qmax) >> 5 : p0 >> 5;
        // The window bit of a field, rel, is at or past 64 exactly when the
        // field is not in the window: a bitmap's first ID (v - vb1b wraps),
        // and every field of a bit-pack too wide for it (its run starts at
        // 2^31).  Bitmap bits past the window: a lane's IDs increase, so its
        // last one tells (unsorted input, already flagged, may lose bits but
        // writes nothing outside the block's words).
        const uint32_t one = isbm ? 1u : 0u, base32 = 32 * b0, vb1b = vb1 + base32;
        uint32_t relbp = narrow ? p0 - base32 - (ri ? 0u : pw) : 0x80000000u;  // bit-pack: field k
        uint64_t win = 0;
        const bool ofl = isbm & (v[7] - vb1b >= 64);
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) {
            const uint32_t rel = isbm ? v[k] - vb1b : relbp;
            const uint32_t val = (BFSC_D(k) & mask) | one;
            win |= (uint64_t)(rel < 64 ? val : 0u) << (rel & 63);
            pin64(win);  // one field at a time: keeps the live registers few
            relbp += pw;
        }
        atomicOr(narrow ? &sg[b0] : dmy0, (uint32_t)win);
        atomicOr(narrow ? &sg[b0 + 1] : dmy1, (uint32_t)(win >> 32));
        if (ballot(ofl) != 0ull) {
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) {
                const bool has = k != 0 || ri != 0;
                const uint32_t q = min(v[k] - vb1, qmax);
                const bool o = has & isbm & (q - 32 * b0 >= 64);
                atomicOr(o ? &sg[q >> 5] : dmy0, 1u << (q & 31));
            }
        }
        if (ballot(!narrow) != 0ull) {
            uint32_t pos = p0;
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) {
                const bool go = !narrow & (k != 0 || ri != 0);
                const uint64_t x = (uint64_t)(BFSC_D(k) & mask) << (pos & 31);
                atomicOr(go ? sg + (pos >> 5) : dmy0, (uint32_t)x);
                atomicOr(go ? sg + (pos >> 5) + 1 : dmy1, (uint32_t)(x >> 32));
                pos += k != 0 || ri != 0 ? pw : 0u;
            }
        }
        // PFOR exceptions: positions (bytes, j - 1) and high parts, in order.
        // A block has at most 12 over its 16 lanes, so the counting pass
        // keeps the first two of each lane (field, delta) and only those are
        // written; a lane with more (rare) takes the field-by-field loop.
        const bool ispf = cls == kClsPfor;
        if (ballot(ispf) != 0ull) {
            const uint32_t E = aux & 0xFFu, h = aux >> 8;
            const uint32_t lw = (m * pw + 31) >> 5, qw = (E + 3) >> 2;
            uint32_t xc = 0, k0x = 0, d0x = 0, k1x = 0, d1x = 0;
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) {
                const uint32_t dk = BFSC_D(k);
                const bool x = ispf & (dk > mask);
                k1x = (x & (xc == 1)) ? k : k1x;
                d1x = (x & (xc == 1)) ? dk : d1x;
                k0x = (x & (xc == 0)) ? k : k0x;
                d0x = (x & (xc == 0)) ? dk : d0x;
                xc += x;
            }
            const uint32_t e0 = row_excl_scan(xc);
            // exception number e of this lane at field k with delta dk
            auto put = [&](uint32_t e, uint32_t k, uint32_t dk) {
                const uint32_t bp = lw * 32 + e * 8, hp = (lw + qw) * 32 + e * h;
                atomicOr(sg + (bp >> 5), (8 * ri + k - 1) << (bp & 31));  // position byte: one word
                const uint64_t hx = (uint64_t)(dk >> (pw & 31)) << (hp & 31);
                atomicOr(sg + (hp >> 5), (uint32_t)hx);
                atomicOr(sg + (hp >> 5) + 1, (uint32_t)(hx >> 32));
            };
            if (xc > 0) put(e0, k0x, d0x);
            if (xc > 1) put(e0 + 1, k1x, d1x);
            if (ballot(xc > 2) != 0ull) {
                uint32_t e = e0;
#pragma unroll
                for (uint32_t k = 0; k < 8; ++k) {
                    const uint32_t dk = BFSC_D(k);
                    const bool x = ispf & (dk > mask);
                    if (x & (e >= e0 + 2)) put(e, k, dk);
                    e += x;
                }
            }
        }
#undef BFSC_D
        // directory entries: lanes 0 / 1 of row r write block 4p + r's words
        if (ri < 2) dir[8 * p + 2 * r + ri] = ri ? cls | (param << 8) | (aux << 16) : v0 - lo;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t q = 4 * lane; q < total; q += 256) *(uint4 *)(pay + q) = *(const uint4 *)(st + q);
    return total;
}

// Units a wave handles: a contiguous run (consecutive units mostly share a
// segment, so the segment is found once and then walked forward) or every
// NW-th unit.
struct UnitRange {
    uint32_t begin, end, step;
};
__device__ __forceinline__ UnitRange unit_range(uint32_t units, uint32_t waves, uint32_t w, bool strided) {
    const uint64_t W = (uint64_t)blockIdx.x * waves + w, NW = (uint64_t)gridDim.x * waves;
    UnitRange ur;
    if (strided) {
        ur.begin = (uint32_t)W;
        ur.end = units;
        ur.step = (uint32_t)NW;
    } else {
        ur.begin = (uint32_t)(W * units / NW);
        ur.end = (uint32_t)((W + 1) * units / NW);
        ur.step = 1;
    }
    return ur;
}

// The segment of the current tile and its fields, kept across the units of
// a wave.  seek() returns true when the segment changed (fields to reload).
struct SegCursor {
    uint32_t r = 0, t_first = 0, t_next = 0;
    bool have = false;
    uint32_t bb = 0, nb = 0, n = 0, lo = 0, hi = 0;
    uint32_t form = 0;  // decoder: 1 raw, 2 compressed
    uint64_t base = 0, S = 0, bytes = 0;
    __device__ __forceinline__ bool seek(const uint32_t *tile_base, uint32_t nseg, uint32_t t, uint32_t lane,
                                         bool jump) {
        if (have && t < t_next) return false;
        if (!have || jump) {
            r = wave_find(tile_base, nseg, t, lane);
            t_next = readfirst(tile_base[r + 1]);
        } else {
            while (t >= t_next) {
                ++r;
                t_next = readfirst(tile_base[r + 1]);
            }
        }
        t_first = readfirst(tile_base[r]);
        have = true;
        return true;
    }
};

// Pack pass, one wave per unit (half a tile: up to 8 blocks, 1024 IDs), the
// units being small enough that every wave gets several and none is left
// working alone at the end.  STAGE: the wave first stages the unit's IDs in
// LDS with every load in flight at once; otherwise it loads block by block,
// the next block's load in flight while the current one is packed.  Either
// way it analyses, chooses and packs the blocks in order into the unit's half
// of the tile's slot.
template <int WAVES, bool SCANPACK, bool STAGE>
__global__ __launch_bounds__(WAVES * 64, 6) void k_enc_pack_u(EncArgs a) {
    constexpr uint32_t kIds = kHalf * kBlock;
    constexpr uint32_t kPerLane = kIds / 64;
    // full units take the 16-lane-row encoder in the per-block packing
    // variants; it assembles payloads in the same per-wave LDS area that the
    // staged variant loads IDs into
    constexpr bool kGrp = !SCANPACK;
    __shared__ __align__(16) uint32_t s_ids[STAGE || kGrp ? WAVES : 1][STAGE || kGrp ? kUnitStage : 4];
    __shared__ uint32_t s_buf[WAVES][132];
    __shared__ uint32_t s_pj[SCANPACK ? WAVES : 1][128];
    __shared__ uint32_t s_dj[SCANPACK ? WAVES : 1][128];
    // wave index made scalar: the unit loop and the segment fields stay in
    // scalar registers
    const uint32_t lane = threadIdx.x & 63, w = readfirst(threadIdx.x >> 6);
    const uint32_t tiles = readfirst(a.p.tile_base[a.nseg]);
    // whole tiles per wave when every wave gets many (the segment is then
    // found once for both halves), else half tiles so that the waves end
    // evenly
    const bool by_tile = (uint64_t)tiles >= 8ull * gridDim.x * WAVES;
    uint32_t *sid = s_ids[STAGE || kGrp ? w : 0];
    UnitRange ur = unit_range(by_tile ? tiles : 2 * tiles, WAVES, w, a.strided);
    // the tile's segment from the plan's tile map, loaded one unit ahead
    // (the last unit's again at the end: the load is unconditional, so that
    // it stays in flight); the segment's fields are loaded again for every
    // unit (from the cache), so that nothing is carried from unit to unit
    // and they all stay scalar.  All by scalar loads, in one round: the wave
    // waits on them without waiting for its stores of the unit before.
    uint64_t tsn = 0;  // (segment, its first tile) of a tile, as one word
    if (ur.begin < ur.end) tsn = ldc((const uint64_t *)(a.p.tile_seg + (by_tile ? ur.begin : ur.begin >> 1)));
    for (uint32_t u = ur.begin; u < ur.end; u += ur.step) {
        const uint32_t t = by_tile ? u : u >> 1;
        const uint32_t h0 = by_tile ? 0u : (u & 1), h1 = by_tile ? 2u : h0 + 1;  // the halves to pack
        const uint32_t r = (uint32_t)tsn, t_first = (uint32_t)(tsn >> 32);
        const uint32_t un = min(u + ur.step, ur.end - 1);
        tsn = ldc((const uint64_t *)(a.p.tile_seg + (by_tile ? un : un >> 1)));
        const uint32_t bb = ldc(a.p.blk_base + r), be = ldc(a.p.blk_base + r + 1);
        const uint32_t n = ldc(a.p.seg_n + r);
        const uint32_t lo = ldc(a.seg_lo + r), hi = ldc(a.seg_hi + r);
        const uint64_t base = ldc(a.seg_off + r);
        asm volatile("" ::"s"(bb), "s"(be), "s"(n), "s"(lo), "s"(hi), "s"(base));
        // a raw segment's IDs are copied by the place pass: no blocks
        const uint32_t nb = n < a.p.raw_below ? 0u : be - bb;
        const uint32_t g = t - t_first;
        for (uint32_t h = h0; h < h1; ++h) {
            const uint32_t k0 = g * kGroup + h * kHalf;
            const uint32_t nblk = nb > k0 ? min(kHalf, nb - k0) : 0u;
            uint32_t run = 0;  // payload words of the unit so far
            if (nblk) {
                const uint32_t cnt = min(n - k0 * kBlock, nblk * kBlock);
                const uint32_t *src = a.ids + base + (uint64_t)k0 * kBlock;
                uint32_t *slot = a.p.slots + (uint64_t)t * kSlotWords;
                if (kGrp && !a.classes && cnt == kIds) {
                    run = enc_unit_r(src, ((uintptr_t)src & 15) == 0, lo, hi,
                                     a.mode == BFSC_SEL_PLAIN_BP ? kSelPlain : kSelExhaustive, nullptr,
                                     slot + kSlotDirWords + h * kSlotHalfWords, slot + 2 * h * kHalf, sid, lane, a.err);
                    if (lane == 0) a.p.unit_words[2 * t + h] = run;
                    continue;
                }
                const uint32_t cl = a.classes && lane < nblk ? (uint32_t)a.classes[bb + k0 + lane] : 0u;
                uint32_t va = 0, vb = 0;
                if constexpr (STAGE) {
                    uint32_t v[kPerLane];
#pragma unroll
                    for (uint32_t i = 0; i < kPerLane; ++i) v[i] = lane + 64 * i < cnt ? src[lane + 64 * i] : 0u;
#pragma unroll
                    for (uint32_t i = 0; i < kPerLane; ++i) sid[lane + 64 * i] = v[i];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                } else {
                    fetch_block(src, min(kBlock, cnt), lane, va, vb);
                }
                uint32_t *pay = slot + kSlotDirWords + h * kSlotHalfWords;
                uint32_t dirv = 0;  // lane 2k, 2k+1: directory entry of block k
                for (uint32_t kk = 0; kk < nblk; ++kk) {
                    const uint32_t nk = min(kBlock, cnt - kk * kBlock);
                    uint32_t na = 0, nbv = 0;
                    if constexpr (STAGE) {
                        va = sid[kk * kBlock + lane];
                        vb = sid[kk * kBlock + 64 + lane];
                    } else if (kk + 1 < nblk) {
                        fetch_block(src + (kk + 1) * kBlock, min(kBlock, cnt - (kk + 1) * kBlock), lane, na, nbv);
                    }
                    const int given = a.classes ? (int)readlane(cl, kk) : -1;
                    uint32_t *dst = pay + run, d0, d1;
                    run += nk == kBlock
                               ? enc_block<true, SCANPACK>(va, vb, nk, lo, hi, a.mode, given, d0, d1, dst, s_buf[w],
                                                           s_pj[SCANPACK ? w : 0], s_dj[SCANPACK ? w : 0], lane,
                                                           a.err)
                               : enc_block<false, SCANPACK>(va, vb, nk, lo, hi, a.mode, given, d0, d1, dst, s_buf[w],
                                                            s_pj[SCANPACK ? w : 0], s_dj[SCANPACK ? w : 0], lane,
                                                            a.err);
                    dirv = lane == 2 * kk ? d0 : lane == 2 * kk + 1 ? d1 : dirv;
                    if constexpr (!STAGE) {
                        va = na;
                        vb = nbv;
                    }
                }
                if (lane < 2 * nblk) slot[2 * h * kHalf + lane] = dirv;
            }
            if (lane == 0) a.p.unit_words[2 * t + h] = run;
        }
    }
}

// The eight fp16 features (block_features) of NP x 4 full blocks (NP = 2:
// a unit, 4: a tile), one block per 16-lane row in NP passes as in
// enc_unit_r: x[k][0..7] and the span of block k in span[k] (LDS).  The
// loads of every pass are issued before the first pass is worked on.  The
// statistics are the ones analyze_block computes for a block of 128 IDs.
// The IDs are not checked here: the row packer that follows checks the same
// words and reports a bad block (its stream is then void, whatever class was
// predicted).
template <uint32_t NP>
__device__ __forceinline__ void unit_features_r(const uint32_t *src, bool al16, uint32_t seg_n, int32_t level,
                                                uint16_t (*x)[kIn], uint32_t *span_out, uint32_t lane) {
    constexpr uint32_t m = kBlock - 1;
    const uint32_t ri = lane & 15, r = lane >> 4;
    const int32_t L = level < 0 ? 0 : (level > 63 ? 63 : level);
    uint32_t v[NP][8];
#pragma unroll
    for (uint32_t p = 0; p < NP; ++p) {
        const uint32_t *ps = src + 512 * p + 8 * lane;
        if (al16) {
            const uint4 x0 = ((const uint4 *)ps)[0], x1 = ((const uint4 *)ps)[1];
            v[p][0] = x0.x, v[p][1] = x0.y, v[p][2] = x0.z, v[p][3] = x0.w;
            v[p][4] = x1.x, v[p][5] = x1.y, v[p][6] = x1.z, v[p][7] = x1.w;
        } else {
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) v[p][k] = ps[k];
        }
    }
#pragma unroll
    for (uint32_t p = 0; p < NP; ++p) {
        const uint32_t pv = dpp<0x111>(v[p][0], v[p][7]);  // the row's first lane: its own first ID
        uint32_t dmax = v[p][0] - pv, dmin = ri ? v[p][0] - pv : 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t k = 1; k < 8; ++k) {
            dmax = max(dmax, v[p][k] - v[p][k - 1]);
            dmin = min(dmin, v[p][k] - v[p][k - 1]);
        }
        const uint32_t v0 = dpp<0x150>(v[p][0], v[p][0]), vl = dpp<0x15F>(v[p][7], v[p][7]);
        const uint32_t wmin = bitlen32(row_max(dmax)), mn = row_min(dmin), span = vl - v0;
        // lane ri of the row produces feature ri: the five bit-length
        // features share one conversion (a bit length over 32 is exact in
        // fp32 either way)
        const uint32_t bl = ri == 1 ? bitlen32(mn)
                            : ri == 2 ? wmin
                            : ri == 3 ? bitlen32(span / m)
                            : ri == 4 ? bitlen32(span)
                                      : bitlen32(seg_n);
        float fv = (float)bl * (1.0f / 32.0f);
        fv = ri == 0   ? 1.0f
             : ri == 5 ? __fdiv_rn((float)kBlock, (float)((uint64_t)span + 1ull))
             : ri == 6 ? (float)L / 64.0f
                       : fv;
        if (ri < 8) x[4 * p + r][ri] = f16bits(fv);
        if (ri == 0) span_out[4 * p + r] = span;
    }
}

// The network on a unit's blocks (sample k: block k < nblk, features
// x[k], the other samples zero): the predicted class of sample lane & 15.
__device__ __forceinline__ uint32_t unit_predict(const MlpMfma &W, const uint16_t (*x)[kIn], uint32_t nblk,
                                                 uint32_t lane) {
    half4_t xv = {(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
    const uint32_t smp = lane & 15;
    if (lane < 32 && smp < nblk) {
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[j] = __builtin_bit_cast(_Float16, x[smp][(lane >> 4) * 4 + j]);
    }
    float4_t z[3];
    // operand tiles are read from LDS here, not kept in registers across the
    // unit loop (that would cost 64 VGPRs of occupancy)
    __asm__ volatile("" ::: "memory");
    mlp16(W, xv, lane, z);
    return mlp16_argmax(z, lane);
}

// Pack pass with the learned choice fused in, one wave per unit.  The wave
// computes every block's eight fp16 features, evaluates the network for the
// unit's blocks at once on the matrix cores (block k is sample k, the other
// columns zero), resolves each prediction (bitmap if it is valid, bit-pack
// at the minimal width, PFOR at its best b, the exhaustive choice when the
// bitmap is invalid or a logit is NaN) and packs the blocks.  When there are
// enough tiles for every wave to get many, a unit is a whole tile and a tile
// of sixteen full blocks takes one evaluation for both halves (16 samples);
// otherwise a unit is half a tile.  The logits of a sample depend only on
// its own features, so the classes equal those of the separate selection
// pass.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 4) void k_enc_pack_l(EncArgs a) {
    constexpr uint32_t kIds = kHalf * kBlock;
    constexpr uint32_t kPerLane = kIds / 64;
    __shared__ MlpMfma s_w;
    // staged IDs (partial units) or the row encoder's payload area (full units)
    __shared__ __align__(16) uint32_t s_ids[WAVES][kUnitStage];
    __shared__ uint32_t s_buf[WAVES][132];
    __shared__ uint16_t s_x[WAVES][kGroup][kIn];
    __shared__ uint32_t s_span[WAVES][kGroup];
    __shared__ uint32_t s_wmin[WAVES][kHalf];
    __shared__ uint8_t s_sel[WAVES][kGroup];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = readfirst(tid >> 6);  // scalar wave index: units and tiles are scalar
    mlp_mfma_stage(&s_w, a.w, tid, WAVES * 64);
    __syncthreads();
    const uint32_t tiles = ldc(a.p.tile_base + a.nseg);
    const bool by_tile = (uint64_t)tiles >= 8ull * gridDim.x * WAVES;
    uint32_t *sid = s_ids[w];
    UnitRange ur = unit_range(by_tile ? tiles : 2 * tiles, WAVES, w, a.strided);
    // the tile's segment and its fields as in k_enc_pack_u
    uint64_t tsn = 0;  // (segment, its first tile) of a tile, as one word
    if (ur.begin < ur.end) tsn = ldc((const uint64_t *)(a.p.tile_seg + (by_tile ? ur.begin : ur.begin >> 1)));
    for (uint32_t u = ur.begin; u < ur.end; u += ur.step) {
        const uint32_t t = by_tile ? u : u >> 1;
        const uint32_t h0 = by_tile ? 0u : (u & 1), h1 = by_tile ? 2u : h0 + 1;  // the halves to pack
        const uint32_t r = (uint32_t)tsn, t_first = (uint32_t)(tsn >> 32);
        const uint32_t un = min(u + ur.step, ur.end - 1);
        tsn = ldc((const uint64_t *)(a.p.tile_seg + (by_tile ? un : un >> 1)));
        const uint32_t bb = ldc(a.p.blk_base + r), be = ldc(a.p.blk_base + r + 1);
        const uint32_t n = ldc(a.p.seg_n + r);
        const uint32_t lo = ldc(a.seg_lo + r), hi = ldc(a.seg_hi + r);
        const uint64_t base = ldc(a.seg_off + r);
        const int32_t level = a.seg_level ? ldc(a.seg_level + r) : 0;
        asm volatile("" ::"s"(bb), "s"(be), "s"(n), "s"(lo), "s"(hi), "s"(base), "s"(level));
        // a raw segment's IDs are copied by the place pass: no blocks
        const uint32_t nb = n < a.p.raw_below ? 0u : be - bb;
        const uint32_t g = t - t_first;
        if (by_tile && nb >= (g + 1) * kGroup && (uint64_t)(g + 1) * kGroup * kBlock <= n) {
            // sixteen full blocks: features of both halves, one evaluation of
            // the network, then the row packer on each half
            const uint32_t *src = a.ids + base + (uint64_t)g * kGroup * kBlock;
            const bool al16 = ((uintptr_t)src & 15) == 0;
            unit_features_r<4>(src, al16, n, level, s_x[w], s_span[w], lane);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const uint32_t pred = unit_predict(s_w, s_x[w], kGroup, lane);
            if (lane < kGroup) {
                const uint32_t sel = pred == 255u ? kSelExhaustive
                                     : pred == kClsBitmap ? (s_span[w][lane] <= kBitmapMaxSpan ? kSelBitmap
                                                                                              : kSelExhaustive)
                                     : pred <= 33u ? kSelPlain : kSelPfor;
                s_sel[w][lane] = (uint8_t)sel;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            uint32_t *slot = a.p.slots + (uint64_t)t * kSlotWords;
            for (uint32_t h = 0; h < 2; ++h) {
                const uint32_t run = enc_unit_r(src + h * kIds, al16, lo, hi, kSelExhaustive, s_sel[w] + kHalf * h,
                                                slot + kSlotDirWords + h * kSlotHalfWords, slot + 2 * h * kHalf, sid,
                                                lane, a.err);
                if (lane == 0) a.p.unit_words[2 * t + h] = run;
            }
            continue;
        }
        for (uint32_t h = h0; h < h1; ++h) {
            const uint32_t k0 = g * kGroup + h * kHalf;
            const uint32_t nblk = nb > k0 ? min(kHalf, nb - k0) : 0u;
            uint32_t run = 0;
            if (nblk) {
                const uint32_t cnt = min(n - k0 * kBlock, nblk * kBlock);
                const uint32_t *src = a.ids + base + (uint64_t)k0 * kBlock;
                if (cnt == kIds) {
                    // full unit: features and packing one block per 16-lane row
                    const bool al16 = ((uintptr_t)src & 15) == 0;
                    unit_features_r<2>(src, al16, n, level, s_x[w], s_span[w], lane);
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    const uint32_t pred = unit_predict(s_w, s_x[w], kHalf, lane);
                    // resolved selection of block lane (bitmap only when valid; NaN
                    // or an invalid bitmap: the exhaustive choice)
                    if (lane < kHalf) {
                        const uint32_t sel = pred == 255u ? kSelExhaustive
                                             : pred == kClsBitmap ? (s_span[w][lane] <= kBitmapMaxSpan ? kSelBitmap
                                                                                                      : kSelExhaustive)
                                             : pred <= 33u ? kSelPlain : kSelPfor;
                        s_sel[w][lane] = (uint8_t)sel;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    uint32_t *slot = a.p.slots + (uint64_t)t * kSlotWords;
                    run = enc_unit_r(src, al16, lo, hi, kSelExhaustive, s_sel[w],
                                     slot + kSlotDirWords + h * kSlotHalfWords, slot + 2 * h * kHalf, sid, lane,
                                     a.err);
                    if (lane == 0) a.p.unit_words[2 * t + h] = run;
                    continue;
                }
                uint32_t v[kPerLane];
    #pragma unroll
                for (uint32_t i = 0; i < kPerLane; ++i) v[i] = lane + 64 * i < cnt ? src[lane + 64 * i] : 0u;
    #pragma unroll
                for (uint32_t i = 0; i < kPerLane; ++i) sid[lane + 64 * i] = v[i];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // features of every block
                for (uint32_t kk = 0; kk < nblk; ++kk) {
                    const uint32_t nk = readfirst(min(kBlock, cnt - kk * kBlock));
                    const uint32_t va = sid[kk * kBlock + lane], vb = sid[kk * kBlock + 64 + lane];
                    BlockRegs R;
                    BlockStats S;
                    if (nk == kBlock)
                        analyze_block(va, vb, kBlock, lo, hi, lane, true, R, S, a.err);
                    else
                        analyze_block(va, vb, nk, lo, hi, lane, true, R, S, a.err);
                    if (lane == 0) s_wmin[w][kk] = S.wmin;
                    float f[8];
                    block_features(S, n, level, f);
                    float fv = f[0];
    #pragma unroll
                    for (int q = 1; q < 8; ++q) fv = lane == (uint32_t)q ? f[q] : fv;
                    if (lane < 8) s_x[w][kk][lane] = f16bits(fv);
                    if (lane == 0) s_span[w][kk] = S.span;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // the network on the unit's blocks
                const uint32_t pred = unit_predict(s_w, s_x[w], nblk, lane);
                // resolve and pack
                uint32_t *slot = a.p.slots + (uint64_t)t * kSlotWords;
                uint32_t *pay = slot + kSlotDirWords + h * kSlotHalfWords;
                uint32_t dirv = 0;  // lane 2k, 2k+1: directory entry of block k
                for (uint32_t kk = 0; kk < nblk; ++kk) {
                    const uint32_t nk = min(kBlock, cnt - kk * kBlock);
                    const uint32_t va = sid[kk * kBlock + lane], vb = sid[kk * kBlock + 64 + lane];
                    const uint32_t p = readlane(pred, kk);
                    const bool bitmap_ok = s_span[w][kk] <= kBitmapMaxSpan;
                    // resolved selection: -1 exhaustive, else the class to use
                    const int sel = p == 255u ? kSelExhaustive
                                    : p == kClsBitmap ? (bitmap_ok ? kSelBitmap : kSelExhaustive)
                                    : p <= 33u ? kSelPlain : kSelPfor;
                    uint32_t *dst = pay + run, d0, d1;
                    if (nk == kBlock) {
                        run += enc_full(va, vb, lo, hi, sel, d0, d1, dst, s_buf[w], lane, a.err, (int)s_wmin[w][kk]);
                    } else {
                        // the last block of a segment: the general routine with the
                        // resolved class (BP at the minimal width is what plain picks)
                        const int given = sel == kSelBitmap ? (int)kClsBitmap : sel == kSelPfor ? (int)kClsPfor : -1;
                        const int mode = sel == kSelPlain ? BFSC_SEL_PLAIN_BP : BFSC_SEL_EXHAUSTIVE;
                        run += enc_block<false, false>(va, vb, nk, lo, hi, mode, given, d0, d1, dst, s_buf[w], nullptr,
                                                       nullptr, lane, a.err);
                    }
                    dirv = lane == 2 * kk ? d0 : lane == 2 * kk + 1 ? d1 : dirv;
                }
                if (lane < 2 * nblk) slot[2 * h * kHalf + lane] = dirv;
            }
            if (lane == 0) a.p.unit_words[2 * t + h] = run;
        }
    }
}

// Unit sizes -> offsets, one workgroup per chunk of kScanChunk units (4 per
// thread, coalesced 16-byte loads and stores): the offsets within the chunk
// and the chunk's total.  The place pass adds the totals of the chunks before.
__global__ __launch_bounds__(1024) void k_enc_scan(EncArgs a) {
    __shared__ uint32_t s_tmp[17];
    const uint32_t units = 2 * readfirst(a.p.tile_base[a.nseg]);
    const uint32_t c0 = blockIdx.x * kScanChunk;
    if (c0 >= units) return;
    const uint32_t i0 = c0 + 4 * threadIdx.x;
    uint4 v = {0u, 0u, 0u, 0u};
    if (i0 + 4 <= units) {
        v = *(const uint4 *)(a.p.unit_words + i0);
    } else if (i0 < units) {
        v.x = a.p.unit_words[i0];
        v.y = i0 + 1 < units ? a.p.unit_words[i0 + 1] : 0u;
        v.z = i0 + 2 < units ? a.p.unit_words[i0 + 2] : 0u;
    }
    uint32_t total;
    const uint32_t ex = wg_excl_scan(v.x + v.y + v.z + v.w, s_tmp, &total);
    const uint4 o = {ex, ex + v.x, ex + v.x + v.y, ex + v.x + v.y + v.z};
    if (i0 + 4 <= units) {
        *(uint4 *)(a.p.unit_off + i0) = o;
    } else if (i0 < units) {
        a.p.unit_off[i0] = o.x;
        if (i0 + 1 < units) a.p.unit_off[i0 + 1] = o.y;
        if (i0 + 2 < units) a.p.unit_off[i0 + 2] = o.z;
    }
    if (threadIdx.x == 0) a.p.chunk_words[blockIdx.x] = total;
}

// Payload words of chunks k0 .. k1-1 (the whole wave).
__device__ __forceinline__ uint64_t chunk_prefix(const uint32_t *chunk_words, uint32_t k0, uint32_t k1, uint32_t lane) {
    uint64_t s = 0;
    for (uint32_t k = k0 + lane; k < k1; k += 64) s += chunk_words[k];
    return wave_sum64(s);
}

// Place pass, one wave per tile (tiles are independent, so every wave's
// chain of dependent loads runs in parallel with all others): the segment's
// start offset (written by its first tile), then for a compressed segment
// its header (first tile), the tile's directory entries, group-table entry
// and payload words, copied from the two halves of its slot to their final
// position; for a raw segment its IDs, copied from the input.  A wave waits
// on memory twice before its stores: for everything that depends on the
// tile index alone (the tile count, the tile's segment record, unit sizes
// and offset, and the payload totals of the chunks of units before it, four
// per lane), then for the segment's fields, the offset of its first unit,
// the directory and the payload words.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_enc_place(EncArgs a) {
    constexpr uint32_t kCw = 4;  // chunk totals held per lane
    const uint32_t lane = threadIdx.x & 63, w = readfirst(threadIdx.x >> 6);
    const uint32_t t = blockIdx.x * WAVES + w;
    if (t >= a.p.max_tiles) return;
    // first round: reads inside the plan's arrays for any t < max_tiles
    // (a tile past the batch's count reads stale words and drops them)
    const uint32_t total = a.p.tile_base[a.nseg];
    const uint2 ts = a.p.tile_seg[t];
    const uint32_t A0 = a.p.unit_words[2 * t], A1 = a.p.unit_words[2 * t + 1];
    const uint32_t ot = a.p.unit_off[2 * t];
    const uint32_t ct = 2 * t / kScanChunk;
    uint32_t cw[kCw];
#pragma unroll
    for (uint32_t i = 0; i < kCw; ++i) {
        const uint32_t k = lane + 64 * i;
        cw[i] = k < ct ? a.p.chunk_words[k] : 0u;
    }
    // every first-round value is needed here, so all of its loads are in
    // flight together before the one wait
    asm volatile("" ::"s"(total), "s"(ts.x), "s"(ts.y), "s"(A0), "s"(A1), "s"(ot), "v"(cw[0]), "v"(cw[1]),
                 "v"(cw[2]), "v"(cw[3]));
    if (t >= total) return;
    const uint64_t capw = a.out_cap >> 2;
    // second round: up to 512 payload words held in registers (every index
    // stays inside the tile's slot whatever the unit sizes read), the
    // directory words and the segment's fields
    const uint32_t *slot = a.p.slots + (uint64_t)t * kSlotWords;
    constexpr uint32_t kC = 8;
    const uint32_t nw = A0 + A1;
    auto src = [&](uint32_t q) {
        return q < A0 ? kSlotDirWords + q : kSlotDirWords + kSlotHalfWords + (q - A0);
    };
    uint32_t x[kC];
#pragma unroll
    for (uint32_t i = 0; i < kC; ++i) {
        const uint32_t q = lane + 64 * i;
        x[i] = q < nw ? slot[src(q)] : 0u;
    }
    const uint32_t dirw = lane < kSlotDirWords ? slot[lane] : 0u;
    const uint32_t r = ts.x;
    const uint32_t t_first = ts.y;
    const uint32_t n = a.p.seg_n[r];
    const uint32_t bb = a.p.blk_base[r];
    const uint32_t nb = a.p.blk_base[r + 1] - bb;
    const uint32_t gb = a.p.grp_base[r];
    const uint32_t ng = a.p.grp_base[r + 1] - gb;
    const uint32_t fb = a.p.fix_base[r];
    const uint32_t of = a.p.unit_off[2 * t_first];
    asm volatile("" ::"v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(x[4]), "v"(x[5]), "v"(x[6]), "v"(x[7]),
                 "v"(dirw));
    // payload words before the segment (chunks before cf, then units of
    // chunk cf before its first) and before the tile (chunks before ct)
    const uint32_t cf = 2 * t_first / kScanChunk;
    uint32_t sf = 0, st = 0;
#pragma unroll
    for (uint32_t i = 0; i < kCw; ++i) {
        st += cw[i];
        sf += lane + 64 * i < cf ? cw[i] : 0u;
    }
    uint64_t Pf = wave_sum(sf), Pc = wave_sum(st);  // 256 chunks of at most 2^22 words
    if (ct > 64 * kCw) {
        Pf += chunk_prefix(a.p.chunk_words, 64 * kCw, cf, lane);
        Pc += chunk_prefix(a.p.chunk_words, 64 * kCw, ct, lane);
    }
    const uint64_t P = Pf + of;
    const uint64_t Pt = Pc + ot;
    const uint64_t sw = (uint64_t)fb + gb + P;
    const uint32_t g = t - t_first;
    if (t == 0) {
        // the batch end, from the totals of all chunks
        const uint32_t units = 2 * total;
        const uint64_t words = chunk_prefix(a.p.chunk_words, 0, (units + kScanChunk - 1) / kScanChunk, lane);
        if (lane == 0) {
            const uint64_t end = 4ull * ((uint64_t)a.p.fix_base[a.nseg] + a.p.grp_base[a.nseg] + words);
            a.seg_byte_off[a.nseg] = end;
            if (end > a.out_cap) raise_err(a.err, kErrCapacity);
        }
    }
    if (g == 0 && lane == 0) a.seg_byte_off[r] = sw << 2;
    if (n == 0) return;
    if (n < a.p.raw_below) {
        // raw form: the IDs as they are (one tile per raw segment), checked
        // as the pack pass checks the others: strictly increasing, inside
        // [lo, hi)
        const uint32_t *ids = a.ids + a.seg_off[r];
        const uint32_t lo = readfirst(a.seg_lo[r]), hi = readfirst(a.seg_hi[r]);
        const bool fits = sw + n <= capw;
        bool bad = false;
        uint32_t carry = 0;
        for (uint32_t q0 = 0; q0 < n; q0 += 64) {
            const uint32_t q = q0 + lane;
            const bool in = q < n;
            const uint32_t v = in ? ids[q] : 0u;
            const uint32_t pv = pin(lane_prev(v, carry));
            bad |= in & ((v < lo) | (v >= hi) | ((q > 0) & (v <= pv)));
            if (in && fits) a.out[sw + q] = v;
            carry = readlane(v, 63);
        }
        if (lane == 0) {
            if (!fits) raise_err(a.err, kErrCapacity);
        }
        if (ballot(bad) != 0ull && lane == 0) raise_err(a.err, kErrInval);
        return;
    }
    if (g == 0 && lane < 4) {
        if (sw + 4 <= capw) {
            const uint32_t hv = lane == 0 ? n : lane == 1 ? a.seg_hi[r] : lane == 2 ? a.seg_lo[r] : kMagic;
            a.out[sw + lane] = hv;
        }
    }
    const uint32_t k0 = g * kGroup;
    const uint32_t nblk = nb > k0 ? min(kGroup, nb - k0) : 0u;
    if (!nblk) return;
    const uint64_t rel = Pt - P;
    const uint64_t pwb = sw + 4 + 2ull * nb + ng + rel;
    const uint64_t dwb = sw + 4 + 2ull * k0;
    if (pwb + A0 + A1 > capw || sw + 4 + 2ull * nb + ng > capw) {
        if (lane == 0) raise_err(a.err, kErrCapacity);
        return;
    }
    if (lane < 2 * nblk) a.out[dwb + lane] = dirw;
    if (lane == 0) a.out[sw + 4 + 2ull * nb + g] = (uint32_t)rel;
    // payload words q < A0 + A1 of the tile (half 0, then half 1): the first
    // 512 were loaded above, before any store (the stores may alias the slot
    // as far as the compiler knows), the rest in a loop
#pragma unroll
    for (uint32_t i = 0; i < kC; ++i) {
        const uint32_t q = lane + 64 * i;
        if (q < nw) a.out[pwb + q] = x[i];
    }
    for (uint32_t q = lane + 64 * kC; q < nw; q += 64) a.out[pwb + q] = slot[src(q)];
}

// ------------------------------------------------------------------ select / features

struct SelArgs {
    const uint32_t *ids;
    const uint64_t *seg_off;
    const uint32_t *seg_lo;
    const uint32_t *seg_hi;
    const int32_t *seg_level;
    uint32_t nseg;
    int mode;
    uint8_t *classes;
    uint16_t *feat;           // features out (may be NULL)
    uint64_t *fallbacks;
    const MlpMfma *w;         // the network in MFMA operand order (learned mode)
    Plan p;
    uint32_t *err;
    uint32_t literal;         // learned mode: keep a predicted width that holds the block
};

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_select(SelArgs a) {
    constexpr int BPW = (int)kGroup / WAVES;
    // learned mode: the network, and the tile's features (fp16 bits) and
    // the per-block facts that resolve needs
    __shared__ MlpMfma s_w;
    __shared__ uint16_t s_x[kGroup][kIn];
    __shared__ uint32_t s_wmin[kGroup], s_span[kGroup];
    __shared__ uint32_t s_ex[kGroup];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t total = a.p.tile_base[a.nseg];
    const bool learned = a.mode == BFSC_SEL_LEARNED;
    if (learned) {
        mlp_mfma_stage(&s_w, a.w, tid, WAVES * 64);
        __syncthreads();
    }
    __shared__ EncTile s_tm[kMetaChunk];
    const uint32_t G = gridDim.x;
    for (uint32_t base = blockIdx.x; base < total; base += G * kMetaChunk) {
    if (tid < kMetaChunk) {
        const uint32_t t = base + tid * G;
        if (t < total)
            s_tm[tid] = enc_tile_meta(a.p, a.seg_off, a.seg_lo, a.seg_hi, a.nseg, t, a.seg_level);
    }
    __syncthreads();
    for (uint32_t it = 0; it < kMetaChunk; ++it) {
        const uint32_t t = base + it * G;
        if (t >= total) break;
        const EncTile m = s_tm[it];
        const uint32_t nb = m.nb, n = m.n, lo = m.lo, hi = m.hi, bb = m.bb;
        const int32_t level = m.level;
        const uint32_t *ids = a.ids + m.id_base;
        const uint32_t g = m.g;
        const uint32_t k0 = g * kGroup;
        const uint32_t nblk = nb > k0 ? min(kGroup, nb - k0) : 0u;
        const uint32_t gb = bb + k0;
        uint32_t va[BPW], vb[BPW];
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            const uint32_t kk = w + (uint32_t)i * WAVES;
            const uint32_t k = k0 + kk;
            const uint32_t nk = kk < nblk ? min(kBlock, n - k * kBlock) : 0u;
            fetch_block(ids + (uint64_t)k * kBlock, nk, lane, va[i], vb[i]);
        }
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            const uint32_t kk = w + (uint32_t)i * WAVES;
            if (kk < nblk) {
                const uint32_t k = k0 + kk;
                const uint32_t nk = min(kBlock, n - k * kBlock);
                BlockRegs R;
                BlockStats S;
                const bool feats = a.feat || learned;
                analyze_block(va[i], vb[i], nk, lo, hi, lane, feats, R, S, a.err);
                if (feats) {
                    float f[8];
                    block_features(S, n, level, f);
                    if (lane < 8) {
                        float fv = f[0];
#pragma unroll
                        for (int q = 1; q < 8; ++q) fv = lane == (uint32_t)q ? f[q] : fv;
                        const uint16_t hb = f16bits(fv);
                        if (a.feat) a.feat[(uint64_t)(gb + kk) * 8 + lane] = hb;
                        s_x[kk][lane] = hb;
                    }
                }
                if (learned) {
                    // exhaustive class kept for the fallback
                    const BlockInfo ex = choose(R, S, BFSC_SEL_EXHAUSTIVE, -1, a.err);
                    if (lane == 0) {
                        s_wmin[kk] = S.wmin;
                        s_span[kk] = S.span;
                        s_ex[kk] = ex.cls;
                    }
                } else if (a.classes) {
                    const BlockInfo I = choose(R, S, a.mode, -1, a.err);
                    if (lane == 0) a.classes[gb + kk] = (uint8_t)I.cls;
                }
            }
        }
        if (!learned) continue;
        __syncthreads();
        // the network on the tile's blocks, one wave on the matrix cores
        // (block b is sample b; rows past the tile's blocks are zero)
        if (w == 0) {
            const uint32_t smp = lane & 15;
            half4_t x = {(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
            if (lane < 32 && smp < nblk) {
#pragma unroll
                for (int j = 0; j < 4; ++j) x[j] = __builtin_bit_cast(_Float16, s_x[smp][(lane >> 4) * 4 + j]);
            }
            float4_t z[3];
            mlp16(s_w, x, lane, z);
            const uint32_t best = mlp16_argmax(z, lane);
            if (lane < nblk) {
                const uint32_t bi = lane;
                uint32_t res;
                const uint32_t wmin = s_wmin[bi], span = s_span[bi];
                bool fb = false;
                if (best == 255u) {
                    fb = true;
                    res = s_ex[bi];
                } else if (best == kClsBitmap) {
                    if (span <= kBitmapMaxSpan) {
                        res = kClsBitmap;
                    } else {
                        fb = true;
                        res = s_ex[bi];
                    }
                } else if (best <= 33) {
                    if (!a.literal || best - 1u >= wmin) {
                        res = a.literal ? best : 1u + wmin;
                    } else {
                        fb = true;
                        res = s_ex[bi];
                    }
                } else {
                    res = kClsPfor;
                }
                if (a.classes) a.classes[gb + bi] = (uint8_t)res;
                if (fb && a.fallbacks) atomicAdd((unsigned long long *)a.fallbacks, 1ull);
            }
        }
        __syncthreads();
    }
    __syncthreads();  // s_tm is rewritten by the next chunk
    }
}

// ------------------------------------------------------------------ decode

// Workgroups of the block decoder per SIMD that its registers allow.
#ifndef DEC_OCC
#define DEC_OCC 6
#endif

struct DecPlanArgs {
    const uint8_t *in;
    const uint64_t *seg_byte_off;
    uint32_t nseg;
    uint64_t out_cap;
    uint64_t *out_off;
    uint32_t *seg_n;      // 0 for bad / empty
    uint32_t *seg_form;   // 0 empty or bad, 1 raw, 2 compressed
    uint32_t *tile_base;  // [nseg+1]
    uint64_t *chunk_n;    // [prep chunks] IDs of every kPrepChunk segments
    uint32_t *chunk_t;    // [prep chunks] tiles of every kPrepChunk segments
    uint32_t *tile_seg;   // [map_cap] segment of every tile (NULL: not kept)
    uint64_t map_cap;
    uint64_t max_ids;
    uint32_t *err;
};

// Tiles of a compressed segment of n IDs: groups of 16 blocks of 128.
__device__ __forceinline__ uint32_t dec_seg_tiles(uint32_t n) {
    const uint32_t nb = (n >> 7) + ((n & 127u) != 0u);
    return (nb >> 4) + ((nb & 15u) != 0u);
}

// The segment of every tile: tile_seg[tb + q] = r for q < ng.  A segment of
// up to 64 tiles is written by its own lane; longer ones by the whole wave,
// one after another, their tiles across the lanes.  Tiles at or past
// map_cap are not written (the decoder then searches instead).
__device__ __forceinline__ void dec_tile_map(const DecPlanArgs &a, uint32_t r, uint32_t tb, uint32_t ng,
                                             uint32_t lane) {
    const bool own = ng <= 64u;
    if (own)
        for (uint32_t q = 0; q < ng && (uint64_t)tb + q < a.map_cap; ++q) a.tile_seg[tb + q] = r;
    uint64_t m = ballot(!own);
    while (m) {
        const uint32_t j = (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        const uint32_t rj = readlane(r, j), tj = readlane(tb, j), nj = readlane(ng, j);
        for (uint32_t q = lane; q < nj && (uint64_t)tj + q < a.map_cap; q += 64) a.tile_seg[tj + q] = rj;
    }
}

// Pass 1 of the decoder's plan, one workgroup per kPrepChunk segments: each
// segment's form, ID count and tiles (a group of 16 blocks of a compressed
// segment, or the whole of a raw one), their exclusive scans inside the
// chunk, and the chunk's totals.  A segment of L bytes is empty if L = 0;
// raw if L < 16 or its words 1 and 2 increase (IDs strictly increase);
// compressed if they decrease (header n, hi, lo, magic with hi > lo).
// The batch totals at index nseg (tiles, output IDs) and the capacity check
// (against the output's capacity and against max_ids);
// with a single chunk the pass is complete and also writes the tile map.
__device__ __forceinline__ void dec_plan_end(const DecPlanArgs &a, uint32_t tiles, uint64_t ids) {
    a.tile_base[a.nseg] = tiles;
    a.out_off[a.nseg] = ids;
    if (ids > a.out_cap || ids > a.max_ids) raise_err(a.err, kErrCapacity);
}

__global__ __launch_bounds__(1024) void k_dec_local(DecPlanArgs a) {
    __shared__ uint32_t s_tmp[17];
    __shared__ unsigned long long s_w[16];
    __shared__ unsigned long long s_c;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6, c = blockIdx.x;
    const uint32_t r = c * kPrepChunk + tid;
    uint32_t n = 0, ng = 0;
    if (r < a.nseg) {
        const uint64_t s = a.seg_byte_off[r], e = a.seg_byte_off[r + 1];
        bool bad = e < s || (s & 3) || (e & 3);
        uint32_t form = 0;
        if (!bad && e > s) {
            const uint64_t L = e - s;
            const uint32_t *h = (const uint32_t *)(a.in + s);
            if (L < 16 || h[1] < h[2]) {
                bad = L / 4 > 0xFFFFFFFFull;
                n = (uint32_t)(L / 4);
                ng = 1;
                form = 1;
            } else {
                const uint32_t hn = h[0], hi = h[1], lo = h[2], mg = h[3];
                const uint64_t nb = (uint64_t)(hn >> 7) + ((hn & 127u) != 0u);
                const uint64_t meta = 16ull + 8ull * nb + 4ull * ((nb + kGroup - 1) / kGroup);
                bad = mg != kMagic || lo >= hi || hn == 0 || hn > hi - lo || meta > L;
                n = hn;
                ng = dec_seg_tiles(hn);
                form = 2;
            }
        }
        if (bad) {
            raise_err(a.err, kErrCorrupt);
            n = 0;
            ng = 0;
            form = 0;
        }
        a.seg_n[r] = n;
        a.seg_form[r] = form;
    }
    uint32_t tt;
    const uint32_t xt = wg_excl_scan(ng, s_tmp, &tt);
    // 64-bit exclusive scan of n (waves, then the workgroup)
    uint64_t incl = n;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t l2 = shfl_up((uint32_t)incl, d), h2 = shfl_up((uint32_t)(incl >> 32), d);
        if (lane >= (uint32_t)d) incl += ((uint64_t)h2 << 32) | l2;
    }
    if (lane == 63) s_w[w] = incl;
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
        a.tile_base[r] = xt;
        a.out_off[r] = s_w[w] + incl - n;
    }
    if (tid == 0) {
        a.chunk_t[c] = tt;
        a.chunk_n[c] = s_c;
        if (gridDim.x == 1) dec_plan_end(a, tt, s_c);  // one chunk: complete, no pass 2
    }
    if (gridDim.x == 1 && a.tile_seg) dec_tile_map(a, r, xt, ng, lane);
}

// Pass 2: adds the totals of the chunks before each chunk and writes the
// tile map; the last workgroup writes the batch totals at index nseg and
// checks the capacity.
__global__ __launch_bounds__(1024) void k_dec_fix(DecPlanArgs a) {
    __shared__ unsigned long long s_n[16];
    __shared__ uint32_t s_t[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6, c = blockIdx.x;
    uint64_t qn = 0;
    uint32_t qt = 0;
    for (uint32_t i = tid; i < c; i += blockDim.x) {
        qn += a.chunk_n[i];
        qt += a.chunk_t[i];
    }
    qn = wave_sum64(qn);
    qt = wave_sum(qt);
    if (lane == 0) {
        s_n[w] = qn;
        s_t[w] = qt;
    }
    __syncthreads();
    uint64_t pn = 0;
    uint32_t pt = 0;
    for (uint32_t i = 0; i < (blockDim.x >> 6); ++i) {
        pn += s_n[i];
        pt += s_t[i];
    }
    const uint32_t r = c * kPrepChunk + tid;
    uint32_t tb = 0, ng = 0;
    if (r < a.nseg) {
        tb = a.tile_base[r] + pt;
        a.tile_base[r] = tb;
        a.out_off[r] += pn;
        const uint32_t form = a.seg_form[r];
        ng = form == 1 ? 1u : form == 2 ? dec_seg_tiles(a.seg_n[r]) : 0u;
    }
    if (c + 1 == gridDim.x && tid == 0) dec_plan_end(a, pt + a.chunk_t[c], pn + a.chunk_n[c]);
    if (a.tile_seg) dec_tile_map(a, r, tb, ng, lane);
}

struct DecArgs {
    const uint8_t *in;
    const uint64_t *seg_byte_off;
    uint32_t nseg;
    const uint32_t *seg_n;
    const uint32_t *seg_form;
    const uint32_t *tile_base;
    const uint64_t *out_off;
    uint32_t *out;
    uint64_t out_cap;
    uint32_t *err;
    uint32_t strided;       // unit order of the staged decoder (else contiguous per wave)
    const uint32_t *tile_seg;  // segment of every tile (NULL: found by search)
    uint64_t map_cap;          // tiles the map holds
};

// w-bit field at bit pos of the staged words (funnel shift of two words).
__device__ __forceinline__ uint32_t get_field(const uint32_t *buf, uint32_t pos, uint32_t w) {
    const uint32_t wi = pos >> 5, sh = pos & 31;
    const uint32_t v = __builtin_amdgcn_alignbit(buf[wi + 1], buf[wi], sh);
    return w >= 32 ? v : (v & ((1u << w) - 1u));
}

__device__ __forceinline__ uint32_t block_words(uint32_t cls, uint32_t param, uint32_t aux, uint32_t m) {
    if (cls == kClsBitmap) return cdiv32(aux, 32);
    if (cls <= 33) return cdiv32(m * (cls - 1), 32);
    const uint32_t E = aux & 0xFFu;
    return cdiv32(m * param, 32) + cdiv32(E, 4) + cdiv32(E * (aux >> 8), 32);
}

// Whether a block's last ID, v0 + s (s < 2^32), reaches hi or the next
// block's first ID: in 32-bit scalar arithmetic, a sum that wraps being past
// both (each below 2^32).
__device__ __forceinline__ bool last_past(uint32_t v0, uint32_t s, uint32_t hi, bool has_next, uint32_t nxt) {
    const uint32_t l = v0 + s;
    return (l < v0) | (l >= hi) | (has_next & (l >= nxt));
}

// The IDs of one block (lane: xa = ID lane, xb = ID 64 + lane) and whether
// it passed every check; stores nothing.  FULL: a block of exactly 128 IDs,
// where every per-lane validity test folds away at compile time.
template <bool FULL>
__device__ __forceinline__ bool decode_vals(const uint32_t *buf, uint32_t bw, uint32_t *val, uint32_t cls,
                                            uint32_t param, uint32_t aux, uint32_t v0, uint32_t nk, uint32_t hi,
                                            bool has_next, uint32_t nxt, uint32_t lane, uint32_t &xa_out,
                                            uint32_t &xb_out) {
    if constexpr (FULL) {
        nk = kBlock;
        if (cls >= 2 && cls <= 25) {
            // bit-pack, width 1..24: 127 deltas sum to under 2^31, so the
            // 32-bit prefix sums cannot wrap; with every delta >= 1 the IDs
            // increase, and only the last one has to be checked (in 64 bits)
            const uint32_t w = cls - 1;
            const uint32_t da = lane ? get_field(buf, (lane - 1) * w, w) : 0u;
            const uint32_t db = get_field(buf, (63 + lane) * w, w);
            const uint64_t zero = ballot((lane != 0) & (da == 0u)) | ballot(db == 0u);
            const uint32_t sa = wave_incl_scan(da);
            const uint32_t sb = wave_incl_scan(db) + readlane(sa, 63);
            xa_out = v0 + sa;
            xb_out = v0 + sb;
            return !((zero != 0ull) | last_past(v0, readlane(sb, 63), hi, has_next, nxt));
        }
        if ((cls == kClsPfor) & (param + (aux >> 8) <= 24)) {
            // PFOR whose deltas have at most 24 bits (b low bits, h high bits
            // in the exceptions): as for the bit-pack case no prefix sum can
            // wrap, so with every delta >= 1 only the last ID is checked; the
            // exception positions are checked as always (inside the block,
            // strictly increasing)
            constexpr uint32_t m = kBlock - 1;
            const uint32_t b = param, E = aux & 0xFFu, h = aux >> 8;
            const uint32_t lw = cdiv32(m * b, 32), qw = cdiv32(E, 4);
            uint32_t da = ((lane != 0) & (b != 0)) ? get_field(buf, (lane - 1) * b, b) : 0u;
            uint32_t db = b ? get_field(buf, (63 + lane) * b, b) : 0u;
            val[lane] = 0u;
            val[lane + 64] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            uint32_t p = 0;
            if (lane < E) {
                p = (buf[lw + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu;
                const uint32_t hv = h ? get_field(buf + lw + qw, lane * h, h) : 0u;
                if (p < m) val[p + 1] = hv << b;
            }
            const uint32_t pp = lane_prev(p, 0u);
            const bool badx = (lane < E) & ((p >= m) | ((lane > 0) & (p <= pp)));
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            da |= val[lane];
            db |= val[lane + 64];
            const uint64_t bad = ballot(badx) | ballot((lane != 0) & (da == 0u)) | ballot(db == 0u);
            const uint32_t sa = wave_incl_scan(da);
            const uint32_t sb = wave_incl_scan(db) + readlane(sa, 63);
            xa_out = v0 + sa;
            xb_out = v0 + sb;
            return !((bad != 0ull) | last_past(v0, readlane(sb, 63), hi, has_next, nxt));
        }
    } else {
        nk = readfirst(nk);
    }
    const uint32_t m = nk - 1;
    bool bad = false;
    uint32_t xa = 0, xb = 0;
    const bool ina = lane < nk, inb = lane + 64 < nk;
    if (cls == kClsBitmap) {
        const uint32_t nch = (aux + 63) >> 6;
        uint32_t cnt = 1;
        if (lane == 0) val[0] = v0;
        // word 2c for lanes 0..31, 2c+1 for 32..63, read one step ahead and
        // unconditionally: wi + 2 <= 2 nch + 1 <= bw + 2, at most two words
        // past the block, still inside the staging buffer (132 words, or the
        // unit's words + 4); words past bw count as zero
        uint32_t wi = lane < 32 ? 0u : 1u;
        uint32_t rw = buf[wi];
        for (uint32_t c = 0; c < nch; ++c, wi += 2) {
            const uint32_t rn = buf[wi + 2];
            const uint32_t word = wi < bw ? rw : 0u;
            rw = rn;
            const bool set = (word >> (lane & 31)) & 1u;
            const uint64_t mk = ballot(set);
            // every lane stores (no exec-mask branch): a lane without a bit
            // writes its spare slot 128 + lane.  A damaged block may set more
            // than 127 bits: it is rejected below, and its writes stay inside val
            const uint32_t rk = pin(min(cnt + mbcnt64(mk), 127u));
            val[set ? rk : 128u + lane] = v0 + 64 * c + lane + 1;
            cnt += popc64(mk);
        }
        const uint32_t tailw = aux >> 5, tailb = aux & 31;
        bad |= tailb && lane == 0 && (buf[tailw] >> tailb) != 0u;
        bad |= cnt - 1 != m;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        xa = val[lane];
        xb = val[lane + 64];
        if (cnt - 1 == m) {
            const uint32_t lastv = m ? (nk <= 64 ? readlane(xa, nk - 1) : readlane(xb, nk - 65)) : v0;
            bad |= (uint64_t)v0 + (lastv - v0) >= (uint64_t)hi;
        }
    } else {
        const uint32_t b = cls <= 33 ? cls - 1 : param;
        const uint32_t ja = lane, jb = 64 + lane;
        uint32_t da = (ina && ja >= 1 && b) ? get_field(buf, (ja - 1) * b, b) : 0u;
        uint32_t db = (inb && b) ? get_field(buf, (jb - 1) * b, b) : 0u;
        if (cls == kClsPfor) {
            const uint32_t E = aux & 0xFFu, h = aux >> 8;
            const uint32_t lw = cdiv32(m * b, 32), qw = cdiv32(E, 4);
            val[lane] = 0u;
            val[lane + 64] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            uint32_t p = 0;
            if (lane < E) {
                p = (buf[lw + (lane >> 2)] >> (8 * (lane & 3))) & 0xFFu;
                const uint32_t hv = h ? get_field(buf + lw + qw, lane * h, h) : 0u;
                if (p < m) val[p + 1] = b >= 32 ? 0u : (hv << b);
            }
            const uint32_t pp = lane_prev(p, 0u);
            bad |= lane < E && (p >= m || (lane > 0 && p <= pp));
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            da |= val[lane];
            db |= val[lane + 64];
        }
        bad |= (ina && ja >= 1 && da == 0) || (inb && db == 0);
        const uint32_t sa = wave_incl_scan(da);
        const uint32_t ta = readlane(sa, 63);
        const uint32_t sb = wave_incl_scan(db) + ta;
        xa = v0 + sa;
        xb = v0 + sb;
        const uint32_t a63 = readlane(xa, 63);
        const uint32_t prva = lane_prev(xa, 0u);
        const uint32_t prvb = lane_prev(xb, a63);
        bad |= (ina && lane >= 1 && xa <= prva) || (inb && xb <= prvb);
    }
    const uint32_t last = nk <= 64 ? readlane(xa, nk - 1) : readlane(xb, nk - 65);
    bad |= last >= hi || (has_next && last >= nxt);
    xa_out = xa;
    xb_out = xb;
    return ballot(bad) == 0ull;
}

// Decodes and validates one block whose bw payload words start at buf (LDS;
// words past bw may hold anything and are never taken as payload); writes
// its IDs to out[ob ..] unless it is damaged.  val: 192 words of LDS (the
// block's IDs, then a spare slot per lane).
template <bool FULL>
__device__ __forceinline__ void decode_one_block(const uint32_t *buf, uint32_t bw, uint32_t *val,
                                                 uint32_t cls, uint32_t param, uint32_t aux,
                                                 uint32_t v0, uint32_t nk, uint32_t hi, bool has_next,
                                                 uint32_t nxt, uint32_t *out, uint64_t ob,
                                                 uint64_t out_cap, uint32_t *err, uint32_t lane) {
    uint32_t xa, xb;
    if (!decode_vals<FULL>(buf, bw, val, cls, param, aux, v0, nk, hi, has_next, nxt, lane, xa, xb)) {
        if (lane == 0) raise_err(err, kErrCorrupt);
    } else if (FULL && ob + kBlock <= out_cap) {  // uniform: unmasked stores
        out[ob + lane] = xa;
        out[ob + 64 + lane] = xb;
    } else {
        const uint32_t n = FULL ? kBlock : readfirst(nk);
        if (lane < n && ob + lane < out_cap) out[ob + lane] = xa;
        if (lane + 64 < n && ob + 64 + lane < out_cap) out[ob + 64 + lane] = xb;
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void decode_block(const uint32_t *buf, uint32_t bw, uint32_t *val, uint32_t cls,
                                             uint32_t param, uint32_t aux, uint32_t v0, uint32_t nk,
                                             uint32_t hi, bool has_next, uint32_t nxt, uint32_t *out,
                                             uint64_t ob, uint64_t out_cap, uint32_t *err, uint32_t lane) {
    if (nk == kBlock)
        decode_one_block<true>(buf, bw, val, cls, param, aux, v0, nk, hi, has_next, nxt, out, ob, out_cap,
                               err, lane);
    else
        decode_one_block<false>(buf, bw, val, cls, param, aux, v0, nk, hi, has_next, nxt, out, ob, out_cap,
                                err, lane);
}

// ds_write_b32 of v to LDS byte address addr on the lanes of mask only: exec
// is narrowed for the one store and restored inside the same asm block, so
// the compiler never sees a changed exec (no per-lane test of the bit is
// needed).  The store has no result register.
__device__ __forceinline__ void lds_store_lanes(uint32_t addr, uint32_t v, uint64_t mask) {
    uint64_t save;
    asm volatile(
        "s_and_saveexec_b64 %0, %3\n\t"
        "ds_write_b32 %1, %2\n\t"
        "s_mov_b64 exec, %0"
        : "=&s"(save)
        : "v"(addr), "v"(v), "s"(mask)
        : "memory");
}

// LDS byte address of a pointer into a __shared__ array.
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// Chunk c (64 bits: words wi, wi + 1 of a bitmap held one word per lane in
// src) of a full bitmap block: every lane whose bit is set writes its ID
// (vl + 64 c, vl = v0 + 1 + lane) at its rank, cnt + the set bits below it.
// The chunk's two words come to scalar registers, so the mask, the count
// and the loop are scalar work; each lane spends two mbcnt, an address and a
// value on it.  vbase: LDS byte address of the wave's val array (uniform).
// A damaged block may hold more than 127 bits: the rank base is clamped at
// 128, so such chunks land in val[128 .. 191] and the block is rejected by
// its count.
__device__ __forceinline__ void bitmap_chunk(uint32_t src, uint32_t wi, uint32_t vl, uint32_t &cnt,
                                             uint32_t vbase) {
    const uint32_t lo = readlane(src, wi), hi = readlane(src, wi + 1);
    const uint64_t mk = ((uint64_t)hi << 32) | lo;
    const uint32_t rk = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
    uint32_t b4 = vbase + 4 * min(cnt, kBlock);
    asm("" : "+s"(b4));  // kept scalar: one v_lshl_add per lane for the address
    lds_store_lanes(b4 + 4 * rk, vl, mk);
    cnt += popc64(mk);
}

// A full bitmap block (128 IDs) decoded from its payload words in registers
// (lane i: word i in px, word 64 + i in py, zero past the block's words), so
// it is never staged in LDS.  Checks as for every block: the set bits number
// m = 127, none lies past the span (aux), the last ID is below hi and below
// the next block's first.  val: 192 words of the wave's LDS.  Returns false
// (nothing written) for a damaged block.
__device__ __forceinline__ bool dec_bitmap_full(uint32_t px, uint32_t py, uint32_t aux, uint32_t v0, uint32_t hi,
                                                bool has_next, uint32_t nxt, uint32_t *val, uint32_t *out,
                                                uint64_t ob, uint64_t out_cap, uint32_t lane) {
    const uint32_t nch = (aux + 63) >> 6;  // 64-bit chunks
    const uint32_t vbase = readfirst(lds_addr(val));
    if (lane == 0) val[0] = v0;
    uint32_t cnt = 1;
    const uint32_t n1 = min(nch, 32u);
    const uint32_t vl = v0 + 1 + lane;
    for (uint32_t c = 0; c < n1; c += 2) {
        bitmap_chunk(px, 2 * c, vl + 64 * c, cnt, vbase);
        bitmap_chunk(px, (2 * c + 2) & 63, vl + 64 * c + 64, cnt, vbase);
    }
    for (uint32_t c = 32; c < nch; c += 2) {
        bitmap_chunk(py, 2 * c - 64, vl + 64 * c, cnt, vbase);
        bitmap_chunk(py, (2 * c - 62) & 63, vl + 64 * c + 64, cnt, vbase);
    }
    // (the second chunk of a pair past the span reads words that are zero:
    // words past the block's own are not loaded, and chunk pairs never pass
    // word 127 because 2 nch <= 128)
    const uint32_t tailw = aux >> 5, tailb = aux & 31;
    const uint32_t tw = readlane(tailw < 64 ? px : py, tailw & 63);
    bool bad = cnt != kBlock || (tailb != 0 && (tw >> tailb) != 0u);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t xa = val[lane], xb = val[lane + 64];
    if (!bad) {
        const uint32_t last = readlane(xb, 63);
        bad = (uint64_t)v0 + (last - v0) >= (uint64_t)hi || (has_next && last >= nxt);
    }
    if (!bad) {
        if (ob + kBlock <= out_cap) {
            out[ob + lane] = xa;
            out[ob + 64 + lane] = xb;
        } else {
            if (ob + lane < out_cap) out[ob + lane] = xa;
            if (ob + 64 + lane < out_cap) out[ob + 64 + lane] = xb;
        }
    }
    __builtin_amdgcn_wave_barrier();
    return !bad;
}

// One 64-bit chunk (words lo, hi) of a full bitmap block: every lane whose
// bit is set writes its ID idv at its rank, the set bits below it plus the
// rank base.  cb is the base as an LDS byte address (one word per rank) and
// is advanced by the chunk's bits; writes are clamped at cap (rank 128), so
// a damaged block holding more bits lands in the 64 spare slots after it and
// is rejected by its count.  The mask, the count and the base stay scalar;
// each lane spends two mbcnt, an address and the store.
__device__ __forceinline__ void bitmap_chunk_s(uint32_t lo, uint32_t hi, uint32_t idv, uint32_t &cb,
                                               uint32_t cap) {
    const uint64_t mk = ((uint64_t)hi << 32) | lo;
    const uint32_t rk = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
    uint32_t b4 = min(cb, cap);
    asm("" : "+s"(b4));  // kept scalar: one v_lshl_add per lane for the address
    lds_store_lanes(b4 + 4 * rk, idv, mk);
    cb += 4 * popc64(mk);
}

// A full bitmap block's IDs into val[0 .. 127] from its wc payload words at
// bm (LDS; the words after them belong to the next block and are not read):
// two chunks per step from four words, then the one or two chunks left.
// vbase: LDS byte address of val.  Returns the number of IDs (128 when the
// block is sound).
__device__ __forceinline__ uint32_t bitmap_expand_lds(const uint32_t *bm, uint32_t wc, uint32_t v0,
                                                      uint32_t vbase, uint32_t lane) {
    uint32_t cb = vbase + 4;  // val[0] is the first ID
    const uint32_t cap = vbase + 4 * kBlock;
    uint32_t idv = v0 + 1 + lane;
    uint32_t q = wc;
    const uint32_t *bp = bm;
    for (; q >= 4; q -= 4, bp += 4, idv += 128) {
        const uint32_t w0 = readfirst(bp[0]), w1 = readfirst(bp[1]);
        const uint32_t w2 = readfirst(bp[2]), w3 = readfirst(bp[3]);
        bitmap_chunk_s(w0, w1, idv, cb, cap);
        bitmap_chunk_s(w2, w3, idv + 64, cb, cap);
    }
    if (q >= 2) {
        bitmap_chunk_s(readfirst(bp[0]), readfirst(bp[1]), idv, cb, cap);
        q -= 2;
        bp += 2;
        idv += 64;
    }
    if (q) bitmap_chunk_s(readfirst(bp[0]), 0u, idv, cb, cap);
    return (cb - vbase) >> 2;
}

// The full-unit path of the decoder: NB blocks of 128 IDs (a whole group
// of 16, or half of one) whose output lies inside the buffer and whose
// payload (Au words from pu, at most 1,021) fits the wave's LDS window.  The
// payload is copied into LDS by the memory unit (global_load_lds, 16 bytes
// per lane, starting at the 16-byte boundary at or below pu, so no load
// touches a page the payload does not: the words of the unit start at win +
// delta) with every load in flight at once.  Each block's directory fields
// come to scalar registers (lane j of e1v / firstv / offv: block j of the
// group, offsets relative to the unit's first payload word; lane hb + NB of
// firstv: the next block's first, when has_last_next).  Full bitmap blocks
// are expanded from the staged words with scalar chunk masks, the other
// classes by decode_vals.  (Stores through a buffer resource over the unit's
// output were tried: with whole groups they wrote 1.2x and fetched 1.8x the
// bytes that plain stores do, and took 1.20 against 1.07 ms at scale 26.)
__device__ __forceinline__ void dec_full_unit(uint32_t NB, const uint32_t *pu, uint32_t Au, uint32_t *win,
                                              uint32_t *val, uint32_t e1v, uint32_t firstv, uint32_t offv, uint32_t hb,
                                              uint32_t lo, uint32_t hi, bool has_last_next, uint32_t *dst,
                                              uint32_t *err, uint32_t lane) {
    const uint32_t delta = (uint32_t)(((uintptr_t)pu & 15) >> 2);
    const uint32_t last = (delta + Au - 1) >> 2;  // last 16-byte chunk holding payload (Au >= 1)
    const uint32_t *base = pu - delta;
    asm volatile("" ::: "memory");  // earlier LDS reads of win are done before it is overwritten
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i)
        if (64 * i <= last)
            __builtin_amdgcn_global_load_lds((const void *)(base + 4 * (min(lane, last - 64 * i) + 64 * i)),
                                             (__attribute__((address_space(3))) void *)(win + 256 * i), 16, 0, 0);
    // vmcnt(0) (expcnt and lgkmcnt left at their maxima), as a builtin so that
    // the compiler's wait bookkeeping knows the copy into LDS has landed and
    // puts no further waits for it before the LDS reads below
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_wave_barrier();
    const uint32_t *pw = win + delta;
    const uint32_t vbase = readfirst(lds_addr(val));
    for (uint32_t kk = 0; kk < NB; ++kk) {
        const uint32_t j = hb + kk;
        const uint32_t e1 = readlane(e1v, j), v0 = lo + readlane(firstv, j), o = readlane(offv, j);
        const bool has_next = kk + 1 < NB || has_last_next;
        const uint32_t nxt = lo + readlane(firstv, j + 1);
        const uint32_t cls = e1 & 0xFFu, aux = e1 >> 16;
        const uint32_t *bm = pw + o;
        uint32_t xa = 0, xb = 0;
        bool ok;
        if (cls == kClsBitmap) {
            if (lane == 0) val[0] = v0;
            const uint32_t cnt = bitmap_expand_lds(bm, (aux + 31) >> 5, v0, vbase, lane);
            const uint32_t tailw = aux >> 5, tailb = aux & 31;
            ok = cnt == kBlock && (tailb == 0 || (readfirst(bm[tailw]) >> tailb) == 0u);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            xa = val[lane];
            xb = val[lane + 64];
            if (ok) ok = !last_past(v0, readlane(xb, 63) - v0, hi, has_next, nxt);
        } else {
            ok = decode_vals<true>(bm, 0u, val, cls, (e1 >> 8) & 0xFFu, aux, v0, kBlock, hi, has_next, nxt, lane,
                                   xa, xb);
        }
        // a scalar branch, both sides uniform (the compiler issues the
        // atomic from one lane)
        if (readfirst(ok ? 1u : 0u)) {
            dst[kk * kBlock + lane] = xa;
            dst[kk * kBlock + 64 + lane] = xb;
        } else {
            raise_err(err, kErrCorrupt);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// A block's payload words (wc of them, at word o of the segment's payload
// area) into lane / 64+lane.  Only the block's own words are read: reading
// whole 512-byte windows pulled the next units' lines into this XCD's L2 as
// well: over twice the stream's bytes in fetches.
__device__ __forceinline__ void load_payload(const uint32_t *pay, uint32_t o, uint32_t wc, uint32_t lane,
                                             uint32_t &x, uint32_t &y) {
    x = lane < wc ? pay[o + lane] : 0u;
    y = lane + 64 < wc ? pay[o + 64 + lane] : 0u;
}

// A full unit (8 blocks of 128 IDs) decoded in two passes of four blocks,
// one block per 16-lane row: lane i of row r produces IDs 8i .. 8i+7 of
// group block jr = hb + 4p + r in pass p.  The group's checked directory is
// held one block per lane (e1: class | param << 8 | aux << 16; first; off:
// payload word offset; lane gblk holds the next block's first value).  win:
// the unit's staged payload words, from payload word ub; val: 512 words of
// the wave's LDS.  Bit-pack fields (and PFOR low parts) are taken from a
// 64-bit window per lane for widths <= 4, else field by field; PFOR
// exceptions are patched through val; a bitmap is expanded one word per
// lane per step (popcount, row scan for the ranks, then the lane writes its
// set bits' IDs into val).  The prefix sums run inside the lane and then as
// a row scan.  A block that fails a check is reported and not written.
__device__ __forceinline__ void dec_unit_r(const uint32_t *win, uint32_t *val, uint32_t ub, uint32_t hb,
                                           uint32_t k0, uint32_t nb, uint32_t e1, uint32_t first, uint32_t off,
                                           uint32_t lo, uint32_t hi, uint32_t *out, uint64_t oo,
                                           uint64_t out_cap, uint32_t *err, uint32_t lane) {
    constexpr uint32_t m = kBlock - 1;
    const uint32_t ri = lane & 15, r = lane >> 4;
    uint32_t *const vr = val + 128 * r;
    // whole unit inside the output and 16-byte aligned: two vector stores
    // per lane
    const bool vec = (oo & 3) == 0 && ((uintptr_t)out & 15) == 0 &&
                     oo + (uint64_t)(k0 + hb + kHalf) * kBlock <= out_cap;
#pragma unroll 1
    for (uint32_t p = 0; p < 2; ++p) {
        const uint32_t jr = hb + 4 * p + r;
        const uint32_t me = shfl(e1, (int)jr), mo = shfl(off, (int)jr);
        const uint32_t mf = shfl(first, (int)jr), mn = shfl(first, (int)jr + 1);
        const uint32_t cls = me & 0xFFu, param = (me >> 8) & 0xFFu, aux = me >> 16;
        const uint32_t *buf = win + (mo - ub);
        const uint32_t v0 = lo + mf, nxt = lo + mn;
        const bool hasnx = k0 + jr + 1 < nb;
        const bool isbm = cls == kClsBitmap, ispf = cls == kClsPfor;
        const uint32_t b = isbm ? 0u : cls <= 33 ? cls - 1 : param;
        const uint32_t mask = b >= 32 ? 0xFFFFFFFFu : (1u << b) - 1u;
        const bool has0 = ri != 0;  // the lane's first slot carries a delta
        bool bad = false;
        uint32_t x[8];
        // deltas of a bit-pack / PFOR low part: delta j is field j-1 at bit
        // (j-1) b; delta 0 of the block is 0 (its first ID is v0)
        const uint32_t p0 = has0 ? (8 * ri - 1) * b : 0u;
        {
            const uint32_t wi = p0 >> 5;
            const uint64_t wv = ((uint64_t)buf[wi + 1] << 32) | buf[wi];
            uint32_t rel = (p0 & 31) - (has0 ? 0u : b);
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) {
                x[k] = (k != 0 || has0) ? (uint32_t)(wv >> (rel & 63)) & mask : 0u;
                rel += b;
            }
        }
        if (ballot(b > 4) != 0ull) {
            uint32_t pos = p0;
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) {
                if (k != 0 || has0) {
                    const uint32_t wi = pos >> 5;
                    const uint32_t f = __builtin_amdgcn_alignbit(buf[wi + 1], buf[wi], pos & 31) & mask;
                    x[k] = b > 4 ? f : x[k];
                    pos += b;
                }
            }
        }
        if (ballot(ispf) != 0ull) {
            // exception e < E (one lane each): position byte p_e, high part;
            // delta p_e + 1 gets hv << b
            const uint32_t E = ispf ? aux & 0xFFu : 0u, h = aux >> 8;
            const uint32_t lw = cdiv32(m * b, 32), qw = cdiv32(E, 4);
            *(uint4 *)&vr[8 * ri] = make_uint4(x[0], x[1], x[2], x[3]);
            *(uint4 *)&vr[8 * ri + 4] = make_uint4(x[4], x[5], x[6], x[7]);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const bool ex = ri < E;
            const uint32_t pe = ex ? (buf[lw + (ri >> 2)] >> (8 * (ri & 3))) & 0xFFu : 0u;
            const uint32_t pp = pin(dpp<0x111>(0u, pe));
            bad |= ex && (pe >= m || (ri > 0 && pe <= pp));
            if (ex && pe < m) {
                const uint32_t hv = h ? get_field(buf + lw + qw, ri * h, h) : 0u;
                atomicOr(&vr[pe + 1], b >= 32 ? 0u : hv << b);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const uint4 y0 = *(const uint4 *)&vr[8 * ri], y1 = *(const uint4 *)&vr[8 * ri + 4];
            x[0] = y0.x, x[1] = y0.y, x[2] = y0.z, x[3] = y0.w;
            x[4] = y1.x, x[5] = y1.y, x[6] = y1.z, x[7] = y1.w;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        // prefix sums: inside the lane, then across the row
        {
            uint32_t s = 0;
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) {
                bad |= !isbm & (k != 0 || has0) & (x[k] == 0u);
                s += x[k];
                x[k] = s;
            }
            const uint32_t base = v0 + row_excl_scan(s);
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) x[k] += base;
        }
        if (ballot(isbm) != 0ull) {
            // bitmap: bit q set means ID v0 + q + 1; exactly m bits, none at or
            // past bit aux (the span), read only inside the block's words
            const uint32_t bw = isbm ? cdiv32(aux, 32) : 0u;
            if (ri == 0) vr[0] = v0;
            uint32_t cnt = 1;  // IDs placed so far in the row's block
            const uint32_t nsteps = readfirst(max(wave_max(bw), 1u) + 15) >> 4;
            for (uint32_t st = 0; st < nsteps; ++st) {
                const uint32_t wi = 16 * st + ri;
                uint32_t word = wi < bw ? buf[wi] : 0u;
                if (wi + 1 == bw && (aux & 31)) {
                    bad |= (word >> (aux & 31)) != 0u;
                    word &= (1u << (aux & 31)) - 1u;
                }
                const uint32_t c = __builtin_popcount(word);
                uint32_t rank = cnt + row_excl_scan(c);
                cnt += row_sum(c);
                const uint32_t idb = v0 + 32 * wi + 1;
                while (word) {
                    const uint32_t bit = __builtin_ctz(word);
                    vr[min(rank, 127u)] = idb + bit;
                    ++rank;
                    word &= word - 1u;
                }
            }
            bad |= isbm & (cnt != kBlock);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const uint4 y0 = *(const uint4 *)&vr[8 * ri], y1 = *(const uint4 *)&vr[8 * ri + 4];
            if (isbm) {
                x[0] = y0.x, x[1] = y0.y, x[2] = y0.z, x[3] = y0.w;
                x[4] = y1.x, x[5] = y1.y, x[6] = y1.z, x[7] = y1.w;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        // strictly increasing (this also catches a wrapped sum), the last ID
        // below hi and below the next block's first
        const uint32_t px = pin(dpp<0x111>(0u, x[7]));
        bad |= has0 & (x[0] <= px);
#pragma unroll
        for (uint32_t k = 1; k < 8; ++k) bad |= x[k] <= x[k - 1];
        const uint32_t last = dpp<0x15F>(x[7], x[7]);
        const uint64_t last64 = (uint64_t)v0 + (last - v0);
        bad |= (last64 >= hi) | (hasnx & (last64 >= nxt));
        // a row is bad when any of its lanes is
        const uint64_t bm = ballot(bad);
        const bool rowbad = ((bm >> (16 * r)) & 0xFFFFull) != 0ull;
        if (bm != 0ull) {
            if (lane == 0) raise_err(err, kErrCorrupt);
        }
        const uint64_t ob = oo + (uint64_t)(k0 + jr) * kBlock + 8 * ri;
        if (!rowbad) {
            if (vec) {
                *(uint4 *)(out + ob) = make_uint4(x[0], x[1], x[2], x[3]);
                *(uint4 *)(out + ob + 4) = make_uint4(x[4], x[5], x[6], x[7]);
            } else {
#pragma unroll
                for (uint32_t k = 0; k < 8; ++k)
                    if (ob + k < out_cap) out[ob + k] = x[k];
            }
        }
    }
}

// A raw segment: its n words are the IDs, which must strictly increase;
// the wave copies them 64 at a time.
__device__ __forceinline__ void dec_raw(const uint32_t *src, uint32_t n, uint32_t *out, uint64_t ob,
                                        uint64_t out_cap, uint32_t *err, uint32_t lane) {
    uint32_t carry = 0;
    bool bad = false;
    for (uint32_t q0 = 0; q0 < n; q0 += 64) {
        const uint32_t q = q0 + lane;
        const bool in = q < n;
        const uint32_t v = in ? src[q] : 0xFFFFFFFFu;
        const uint32_t pv = pin(lane_prev(v, carry));
        bad |= in & (q > 0) & (v <= pv);
        if (in && ob + q < out_cap) out[ob + q] = v;
        carry = readlane(v, 63);
    }
    if (ballot(bad) != 0ull && lane == 0) raise_err(err, kErrCorrupt);
}

// Decode, one wave per unit.  The wave reads and checks the group's
// directory entries (one lane per block) and table words, then decodes the
// unit's blocks in order.  STAGE: a unit is half a group (up to 8 blocks)
// whose payload words (at most 1024, since every block holds at most 128)
// are first staged in LDS with every load in flight at once.  Otherwise a
// unit is a whole group (GROUP, chosen by the launcher when every wave gets
// many) or half of one: sixteen full blocks whose payload fits the LDS
// window are decoded in one go (dec_full_unit), any other group half by
// half; a full half that fits goes to dec_full_unit, any other block by
// block, the next block's words in flight while the current one decodes.
// Whole groups read and check each directory entry once.
template <int WAVES, bool STAGE, bool GROUP, bool MAP>
__global__ __launch_bounds__(WAVES * 64, DEC_OCC) void k_decode_u(DecArgs a) {
    constexpr uint32_t kWin = kHalf * kBlock;
    constexpr uint32_t kPerLane = kWin / 64;
    __shared__ uint32_t s_win[WAVES][kWin + 4];
    __shared__ uint32_t s_val[WAVES][192];  // 128 IDs, 64 spare slots
    // (a scalar wave index, which makes units, tiles and groups scalar
    // values, moves address and loop arithmetic onto the scalar unit that
    // the block loop keeps busy: 0.96 against 0.89 ms at scale 26)
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t tiles = ldc(a.tile_base + a.nseg);
    constexpr bool by_group = GROUP && !STAGE;
    uint32_t *win = s_win[w];
    uint32_t *val = s_val[w];
    UnitRange ur = unit_range(by_group ? tiles : 2 * tiles, WAVES, w, a.strided);
    // The segment of the wave's next unit is found while the current one
    // decodes: from the plan's tile map (MAP), else by search.  Nothing about
    // the segment is carried from one unit to the next (its fields are
    // loaded again, from the cache), so that they all stay scalar values to
    // the compiler.  The plan, the map and the stream's headers and group
    // table come by scalar loads: the wave waits on them without waiting for
    // its stores of the unit before.  A batch of more tiles than the map
    // holds claims more than max_ids IDs, which the plan has reported: it is
    // not decoded.
    if (MAP && tiles > a.map_cap) return;
    auto seg_of = [&](uint32_t uu) -> uint32_t {
        const uint32_t tt = by_group ? uu : uu >> 1;
        if constexpr (MAP) return ldc(a.tile_seg + tt);
        else return wave_find(a.tile_base, a.nseg, tt, lane);
    };
    uint32_t rn = ur.begin < ur.end ? seg_of(ur.begin) : 0u;
    for (uint32_t u = ur.begin; u < ur.end; u += ur.step) {
        const uint32_t t = by_group ? u : u >> 1;
        const uint32_t h0 = by_group ? 0u : (u & 1), h1 = by_group ? 2u : h0 + 1;  // the halves to decode
        // this unit's segment, and the next one's (the last unit's again at
        // the end: the load is unconditional, so that it stays in flight)
        const uint32_t r = rn;
        rn = seg_of(min(u + ur.step, ur.end - 1));
        const uint32_t t_first = ldc(a.tile_base + r);
        const uint32_t n = ldc(a.seg_n + r);
        const uint32_t form = ldc(a.seg_form + r);
        const uint64_t S = ldc(a.seg_byte_off + r);
        const uint64_t bytes = ldc(a.seg_byte_off + r + 1) - S;
        const uint64_t oo = ldc(a.out_off + r);
        asm volatile("" ::"s"(t_first), "s"(n), "s"(form), "s"(S), "s"(bytes), "s"(oo));  // one round
        const uint32_t *seg = (const uint32_t *)(a.in + S);
        if (form != 2) {
            // a raw segment's one tile (empty segments have none)
            if (h0 == 0) dec_raw(seg, n, a.out, oo, a.out_cap, a.err, lane);
            continue;
        }
        const uint32_t g = t - t_first;
        const uint32_t nb = cdiv32(n, kBlock), ng = cdiv32(nb, kGroup);
        const uint32_t k0 = g * kGroup;
        const uint32_t gblk = min(kGroup, nb - k0);
        if (h0 * kHalf >= gblk) continue;
        const uint32_t metaw = 4 + 2 * nb + ng;
        const uint64_t availw = bytes / 4 - metaw;
        // one round of loads: the header's bounds and the group-table entries
        // (scalar), the directory entries (lane i < gblk: block k0+i of the
        // group; lane gblk: the next block's first value)
        const uint32_t hi = ldc(seg + 1), lo = ldc(seg + 2);
        const bool last_g = g + 1 >= ng;
        const uint32_t gt = ldc(seg + 4 + 2 * nb + g);
        const uint32_t gtn = last_g ? 0u : ldc(seg + 4 + 2 * nb + g + 1);
        uint32_t first = 0, e1v = 0;
        if (lane <= gblk && k0 + lane < nb) {
            first = seg[4 + 2 * (k0 + lane)];
            e1v = seg[4 + 2 * (k0 + lane) + 1];
        }
        // the round lands here on every path (no load left in flight into
        // the next unit, where a register's reuse would wait for all stores)
        asm volatile("" ::"v"(first), "v"(e1v), "s"(hi), "s"(lo), "s"(gt), "s"(gtn));
        bool bad = false;
        uint32_t words = 0, cls = 0, param = 0, aux = 0;
        if (lane <= gblk && k0 + lane < nb) {
            const uint32_t e1 = e1v;
            if (lane < gblk) {
                cls = e1 & 0xFFu;
                param = (e1 >> 8) & 0xFFu;
                aux = e1 >> 16;
                const uint32_t nk = min(kBlock, n - (k0 + lane) * kBlock), m = nk - 1;
                if (cls == kClsBitmap) {
                    bad = param != 0 || aux > kBitmapMaxSpan;
                } else if (cls <= 33) {
                    bad = param != cls - 1 || aux != 0;
                } else if (cls == kClsPfor) {
                    const uint32_t E = aux & 0xFFu, hh = aux >> 8;
                    bad = param > 32 || param + hh > 32 || 10 * E > m;
                } else {
                    bad = true;
                }
                words = bad ? 0u : block_words(cls, param, aux, m);
                bad |= words > kBlock;
                bad |= (uint64_t)lo + first >= (uint64_t)hi;
            }
        }
        const uint32_t incl = wave_incl_scan(lane < gblk ? words : 0u);
        const uint32_t A = readlane(incl, 63);
        const uint32_t off = gt + incl - words;
        const uint64_t endw = (uint64_t)gt + A;
        // the group's checks combined without short-circuit branches and
        // taken as a scalar: a 64-bit comparison is a vector instruction,
        // and a branch on its lane mask would make the rest of the loop
        // divergent in the compiler's eyes (the cursor and the bounds copied
        // to vector registers, the block loop exec-masked)
        const bool ok = (ballot(bad) == 0ull) & (endw <= availw) & (last_g ? endw == availw : gtn == gt + A);
        if (!readfirst(ok ? 1u : 0u)) {
            raise_err(a.err, kErrCorrupt);
            continue;
        }
        const uint32_t *pay = seg + metaw;
        uint32_t full_nb = 0;  // a whole group decoded in one go
        if constexpr (by_group) {
            const uint64_t og = oo + (uint64_t)k0 * kBlock;
            if ((gblk == kGroup) & ((uint64_t)(k0 + kGroup) * kBlock <= n) & (og + kGroup * kBlock <= a.out_cap) &
                (A > 0) & (A + 3 <= kWin)) {
                full_nb = kGroup;
            }
        }
        for (uint32_t h = h0; h < h1; ++h) {
            const uint32_t hb = h * kHalf;
            if (hb >= gblk) break;
            const uint32_t nblk = min(kHalf, gblk - hb);
            const uint32_t ub = readlane(off, hb);
            if constexpr (!STAGE) {
                const uint32_t fb = full_nb ? full_nb : kHalf;
                const uint64_t ou = oo + (uint64_t)(k0 + hb) * kBlock;
                const uint32_t ue = full_nb ? gt + A : hb + kHalf < gblk ? readlane(off, hb + kHalf) : gt + A;
                if (full_nb || ((nblk == kHalf) & ((uint64_t)(k0 + hb + kHalf) * kBlock <= n) &
                                (ou + kHalf * kBlock <= a.out_cap) & (ue > ub) & (ue - ub + 3 <= kWin))) {
                    dec_full_unit(fb, pay + ub, ue - ub, win, val, e1v, first, off - ub, hb, lo, hi,
                                  k0 + hb + fb < nb, a.out + ou, a.err, lane);
                    if (full_nb) break;
                    continue;
                }
            }
            uint32_t pa = 0, pb = 0;
            if constexpr (STAGE) {
                const uint32_t ue = hb + nblk < gblk ? readlane(off, hb + nblk) : gt + A;
                const uint32_t Au = ue - ub;
                uint32_t v[kPerLane];
#pragma unroll
                for (uint32_t i = 0; i < kPerLane; ++i) v[i] = lane + 64 * i < Au ? pay[ub + lane + 64 * i] : 0u;
#pragma unroll
                for (uint32_t i = 0; i < kPerLane; ++i) win[lane + 64 * i] = v[i];
                if (lane < 4) win[kWin + lane] = 0u;
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
            } else {
                load_payload(pay, ub, readlane(words, hb), lane, pa, pb);
            }
            for (uint32_t kk = 0; kk < nblk; ++kk) {
                const uint32_t j = hb + kk, k = k0 + j;
                const bool has_next = k + 1 < nb;
                const uint32_t nxt = has_next ? lo + readlane(first, j + 1) : 0u;
                const uint32_t nk = min(kBlock, n - k * kBlock);
                const uint32_t cj = readlane(cls, j);
                const uint32_t *buf = win;
                if constexpr (STAGE) {
                    buf = win + (readlane(off, j) - ub);
                } else {
                    uint32_t na = 0, nbw = 0;
                    if (kk + 1 < nblk) load_payload(pay, readlane(off, j + 1), readlane(words, j + 1), lane, na, nbw);
                    if ((cj == kClsBitmap) & (nk == kBlock)) {
                        // full bitmap: decoded from the registers
                        if (!dec_bitmap_full(pa, pb, readlane(aux, j), lo + readlane(first, j), hi, has_next, nxt,
                                             val, a.out, oo + (uint64_t)k * kBlock, a.out_cap, lane)) {
                            if (lane == 0) raise_err(a.err, kErrCorrupt);
                        }
                        pa = na;
                        pb = nbw;
                        continue;
                    }
                    win[lane] = pa;
                    win[lane + 64] = pb;
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    pa = na;
                    pb = nbw;
                }
                decode_block(buf, readlane(words, j), val, cj, readlane(param, j), readlane(aux, j),
                             lo + readlane(first, j), nk, hi, has_next, nxt, a.out,
                             oo + (uint64_t)k * kBlock, a.out_cap, a.err, lane);
            }
        }
    }
}

// The directory side of a decode unit, as read and checked by the wave.
struct DecUnit {
    uint32_t kind;  // 0: nothing to decode (empty half, or a damaged group, reported)
                    // 1: full unit (8 blocks of 128 IDs); 2: any other unit;
                    // 3: a raw segment (n IDs at pay)
    uint32_t hb, k0, nb, n, gblk, nblk, lo, hi, ub, ue;
    uint64_t oo, availw;
    const uint32_t *pay;
    // lane j < gblk: block j of the group (lane gblk: first of the next block)
    uint32_t e1, first, off, words;
};

// Reads and checks unit u's group directory entries (one lane per block)
// and group-table words, as k_decode_u does.
__device__ __forceinline__ DecUnit dec_dir(const DecArgs &a, SegCursor &c, uint32_t u, uint32_t lane) {
    DecUnit U;
    U.kind = 0;
    const uint32_t t = u >> 1, h = u & 1;
    if (c.seek(a.tile_base, a.nseg, t, lane, a.strided)) {
        c.n = readfirst(a.seg_n[c.r]);
        c.form = readfirst(a.seg_form[c.r]);
        c.S = readfirst64(a.seg_byte_off[c.r]);
        c.bytes = readfirst64(a.seg_byte_off[c.r + 1]) - c.S;
        c.base = readfirst64(a.out_off[c.r]);
        if (c.form == 2) {
            const uint32_t *sg = (const uint32_t *)(a.in + c.S);
            c.hi = readfirst(sg[1]);
            c.lo = readfirst(sg[2]);
        }
    }
    if (c.form != 2) {
        // a raw segment's one tile: its first unit copies the IDs
        if (h == 0) {
            U.kind = 3;
            U.n = c.n;
            U.pay = (const uint32_t *)(a.in + c.S);
            U.oo = c.base;
        }
        return U;
    }
    const uint32_t g = t - c.t_first;
    const uint32_t n = c.n;
    const uint32_t nb = cdiv32(n, kBlock), ng = cdiv32(nb, kGroup);
    const uint32_t k0 = g * kGroup;
    const uint32_t gblk = min(kGroup, nb - k0);
    const uint32_t hb = h * kHalf;
    if (hb >= gblk) return U;
    const uint32_t *seg = (const uint32_t *)(a.in + c.S);
    const uint32_t lo = c.lo, hi = c.hi;
    const uint32_t metaw = 4 + 2 * nb + ng;
    const uint64_t availw = c.bytes / 4 - metaw;
    bool bad = false;
    uint32_t words = 0, e1 = 0, first = 0;
    if (lane <= gblk && k0 + lane < nb) {
        first = seg[4 + 2 * (k0 + lane)];
        if (lane < gblk) {
            e1 = seg[4 + 2 * (k0 + lane) + 1];
            const uint32_t cls = e1 & 0xFFu, param = (e1 >> 8) & 0xFFu, aux = e1 >> 16;
            const uint32_t nk = min(kBlock, n - (k0 + lane) * kBlock), m = nk - 1;
            if (cls == kClsBitmap) {
                bad = param != 0 || aux > kBitmapMaxSpan;
            } else if (cls <= 33) {
                bad = param != cls - 1 || aux != 0;
            } else if (cls == kClsPfor) {
                const uint32_t E = aux & 0xFFu, hh = aux >> 8;
                bad = param > 32 || param + hh > 32 || 10 * E > m;
            } else {
                bad = true;
            }
            words = bad ? 0u : block_words(cls, param, aux, m);
            bad |= words > kBlock;
            bad |= (uint64_t)lo + first >= (uint64_t)hi;
        }
    }
    const uint32_t incl = wave_incl_scan(lane < gblk ? words : 0u);
    const uint32_t A = readlane(incl, 63);
    const uint32_t gt = readfirst(seg[4 + 2 * nb + g]);
    bool ok = ballot(bad) == 0ull;
    ok = ok && (uint64_t)gt + A <= availw;
    if (g + 1 < ng) ok = ok && seg[4 + 2 * nb + g + 1] == gt + A;
    else ok = ok && (uint64_t)gt + A == availw;
    if (!ok) {
        if (lane == 0) raise_err(a.err, kErrCorrupt);
        return U;
    }
    const uint32_t nblk = min(kHalf, gblk - hb);
    U.off = gt + incl - words;
    U.hb = hb, U.k0 = k0, U.nb = nb, U.n = n, U.gblk = gblk, U.nblk = nblk, U.lo = lo, U.hi = hi;
    U.ub = readlane(U.off, hb);
    U.ue = hb + nblk < gblk ? readlane(U.off, hb + nblk) : gt + A;
    U.oo = c.base, U.availw = availw, U.pay = seg + metaw;
    U.e1 = e1, U.first = first, U.words = words;
    U.kind = nblk == kHalf && (uint64_t)(k0 + hb + kHalf) * kBlock <= n ? 1u : 2u;
    return U;
}

// Decode with one block per 16-lane row for full units (dec_unit_r),
// software pipelined: while one full unit is decoded from one half of the
// wave's LDS buffer, the payload of the next one is already on its way into
// the other half by direct global-to-LDS loads (two 16-byte loads per lane
// cover 512 words, from the 16-byte boundary at or below its first word, so
// no load crosses a page that the payload does not touch).  Full units whose
// payload does not fit a half are staged and decoded synchronously, the
// others block by block as in k_decode_u.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 6) void k_decode_r(DecArgs a) {
    constexpr uint32_t kHB = 512;  // words per buffer half
    constexpr uint32_t kWin = kHalf * kBlock;
    constexpr uint32_t kPerLane = kWin / 64;
    __shared__ __align__(16) uint32_t s_buf[WAVES][2 * kHB + 4];
    __shared__ __align__(16) uint32_t s_val[WAVES][4 * 128];
    const uint32_t lane = threadIdx.x & 63, w = readfirst(threadIdx.x >> 6);
    const uint32_t units = 2 * readfirst(a.tile_base[a.nseg]);
    uint32_t *const buf = s_buf[w];
    uint32_t *const val = s_val[w];
    UnitRange ur = unit_range(units, WAVES, w, a.strided);
    SegCursor c;
    bool pv = false;  // a full unit is pending: its payload requested into half ps
    uint32_t ps = 0, pdelta = 0;
    DecUnit P;
    P.kind = 0;
    for (uint32_t u = ur.begin;; u += ur.step) {
        const bool more = u < ur.end;
        DecUnit U;
        U.kind = 0;
        if (more) U = dec_dir(a, c, u, lane);
        bool upipe = false;
        uint32_t us = 0, udelta = 0;
        if (U.kind == 1) {
            const uint32_t *src = U.pay + U.ub;
            udelta = (uint32_t)(((uintptr_t)src & 15) >> 2);
            const uint32_t need = udelta + (U.ue - U.ub);
            // (a damaged directory can describe a unit with no payload words:
            // then nothing is loaded ahead, so no load starts past the data)
            if (U.ue > U.ub && need <= kHB) {
                upipe = true;
                us = pv ? ps ^ 1u : 0u;
                const uint32_t *base = src - udelta;
                const uint32_t last = need ? (need - 1) >> 2 : 0u;  // last 16-byte chunk holding payload
                uint32_t *dst = buf + us * kHB;
                asm volatile("" ::: "memory");
#pragma unroll
                for (uint32_t i = 0; i < 2; ++i)
                    __builtin_amdgcn_global_load_lds((const void *)(base + 4 * (min(lane, last - 64 * i) + 64 * i)),
                                                     (__attribute__((address_space(3))) void *)(dst + 256 * i),
                                                     16, 0, 0);
            }
        }
        if (pv) {
            // the pending unit's two loads were issued before this unit's two
            if (upipe) asm volatile("s_waitcnt vmcnt(2)" ::: "memory");
            else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            dec_unit_r(buf + ps * kHB + pdelta, val, P.ub, P.hb, P.k0, P.nb, P.e1, P.first, P.off, P.lo, P.hi,
                       a.out, P.oo, a.out_cap, a.err, lane);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            pv = false;
        }
        if (U.kind == 1 && !upipe) {
            const uint32_t Au = U.ue - U.ub;
            uint32_t v[kPerLane];
#pragma unroll
            for (uint32_t i = 0; i < kPerLane; ++i) v[i] = lane + 64 * i < Au ? U.pay[U.ub + lane + 64 * i] : 0u;
#pragma unroll
            for (uint32_t i = 0; i < kPerLane; ++i) buf[lane + 64 * i] = v[i];
            if (lane < 4) buf[kWin + lane] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            dec_unit_r(buf, val, U.ub, U.hb, U.k0, U.nb, U.e1, U.first, U.off, U.lo, U.hi, a.out, U.oo,
                       a.out_cap, a.err, lane);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else if (U.kind == 3) {
            dec_raw(U.pay, U.n, a.out, U.oo, a.out_cap, a.err, lane);
        } else if (U.kind == 2) {
            uint32_t pa = 0, pb = 0;
            load_payload(U.pay, U.ub, readlane(U.words, U.hb), lane, pa, pb);
            for (uint32_t kk = 0; kk < U.nblk; ++kk) {
                const uint32_t j = U.hb + kk, k = U.k0 + j;
                const bool has_next = k + 1 < U.nb;
                const uint32_t nxt = has_next ? U.lo + readlane(U.first, j + 1) : 0u;
                uint32_t na = 0, nbw = 0;
                if (kk + 1 < U.nblk)
                    load_payload(U.pay, readlane(U.off, j + 1), readlane(U.words, j + 1), lane, na, nbw);
                buf[lane] = pa;
                buf[lane + 64] = pb;
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                pa = na;
                pb = nbw;
                const uint32_t e1 = readlane(U.e1, j);
                decode_block(buf, readlane(U.words, j), val, e1 & 0xFFu, (e1 >> 8) & 0xFFu, e1 >> 16,
                             U.lo + readlane(U.first, j), min(kBlock, U.n - k * kBlock), U.hi, has_next, nxt,
                             a.out, U.oo + (uint64_t)k * kBlock, a.out_cap, a.err, lane);
            }
        }
        if (upipe) {
            pv = true;
            ps = us;
            pdelta = udelta;
            P = U;
        }
        if (!more) break;
    }
}

// ------------------------------------------------------------------ partition

__global__ void k_partition(const uint32_t *ids, const uint32_t *n_dev, const uint32_t *bounds,
                            uint32_t nseg, uint64_t *seg_off) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > nseg) return;
    const uint32_t n = *n_dev;
    if (r == nseg) {
        seg_off[nseg] = n;
        return;
    }
    const uint32_t key = bounds[r];
    uint32_t lo = 0, hi = n;  // first index with ids[i] >= key
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (ids[mid] < key) lo = mid + 1; else hi = mid;
    }
    seg_off[r] = lo;
}

// ------------------------------------------------------------------ launchers

static inline uint32_t persistent_grid(const bfsc_ctx *ctx, uint32_t per_cu, uint64_t max_tiles) {
    uint64_t g = (uint64_t)ctx->n_cu * per_cu;
    if (g > max_tiles) g = max_tiles;
    return (uint32_t)(g ? g : 1);
}

// Persistent grid for one kernel: never more workgroups per CU than can be
// resident together (a late-starting workgroup would add a whole extra
// round at the end of the pass).
static inline uint32_t resident_grid(const bfsc_ctx *ctx, const void *fn, uint32_t threads,
                                     uint32_t per_cu, uint64_t units) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, (int)threads, 0) == hipSuccess && occ > 0 &&
        (uint32_t)occ < per_cu)
        per_cu = (uint32_t)occ;
    return persistent_grid(ctx, per_cu, units);
}

int launch_plan_prep(const bfsc_batch *b, const Plan &p, uint32_t *err, bool zero_status,
                     hipStream_t s) {
    (void)zero_status;
    PlanArgs a;
    a.seg_off = b->seg_off;
    a.seg_lo = b->seg_lo;
    a.seg_hi = b->seg_hi;
    a.nseg = b->nseg;
    a.max_ids = b->max_ids;
    a.p = p;
    a.err = err;
    const uint32_t chunks = prep_chunks(b->nseg);
    hipLaunchKernelGGL(k_plan_local, dim3(chunks), dim3(kPrepChunk), 0, s, a);
    if (chunks > 1) hipLaunchKernelGGL(k_plan_fix, dim3(chunks), dim3(kPrepChunk), 0, s, a);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_encode(bfsc_ctx *ctx, const bfsc_batch *b, const uint8_t *classes, int mode,
                  uint8_t *out, size_t out_cap, uint64_t *seg_byte_off, const Plan &p,
                  hipStream_t s) {
    EncArgs a;
    a.ids = b->ids;
    a.seg_off = b->seg_off;
    a.seg_lo = b->seg_lo;
    a.seg_hi = b->seg_hi;
    a.classes = classes;
    a.mode = mode;
    a.nseg = b->nseg;
    a.out = (uint32_t *)out;
    a.out_cap = out_cap;
    a.seg_byte_off = seg_byte_off;
    a.p = p;
    a.err = ctx->err;
    a.strided = (ctx->tune.enc_pack >> 2) & 1u;
    a.seg_level = b->seg_level;
    a.w = (const MlpMfma *)ctx->mlp_mfma;
    const uint32_t waves = ctx->tune.enc_waves;
    const uint64_t units = 2ull * p.max_tiles;
    const uint32_t per_cu = ctx->tune.enc_wg_per_cu;
    const int slot = timing_begin(ctx, BFSC_OP_ENCODE, s);
    const bool fused_learned = !classes && mode == BFSC_SEL_LEARNED;
    if (fused_learned) {
        // staged units; at most 8 waves per workgroup (the network is staged
        // once per workgroup)
#define BFSC_PACK_L(W)                                                                          \
    hipLaunchKernelGGL((k_enc_pack_l<W>),                                                          \
                       dim3(resident_grid(ctx, (const void *)k_enc_pack_l<W>, W * 64, per_cu, units)), \
                       dim3(W * 64), 0, s, a)
        switch (waves) {
            case 1: BFSC_PACK_L(1); break;
            case 2: BFSC_PACK_L(2); break;
            case 8: case 16: BFSC_PACK_L(8); break;
            default: BFSC_PACK_L(4); break;
        }
#undef BFSC_PACK_L
    } else
    switch (waves) {
#define BFSC_PACK_LAUNCH(K, W)                                                               \
    hipLaunchKernelGGL(K, dim3(resident_grid(ctx, (const void *)K, W * 64, per_cu, units)), \
                       dim3(W * 64), 0, s, a)
#define BFSC_PACK_CASE(W)                                                                  \
    switch (ctx->tune.enc_pack & 3u) {                                                     \
        case 1: BFSC_PACK_LAUNCH((k_enc_pack_u<W, true, true>), W); break;                 \
        case 2: BFSC_PACK_LAUNCH((k_enc_pack_u<W, false, false>), W); break;               \
        case 3: BFSC_PACK_LAUNCH((k_enc_pack_u<W, true, false>), W); break;                \
        default: BFSC_PACK_LAUNCH((k_enc_pack_u<W, false, true>), W); break;               \
    }
        case 1: BFSC_PACK_CASE(1) break;
        case 2: BFSC_PACK_CASE(2) break;
        case 8: BFSC_PACK_CASE(8) break;
        case 16: BFSC_PACK_CASE(16) break;
        default: BFSC_PACK_CASE(4) break;
#undef BFSC_PACK_LAUNCH
#undef BFSC_PACK_CASE
    }
    timing_end(ctx, slot, s);
    hipLaunchKernelGGL(k_enc_scan, dim3((uint32_t)((2ull * p.max_tiles + kScanChunk - 1) / kScanChunk)), dim3(1024),
                       0, s, a);
    const int slot2 = timing_begin(ctx, BFSC_OP_ENCODE_PLACE, s);
    hipLaunchKernelGGL(k_enc_place<4>, dim3((uint32_t)((p.max_tiles + 3) / 4)), dim3(256), 0, s, a);
    timing_end(ctx, slot2, s);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_select(bfsc_ctx *ctx, const bfsc_batch *b, int mode, uint8_t *classes,
                  uint64_t *fallbacks, uint16_t *feat, const Plan &p, hipStream_t s) {
    SelArgs a;
    a.ids = b->ids;
    a.seg_off = b->seg_off;
    a.seg_lo = b->seg_lo;
    a.seg_hi = b->seg_hi;
    a.seg_level = b->seg_level;
    a.nseg = b->nseg;
    a.mode = mode;
    a.classes = classes;
    a.feat = feat;
    a.fallbacks = fallbacks;
    a.w = (const MlpMfma *)ctx->mlp_mfma;
    a.p = p;
    a.err = ctx->err;
    a.literal = ctx->cfg.resolve_literal;
    const uint32_t grid = persistent_grid(ctx, 4, p.max_tiles);
    const int slot = timing_begin(ctx, feat ? BFSC_OP_FEATURES : BFSC_OP_SELECT, s);
    hipLaunchKernelGGL(k_select<4>, dim3(grid), dim3(256), 0, s, a);
    timing_end(ctx, slot, s);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

// The decoding pass for the tuned unit shape: k_decode_r, or k_decode_u
// with whole groups per unit when the batch can give every wave at least
// eight of them (as the pack passes do with tiles), else half groups.
template <int W, bool MAP>
static void launch_dec_units(const bfsc_ctx *ctx, const DecArgs &a, uint32_t per_cu, uint64_t units,
                             uint64_t max_ids, hipStream_t s) {
    if (ctx->tune.dec_mode & 4u) {
        const uint32_t g = resident_grid(ctx, (const void *)k_decode_r<W>, W * 64, per_cu, units);
        hipLaunchKernelGGL((k_decode_r<W>), dim3(g), dim3(W * 64), 0, s, a);
    } else if (ctx->tune.dec_mode & 1u) {
        const uint32_t g = resident_grid(ctx, (const void *)k_decode_u<W, false, true, MAP>, W * 64, per_cu, units);
        if (max_ids / (kBlock * kGroup) >= 8ull * g * W) {
            hipLaunchKernelGGL((k_decode_u<W, false, true, MAP>), dim3(g), dim3(W * 64), 0, s, a);
        } else {
            const uint32_t gh =
                resident_grid(ctx, (const void *)k_decode_u<W, false, false, MAP>, W * 64, per_cu, units);
            hipLaunchKernelGGL((k_decode_u<W, false, false, MAP>), dim3(gh), dim3(W * 64), 0, s, a);
        }
    } else {
        const uint32_t g = resident_grid(ctx, (const void *)k_decode_u<W, true, false, MAP>, W * 64, per_cu, units);
        hipLaunchKernelGGL((k_decode_u<W, true, false, MAP>), dim3(g), dim3(W * 64), 0, s, a);
    }
}

// The per-segment plan, then the segment of every tile (u32 per tile).
size_t decode_ws_bytes(uint64_t max_ids, uint32_t nseg) {
    return dec_ws_bytes(nseg) + align256(plan_max_tiles(max_ids, nseg) * 4);
}

int launch_decode(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                  uint64_t max_ids, uint32_t *out_ids, uint64_t out_cap, uint64_t *out_off,
                  void *ws, hipStream_t s, bool timed, bool tile_map) {
    char *wb = (char *)ws;
    const size_t arr = align256(((size_t)nseg + 1) * 4);
    uint32_t *seg_n = (uint32_t *)wb;
    uint32_t *tile_base = (uint32_t *)(wb + arr);
    uint32_t *seg_form = (uint32_t *)(wb + 2 * arr);
    const uint32_t chunks = prep_chunks(nseg);
    uint64_t *chunk_n = (uint64_t *)(wb + 3 * arr);
    uint32_t *chunk_t = (uint32_t *)(wb + 3 * arr + align256((size_t)chunks * 8));
    DecPlanArgs pa;
    pa.in = in;
    pa.seg_byte_off = seg_byte_off;
    pa.nseg = nseg;
    pa.out_cap = out_cap;
    pa.out_off = out_off;
    pa.seg_n = seg_n;
    pa.seg_form = seg_form;
    pa.tile_base = tile_base;
    pa.chunk_n = chunk_n;
    pa.chunk_t = chunk_t;
    const uint64_t mt = plan_max_tiles(max_ids, nseg);
    pa.tile_seg = tile_map ? (uint32_t *)(wb + dec_ws_bytes(nseg)) : nullptr;
    pa.map_cap = tile_map ? mt : 0;
    pa.max_ids = max_ids;
    pa.err = ctx->err;
    hipLaunchKernelGGL(k_dec_local, dim3(chunks), dim3(kPrepChunk), 0, s, pa);
    if (chunks > 1) hipLaunchKernelGGL(k_dec_fix, dim3(chunks), dim3(kPrepChunk), 0, s, pa);
    DecArgs a;
    a.in = in;
    a.seg_byte_off = seg_byte_off;
    a.nseg = nseg;
    a.seg_n = seg_n;
    a.seg_form = seg_form;
    a.tile_base = tile_base;
    a.out_off = out_off;
    a.out = out_ids;
    a.out_cap = out_cap;
    a.err = ctx->err;
    a.strided = (ctx->tune.dec_mode >> 1) & 1u;
    a.tile_seg = pa.tile_seg;
    a.map_cap = pa.map_cap;
    const uint64_t units = 2 * mt;  // at most (half groups)
    const uint32_t per_cu = ctx->tune.dec_wg_per_cu;
    const int slot = timed ? timing_begin(ctx, BFSC_OP_DECODE, s) : -1;
    if (tile_map) {
        switch (ctx->tune.dec_waves) {
            case 1: launch_dec_units<1, true>(ctx, a, per_cu, units, max_ids, s); break;
            case 2: launch_dec_units<2, true>(ctx, a, per_cu, units, max_ids, s); break;
            case 8: launch_dec_units<8, true>(ctx, a, per_cu, units, max_ids, s); break;
            case 16: launch_dec_units<16, true>(ctx, a, per_cu, units, max_ids, s); break;
            default: launch_dec_units<4, true>(ctx, a, per_cu, units, max_ids, s); break;
        }
    } else {
        launch_dec_units<4, false>(ctx, a, per_cu, units, max_ids, s);
    }
    timing_end(ctx, slot, s);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_partition(const uint32_t *ids, const uint32_t *n_dev, const uint32_t *bounds,
                     uint32_t nseg, uint64_t *seg_off, hipStream_t s) {
    const uint32_t threads = 256, grid = (nseg + 1 + threads - 1) / threads;
    hipLaunchKernelGGL(k_partition, dim3(grid), dim3(threads), 0, s, ids, n_dev, bounds, nseg,
                       seg_off);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

}  // namespace bfsc
