// Internal definitions shared by the bfsc HIP kernels and the C-ABI layer.
// gfx950 (CDNA4) only: wave64, 160 KiB LDS per CU, 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bfsc.h"

namespace bfsc {

constexpr uint32_t kBlock = 128;        // IDs per codec block (format constant)
constexpr uint32_t kGroup = 16;         // blocks per group-table entry (format constant)
constexpr uint32_t kMagic = 0x31434642u;
constexpr uint32_t kClsBitmap = 0;
constexpr uint32_t kClsPfor = 34;
constexpr uint32_t kBitmapMaxSpan = 4096;
constexpr int kWave = 64;

// Latched error bits (device word in the context).
constexpr uint32_t kErrInval = 1u;
constexpr uint32_t kErrCapacity = 2u;
constexpr uint32_t kErrCorrupt = 4u;

// MLP shape 8 -> 64 -> 64 -> 35.
constexpr int kIn = 8, kH = 64, kOut = 35;
constexpr int kW1 = 0, kB1 = kW1 + kH * kIn, kW2 = kB1 + kH, kB2 = kW2 + kH * kH;
constexpr int kW3 = kB2 + kH, kB3 = kW3 + kOut * kH, kNParams = kB3 + kOut;
static_assert(kNParams == 7011, "parameter count");

// ------------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t popc64(uint64_t x) { return (uint32_t)__popcll(x); }

// Lanes strictly below this one.
__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}
// Number of set bits of mk below this lane (v_mbcnt_lo / v_mbcnt_hi).
__device__ __forceinline__ uint32_t mbcnt64(uint64_t mk) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}

__device__ __forceinline__ uint32_t readfirst(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
// Wave-uniform 64-bit value moved to scalar registers (the compiler then
// treats everything derived from it as uniform: scalar loops and branches).
__device__ __forceinline__ uint64_t readfirst64(uint64_t v) {
    return ((uint64_t)readfirst((uint32_t)(v >> 32)) << 32) | readfirst((uint32_t)v);
}

// A load from memory that no kernel writes while the calling one runs,
// through the constant address space: with a wave-uniform address the
// compiler issues a scalar load, which the wave waits on with lgkmcnt and so
// never behind its own outstanding vector stores.
template <typename T>
__device__ __forceinline__ T ldc(const T *p) {
    return *(const __attribute__((address_space(4))) T *)(uintptr_t)p;
}

__device__ __forceinline__ uint32_t shfl_up(uint32_t v, int d) { return __shfl_up(v, d, 64); }
__device__ __forceinline__ uint32_t shfl_down(uint32_t v, int d) { return __shfl_down(v, d, 64); }
__device__ __forceinline__ uint32_t shfl_xor(uint32_t v, int d) { return __shfl_xor(v, d, 64); }
__device__ __forceinline__ uint32_t shfl(uint32_t v, int src) { return __shfl(v, src, 64); }

// DPP lane movement (GFX9 controls): row_shr:n = 0x110+n within rows of 16,
// row_bcast:15 = 0x142, row_bcast:31 = 0x143, wave_shl:1 = 0x130,
// wave_shr:1 = 0x138.  Lanes whose source is outside the pattern, or whose
// row is masked off, receive `old`.
template <int CTRL, int ROWMASK = 0xF, int BANKMASK = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWMASK, BANKMASK, false);
}

// Value of lane-1 (lane 0 receives `first`).
__device__ __forceinline__ uint32_t lane_prev(uint32_t v, uint32_t first) { return dpp<0x138>(first, v); }
// Value of lane+1 (lane 63 receives `last`).
__device__ __forceinline__ uint32_t lane_next(uint32_t v, uint32_t last) { return dpp<0x130>(last, v); }

// Inclusive scans over the 64 lanes: Hillis-Steele inside rows of 16, then
// the row totals are carried across rows with the two broadcasts.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += dpp<0x111>(0u, v);
    v += dpp<0x112>(0u, v);
    v += dpp<0x114>(0u, v);
    v += dpp<0x118>(0u, v);
    v += dpp<0x142, 0xA>(0u, v);
    v += dpp<0x143, 0xC>(0u, v);
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
    v = max(v, dpp<0x111>(0u, v));
    v = max(v, dpp<0x112>(0u, v));
    v = max(v, dpp<0x114>(0u, v));
    v = max(v, dpp<0x118>(0u, v));
    v = max(v, dpp<0x142, 0xA>(0u, v));
    v = max(v, dpp<0x143, 0xC>(0u, v));
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_min(uint32_t v) {
    v = min(v, dpp<0x111>(0xFFFFFFFFu, v));
    v = min(v, dpp<0x112>(0xFFFFFFFFu, v));
    v = min(v, dpp<0x114>(0xFFFFFFFFu, v));
    v = min(v, dpp<0x118>(0xFFFFFFFFu, v));
    v = min(v, dpp<0x142, 0xA>(0xFFFFFFFFu, v));
    v = min(v, dpp<0x143, 0xC>(0xFFFFFFFFu, v));
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) { return readlane(wave_incl_max(v), 63); }
__device__ __forceinline__ uint32_t wave_min(uint32_t v) { return readlane(wave_incl_min(v), 63); }

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t l2 = shfl_xor((uint32_t)v, d), h2 = shfl_xor((uint32_t)(v >> 32), d);
        v += ((uint64_t)h2 << 32) | l2;
    }
    return ((uint64_t)readfirst((uint32_t)(v >> 32)) << 32) | readfirst((uint32_t)v);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return readlane(wave_incl_scan(v), 63); }

__device__ __forceinline__ uint32_t bitlen32(uint32_t x) { return x ? 32u - (uint32_t)__clz(x) : 0u; }

__device__ __forceinline__ uint32_t cdiv32(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ void raise_err(uint32_t *err, uint32_t bit) {
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last r < n with base[r] <= t (base non-decreasing, base[0] <= t), found by
// the whole wave: 64 probes per round, so 2 dependent loads for up to 4096
// entries and 3 for up to 262144.
__device__ __forceinline__ uint32_t wave_find(const uint32_t *base, uint32_t n, uint32_t t,
                                              uint32_t lane) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) >> 6;
        const uint32_t idx = lo + lane * step;
        const bool ok = idx < hi && base[idx] <= t;
        const uint64_t mk = ballot(ok);
        const uint32_t k = 63u - (uint32_t)__builtin_clzll(mk | 1ull);
        lo = lo + k * step;
        hi = min(hi, lo + step);
    }
    return readfirst(lo);
}

// Exclusive prefix sum over a workgroup of up to 1024 threads.
__device__ inline uint32_t wg_excl_scan(uint32_t v, uint32_t *s_tmp /*[17]*/, uint32_t *total) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) s_tmp[w] = incl;
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (uint32_t i = 0; i < nw; ++i) {
            const uint32_t x = s_tmp[i];
            s_tmp[i] = acc;
            acc += x;
        }
        s_tmp[16] = acc;
    }
    __syncthreads();
    const uint32_t r = s_tmp[w] + incl - v;
    *total = s_tmp[16];
    __syncthreads();
    return r;
}

// Index of the last entry of base[0..n] (non-decreasing) that is <= t.
__device__ __forceinline__ uint32_t upper_bound_m1(const uint32_t *base, uint32_t n, uint32_t t) {
    uint32_t lo = 0, hi = n;  // answer in [0, n-1]
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ batch plan

// Per-batch tiling computed by the prep kernel into the workspace.  A tile is
// one group of up to 16 blocks of one compressed segment; an empty or a raw
// segment (fewer IDs than the compression threshold) gets one tile without
// blocks, whose place wave writes the segment's offset and copies a raw
// segment's IDs.  The pack pass
// works on units, the two halves of a tile (8 blocks each), and puts each
// unit's payload into its own half of the tile's private slot; one
// workgroup then turns the unit sizes into output offsets, and the slots are
// placed: no workgroup ever waits for another.
constexpr uint32_t kHalf = kGroup / 2;                 // blocks per pack unit
constexpr uint32_t kSlotDirWords = 2 * kGroup;
constexpr uint32_t kSlotHalfWords = kHalf * kBlock;    // payload words of a unit, at most
constexpr uint32_t kSlotWords = kSlotDirWords + 2 * kSlotHalfWords;
// Units per chunk of the offset scan (one workgroup of 1024 threads, 4 units
// each); a chunk holds at most 4096 x 1024 payload words, so chunk-local
// offsets and chunk totals fit 32 bits.
constexpr uint32_t kScanChunk = 4096;

struct Plan {
    uint32_t *blk_base;   // [nseg+1] first global block of each segment (raw segments'
                          // blocks included: the index into a class vector)
    uint32_t *grp_base;   // [nseg+1] first global group (compressed segments only)
    uint32_t *fix_base;   // [nseg+1] output words before the segment taken by the headers
                          // and directories of compressed segments and the IDs of raw ones
    uint32_t *tile_base;  // [nseg+1] first tile
    uint32_t *seg_n;      // [nseg]   IDs per segment (0 for a rejected segment)
    uint32_t *counter;    // [4]      [0]: workgroups done with the pack pass
    uint32_t *chunk_sums; // [4 x prep chunks] blocks, groups, tiles and fixed words of
                          // every kPrepChunk segments (the plan passes' carries)
    uint32_t *unit_words; // [2 max_tiles] payload words per unit (unit 2t + h: half h of tile t)
    uint32_t *unit_off;   // [2 max_tiles] exclusive prefix of unit_words within the unit's chunk
    uint32_t *chunk_words;  // [chunks] payload words of every chunk of kScanChunk units
    uint2 *tile_seg;      // [max_tiles] segment of each tile and the segment's first tile,
                          // written by the plan passes (encode only)
    uint32_t *slots;      // [max_tiles][kSlotWords] (encode only)
    uint8_t *cls_buf;     // [max blocks] a class vector (encode only: the learned choice
                          // with literal widths runs as a separate pass into it)
    uint32_t max_tiles;
    uint32_t raw_below;   // compression threshold: segments of 1 .. raw_below-1 IDs are raw
};

// Largest compression threshold: a raw segment's blocks then fit the one
// tile it gets (the selection pass covers them tile by tile).
constexpr uint32_t kMaxRawBelow = kBlock * kGroup;

// The most tiles a batch of max_ids IDs in nseg segments can have: a
// segment of n IDs has at most floor(n / 2048) + 1 (a raw or an empty one
// has one), and the floors sum to at most floor(max_ids / 2048).
__host__ __device__ inline uint64_t plan_max_tiles(uint64_t max_ids, uint32_t nseg) {
    return max_ids / (kBlock * kGroup) + nseg + 1;
}

__host__ __device__ constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Segments per workgroup of the plan passes (encode and decode): one
// workgroup scans its chunk, a second pass adds the totals of the chunks
// before it.
constexpr uint32_t kPrepChunk = 1024;
__host__ __device__ constexpr uint32_t prep_chunks(uint32_t nseg) { return (nseg + kPrepChunk - 1) / kPrepChunk; }

// Decoder workspace: seg_n, tile_base, seg_form (u32[nseg+1] each), the
// chunk carries (u64 IDs, u32 tiles per chunk of segments), 256 spare bytes.
__host__ __device__ constexpr size_t dec_ws_bytes(uint32_t nseg) {
    return align256(((size_t)nseg + 1) * 4) * 3 + align256((size_t)prep_chunks(nseg) * 8) +
           align256((size_t)prep_chunks(nseg) * 4) + 256;
}

// Carves a Plan out of a workspace; returns the bytes used.  Slots are only
// laid out (and only counted) for the encoder.
__host__ __device__ inline size_t plan_layout(void *ws, uint64_t max_ids, uint32_t nseg, bool slots,
                                              Plan *p) {
    char *b = (char *)ws;
    size_t off = 0;
    size_t n1 = (size_t)nseg + 1;
    uint64_t mt = plan_max_tiles(max_ids, nseg);
    if (p) p->blk_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->grp_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->fix_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->tile_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->seg_n = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->counter = (uint32_t *)(b + off);
    off = align256(off + 16);
    if (p) p->chunk_sums = (uint32_t *)(b + off);
    off = align256(off + (size_t)prep_chunks(nseg) * 16);
    if (p) p->unit_words = (uint32_t *)(b + off);
    off = align256(off + 2 * mt * 4);
    if (p) p->unit_off = (uint32_t *)(b + off);
    off = align256(off + 2 * mt * 4);
    if (p) p->chunk_words = (uint32_t *)(b + off);
    off = align256(off + ((2 * mt + kScanChunk - 1) / kScanChunk) * 4);
    if (p) p->tile_seg = slots ? (uint2 *)(b + off) : nullptr;
    if (slots) off = align256(off + mt * 8);
    if (p) p->slots = slots ? (uint32_t *)(b + off) : nullptr;
    if (slots) off = align256(off + mt * (size_t)kSlotWords * 4);
    if (p) p->cls_buf = slots ? (uint8_t *)(b + off) : nullptr;
    if (slots) off = align256(off + (max_ids + kBlock - 1) / kBlock + nseg);
    if (p) p->max_tiles = (uint32_t)mt;
    if (p) p->raw_below = 0;
    return off;
}

}  // namespace bfsc

// ------------------------------------------------------------------ context

struct bfsc_ctx {
    int device;
    int n_cu;
    uint32_t *err;          // device error word
    float *mlp_params;      // device fp32 master [7011]
    float *adam_m, *adam_v; // device [7011]
    float *mlp_grad;        // device [7011]
    _Float16 *mlp_w16;      // device fp16 copy of the parameters [7011]
    void *mlp_mfma;         // device: the fp16 weights in MFMA operand order + biases
    uint32_t adam_t;
    bfsc_tune tune;
    bfsc_config cfg;          // settings from bfsc_create (cfg.tune_cache -> tune_cache)
    char tune_cache[1024];
    // per-kernel event timing (bfsc_timing_enable / bfsc_timing_read)
    int timing;
    uint32_t n_timed;
    int timed_op[4096];
    hipEvent_t ev_a[4096], ev_b[4096];
    uint32_t ev_created;
    // direction-optimizing BFS (bfsc_bfs_set_direction); alpha 0: top-down only
    float bfs_alpha, bfs_beta;
    // this device's copy of the decoder scratch array of bfsc_decode_noalloc
    // (its device address, from hipGetSymbolAddress at create)
    void *noalloc_scratch;
};

namespace bfsc {
// Stores the context's launch shapes in its tune cache file (if configured).
void tune_cache_store(const bfsc_ctx *c);
// Brackets one kernel launch with an event pair on stream s when timing is
// on; returns the slot (or -1).
int timing_begin(bfsc_ctx *ctx, int op, hipStream_t s);
void timing_end(bfsc_ctx *ctx, int slot, hipStream_t s);
}  // namespace bfsc

// Launch helpers defined in the kernel files.
namespace bfsc {
int launch_plan_prep(const bfsc_batch *b, const Plan &p, uint32_t *err, bool zero_status,
                     hipStream_t s);
int launch_encode(bfsc_ctx *ctx, const bfsc_batch *b, const uint8_t *classes, int mode,
                  uint8_t *out, size_t out_cap, uint64_t *seg_byte_off, const Plan &p,
                  hipStream_t s);
int launch_select(bfsc_ctx *ctx, const bfsc_batch *b, int mode, uint8_t *classes,
                  uint64_t *fallbacks, uint16_t *feat, const Plan &p, hipStream_t s);
int launch_decode(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                  uint64_t max_ids, uint32_t *out_ids, uint64_t out_cap, uint64_t *out_off,
                  void *ws, hipStream_t s, bool timed = true, bool tile_map = true);
size_t decode_ws_bytes(uint64_t max_ids, uint32_t nseg);
int launch_partition(const uint32_t *ids, const uint32_t *n_dev, const uint32_t *bounds,
                     uint32_t nseg, uint64_t *seg_off, hipStream_t s);
int launch_bfs_init(bfsc_ctx *ctx, const bfsc_csr *g, uint32_t root, int32_t *level,
                    int32_t *parent, uint32_t *frontier, uint32_t *frontier_len, void *ws,
                    hipStream_t s);
int launch_bfs_level(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *frontier,
                     const uint32_t *frontier_len, int32_t *level, int32_t *parent, uint32_t *next,
                     uint32_t *next_len, void *ws, hipStream_t s,
                     const int32_t *cur_level_dev = nullptr);
int launch_level_inc(int32_t *level_dev, hipStream_t s);
size_t mlp_ws_bytes(uint32_t n);
size_t bitmap_ws_bytes(uint64_t max_words, uint32_t nseg);
uint64_t bitmap_encode_bound(uint64_t n_words, uint32_t nseg);
int launch_bitmap_encode(bfsc_ctx *ctx, const uint32_t *bits, const uint64_t *seg_w, uint32_t nseg, uint64_t max_words,
                         uint8_t *out, uint64_t out_cap, uint64_t *seg_byte_off, void *ws, hipStream_t s);
int launch_bitmap_decode(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                         uint64_t max_words, uint32_t *out, uint64_t out_cap, uint64_t *out_off, void *ws,
                         hipStream_t s);
int launch_mlp_forward(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, hipStream_t s);
int launch_mlp_infer(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, uint8_t *cls,
                     hipStream_t s);
int launch_mlp_grad(bfsc_ctx *ctx, const uint16_t *X, const uint8_t *y, uint32_t n, float *grads,
                    float *loss, void *ws, hipStream_t s);
int launch_adam(bfsc_ctx *ctx, const float *grads, const bfsc_adam *opt, hipStream_t s);
}  // namespace bfsc
