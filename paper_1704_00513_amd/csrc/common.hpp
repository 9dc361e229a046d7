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

// Look-back status word: flag in the top two bits, value in the low 62.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagIncl = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr uint64_t kReady = 1ull << 63;

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

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}

__device__ __forceinline__ uint32_t readfirst(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint32_t shfl_up(uint32_t v, int d) { return __shfl_up(v, d, 64); }
__device__ __forceinline__ uint32_t shfl_down(uint32_t v, int d) { return __shfl_down(v, d, 64); }
__device__ __forceinline__ uint32_t shfl_xor(uint32_t v, int d) { return __shfl_xor(v, d, 64); }
__device__ __forceinline__ uint32_t shfl(uint32_t v, int src) { return __shfl(v, src, 64); }

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, shfl_xor(v, d));
    return readfirst(v);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = min(v, shfl_xor(v, d));
    return readfirst(v);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t l2 = shfl_xor((uint32_t)v, d), h2 = shfl_xor((uint32_t)(v >> 32), d);
        v += ((uint64_t)h2 << 32) | l2;
    }
    return ((uint64_t)readfirst((uint32_t)(v >> 32)) << 32) | readfirst((uint32_t)v);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += shfl_xor(v, d);
    return readfirst(v);
}

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = shfl_up(v, d);
        if (l >= (uint32_t)d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t bitlen32(uint32_t x) { return x ? 32u - (uint32_t)__clz(x) : 0u; }

__device__ __forceinline__ uint32_t cdiv32(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ void raise_err(uint32_t *err, uint32_t bit) {
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ld_acq64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_rel64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// one group of up to 16 blocks of one segment; an empty segment gets one
// tile without blocks (so that someone writes its header).
struct Plan {
    uint32_t *blk_base;   // [nseg+1] first global block of each segment
    uint32_t *grp_base;   // [nseg+1] first global group
    uint32_t *tile_base;  // [nseg+1] first tile
    uint64_t *seg_pw;     // [nseg]   payload-word base of each segment (kReady when set)
    uint64_t *status;     // [max_tiles] look-back status
    uint32_t *counter;    // [4]      tile ticket, spare
    uint32_t *seg_n;      // [nseg]   IDs per segment (0 for a rejected segment)
    uint32_t max_tiles;
};

__host__ __device__ inline uint64_t plan_max_tiles(uint64_t max_ids, uint32_t nseg) {
    return max_ids / (kBlock * kGroup) + 2ull * nseg + 2;
}

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves a Plan out of a workspace; returns the bytes used.
__host__ __device__ inline size_t plan_layout(void *ws, uint64_t max_ids, uint32_t nseg, Plan *p) {
    char *b = (char *)ws;
    size_t off = 0;
    size_t n1 = (size_t)nseg + 1;
    uint64_t mt = plan_max_tiles(max_ids, nseg);
    if (p) p->blk_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->grp_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->tile_base = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->seg_pw = (uint64_t *)(b + off);
    off = align256(off + n1 * 8);
    if (p) p->status = (uint64_t *)(b + off);
    off = align256(off + mt * 8);
    if (p) p->counter = (uint32_t *)(b + off);
    off = align256(off + 16);
    if (p) p->seg_n = (uint32_t *)(b + off);
    off = align256(off + n1 * 4);
    if (p) p->max_tiles = (uint32_t)mt;
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
    uint32_t adam_t;
    bfsc_tune tune;
    // per-kernel event timing (bfsc_timing_enable / bfsc_timing_read)
    int timing;
    uint32_t n_timed;
    int timed_op[4096];
    hipEvent_t ev_a[4096], ev_b[4096];
    uint32_t ev_created;
};

namespace bfsc {
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
                  void *ws, hipStream_t s);
size_t decode_ws_bytes(uint64_t max_ids, uint32_t nseg);
int launch_partition(const uint32_t *ids, const uint32_t *n_dev, const uint32_t *bounds,
                     uint32_t nseg, uint64_t *seg_off, hipStream_t s);
int launch_bfs_init(bfsc_ctx *ctx, const bfsc_csr *g, uint32_t root, int32_t *level,
                    int32_t *parent, uint32_t *frontier, uint32_t *frontier_len, void *ws,
                    hipStream_t s);
int launch_bfs_level(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *frontier,
                     const uint32_t *frontier_len, int32_t *level, int32_t *parent, uint32_t *next,
                     uint32_t *next_len, void *ws, hipStream_t s);
size_t mlp_ws_bytes(uint32_t n);
int launch_mlp_forward(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, hipStream_t s);
int launch_mlp_grad(bfsc_ctx *ctx, const uint16_t *X, const uint8_t *y, uint32_t n, float *grads,
                    float *loss, void *ws, hipStream_t s);
int launch_adam(bfsc_ctx *ctx, const float *grads, const bfsc_adam *opt, hipStream_t s);
}  // namespace bfsc
