// C-ABI entry points of libbfsc.so: argument checks on the host, workspace
// carving, and kernel launches on the caller's stream (declared in bfsc.h).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "common.hpp"
#include "exchange.hpp"
#include "mlp_mfma.hpp"

using namespace bfsc;

namespace bfsc {
size_t bfs_ws_bytes_arcs(uint32_t V, uint64_t n_arcs);
int launch_round16(bfsc_ctx *ctx, hipStream_t s);
}

#define HIP_OK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return BFSC_E_HIP;   \
    } while (0)

static inline hipStream_t S(void *s) { return (hipStream_t)s; }

namespace bfsc {

int timing_begin(bfsc_ctx *ctx, int op, hipStream_t s) {
    if (!ctx->timing || ctx->n_timed >= 4096) return -1;
    const uint32_t i = ctx->n_timed;
    if (i >= ctx->ev_created) {
        if (hipEventCreate(&ctx->ev_a[i]) != hipSuccess) return -1;
        if (hipEventCreate(&ctx->ev_b[i]) != hipSuccess) {
            hipEventDestroy(ctx->ev_a[i]);
            return -1;
        }
        ctx->ev_created = i + 1;
    }
    if (hipEventRecord(ctx->ev_a[i], s) != hipSuccess) return -1;
    ctx->timed_op[i] = op;
    ctx->n_timed = i + 1;
    return (int)i;
}

void timing_end(bfsc_ctx *ctx, int slot, hipStream_t s) {
    if (slot < 0) return;
    if (hipEventRecord(ctx->ev_b[slot], s) != hipSuccess) ctx->timed_op[slot] = -1;
}

}  // namespace bfsc

// ------------------------------------------------------------------ decode scratch without allocation
// bfsc_decode_noalloc keeps the decoder's per-segment plan (three u32 arrays
// of nseg + 1 entries and the carries of its chunks of segments, each
// 256-byte aligned, plus 256 bytes) in this file-scope array instead of a
// caller workspace.  Every GPU the library
// runs on holds its own copy until the process ends.  In host code `scratch`
// only names the symbol: its device address on the current GPU comes from
// hipGetSymbolAddress, resolved once per device at bfsc_create.
static constexpr size_t kNoAllocScratchBytes = dec_ws_bytes(BFSC_DECODE_NOALLOC_MAX_SEGS);
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];

// The device address of `scratch` on `device`, which must be current.
static int noalloc_scratch_addr(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return BFSC_E_INVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BFSC_E_HIP;
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return BFSC_OK;
}

static int set_device(const bfsc_ctx *ctx) {
    return hipSetDevice(ctx->device) == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

static bool batch_ok(const bfsc_batch *b) {
    return b && b->ids && b->seg_off && b->seg_lo && b->seg_hi && b->nseg > 0 &&
           b->max_ids < (1ull << 40);
}

// ------------------------------------------------------------------ tune cache
// One line per device: "<arch name> <compute units> enc_waves enc_wg_per_cu
// dec_waves dec_wg_per_cu enc_pack dec_mode".

static void device_key(int device, char *arch, size_t cap, int *n_cu) {
    hipDeviceProp_t prop;
    arch[0] = 0;
    *n_cu = 0;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return;
    snprintf(arch, cap, "%s", prop.gcnArchName);
    for (char *q = arch; *q; ++q)
        if (*q == ' ' || *q == '\n') *q = '_';
    *n_cu = prop.multiProcessorCount;
}

static bool tune_valid(const bfsc_tune *t);

static void tune_cache_load(bfsc_ctx *c) {
    if (!c->cfg.autotune || !c->tune_cache[0]) return;
    FILE *f = fopen(c->tune_cache, "r");
    if (!f) return;
    char arch[256], want[256], line[512];
    int n_cu = 0, want_cu = 0;
    device_key(c->device, want, sizeof want, &want_cu);
    while (fgets(line, sizeof line, f)) {
        bfsc_tune t;
        if (sscanf(line, "%255s %d %u %u %u %u %u %u", arch, &n_cu, &t.enc_waves, &t.enc_wg_per_cu,
                   &t.dec_waves, &t.dec_wg_per_cu, &t.enc_pack, &t.dec_mode) == 8 &&
            n_cu == want_cu && strcmp(arch, want) == 0 && tune_valid(&t))
            c->tune = t;
    }
    fclose(f);
}

namespace bfsc {
// Rewrites the cache file with this device's line replaced (other devices'
// lines kept).  Best effort: a file that cannot be written is left alone.
void tune_cache_store(const bfsc_ctx *c) {
    if (!c->cfg.autotune || !c->tune_cache[0]) return;
    char want[256];
    int want_cu = 0;
    device_key(c->device, want, sizeof want, &want_cu);
    char keep[64][512];
    int nk = 0;
    if (FILE *f = fopen(c->tune_cache, "r")) {
        char line[512], arch[256];
        int n_cu = 0;
        while (nk < 64 && fgets(line, sizeof line, f)) {
            if (sscanf(line, "%255s %d", arch, &n_cu) == 2 && !(n_cu == want_cu && strcmp(arch, want) == 0))
                snprintf(keep[nk++], sizeof keep[0], "%s", line);
        }
        fclose(f);
    }
    FILE *f = fopen(c->tune_cache, "w");
    if (!f) return;
    for (int i = 0; i < nk; ++i) fputs(keep[i], f);
    const bfsc_tune &t = c->tune;
    fprintf(f, "%s %d %u %u %u %u %u %u\n", want, want_cu, t.enc_waves, t.enc_wg_per_cu, t.dec_waves,
            t.dec_wg_per_cu, t.enc_pack, t.dec_mode);
    fclose(f);
}
}  // namespace bfsc

static bool waves_ok(uint32_t w) { return w == 1 || w == 2 || w == 4 || w == 8 || w == 16; }

static bool tune_valid(const bfsc_tune *t) {
    return waves_ok(t->enc_waves) && waves_ok(t->dec_waves) && t->enc_wg_per_cu >= 1 && t->enc_wg_per_cu <= 64 &&
           t->dec_wg_per_cu >= 1 && t->dec_wg_per_cu <= 64 && t->enc_pack <= 7 && t->dec_mode <= 7;
}

// The selection mode a call asks for (BFSC_SEL_DEFAULT: the context's).
static int sel_mode(const bfsc_ctx *ctx, int mode) { return mode == BFSC_SEL_DEFAULT ? ctx->cfg.selector : mode; }

extern "C" {

void bfsc_config_default(bfsc_config *cfg) {
    if (!cfg) return;
    cfg->selector = BFSC_SEL_EXHAUSTIVE;
    cfg->raw_below = 32;
    cfg->resolve_literal = 0;
    cfg->autotune = 0;
    cfg->tune_cache = nullptr;
}

int bfsc_get_config(const bfsc_ctx *ctx, bfsc_config *cfg) {
    if (!ctx || !cfg) return BFSC_E_INVAL;
    *cfg = ctx->cfg;
    return BFSC_OK;
}

int bfsc_create(bfsc_ctx **out, int device, const bfsc_config *cfg) {
    if (!out) return BFSC_E_INVAL;
    *out = nullptr;
    bfsc_config conf;
    bfsc_config_default(&conf);
    if (cfg) conf = *cfg;
    if (conf.selector < BFSC_SEL_PLAIN_BP || conf.selector > BFSC_SEL_LEARNED || conf.raw_below > kMaxRawBelow ||
        conf.resolve_literal > 1 || conf.autotune > 1 ||
        (conf.tune_cache && strlen(conf.tune_cache) >= sizeof(((bfsc_ctx *)0)->tune_cache)))
        return BFSC_E_INVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return BFSC_E_INVAL;
    HIP_OK(hipSetDevice(device));
    bfsc_ctx *c = new (std::nothrow) bfsc_ctx();
    if (!c) return BFSC_E_HIP;
    memset(c, 0, sizeof(*c));
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete c; return BFSC_E_HIP; }
    c->n_cu = prop.multiProcessorCount;
    if (noalloc_scratch_addr(device, &c->noalloc_scratch) != BFSC_OK) { delete c; return BFSC_E_HIP; }
    const size_t np = kNParams;
    if (hipMalloc((void **)&c->err, 256) != hipSuccess ||
        hipMalloc((void **)&c->mlp_params, np * 4) != hipSuccess ||
        hipMalloc((void **)&c->adam_m, np * 4) != hipSuccess ||
        hipMalloc((void **)&c->adam_v, np * 4) != hipSuccess ||
        hipMalloc((void **)&c->mlp_grad, np * 4) != hipSuccess ||
        hipMalloc((void **)&c->mlp_w16, np * 2) != hipSuccess ||
        hipMalloc(&c->mlp_mfma, sizeof(MlpMfma)) != hipSuccess) {
        bfsc_destroy(c);
        return BFSC_E_HIP;
    }
    if (hipMemset(c->err, 0, 256) != hipSuccess || hipMemset(c->mlp_params, 0, np * 4) != hipSuccess ||
        hipMemset(c->adam_m, 0, np * 4) != hipSuccess || hipMemset(c->adam_v, 0, np * 4) != hipSuccess ||
        hipMemset(c->mlp_w16, 0, np * 2) != hipSuccess ||
        hipMemset(c->mlp_mfma, 0, sizeof(MlpMfma)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        bfsc_destroy(c);
        return BFSC_E_HIP;
    }
    // one wave per unit of 8 blocks, loaded block by block, units dealt out
    // every NW-th; 4-wave workgroups, as many resident per CU as fit for the
    // pack passes, six per CU for the decoder (its best at scale 26: 0.96 ms
    // against 1.02 with five and 1.07 with seven or eight)
    c->tune.enc_waves = 4;
    c->tune.enc_wg_per_cu = 8;
    c->tune.dec_waves = 4;
    c->tune.dec_wg_per_cu = 6;
    c->tune.enc_pack = 6;
    c->tune.dec_mode = 3;
    c->cfg = conf;
    if (conf.tune_cache) snprintf(c->tune_cache, sizeof c->tune_cache, "%s", conf.tune_cache);
    c->cfg.tune_cache = c->tune_cache[0] ? c->tune_cache : nullptr;
    tune_cache_load(c);
    *out = c;
    return BFSC_OK;
}

int bfsc_destroy(bfsc_ctx *ctx) {
    if (!ctx) return BFSC_E_INVAL;
    hipSetDevice(ctx->device);
    hipFree(ctx->err);
    hipFree(ctx->mlp_params);
    hipFree(ctx->adam_m);
    hipFree(ctx->adam_v);
    hipFree(ctx->mlp_grad);
    hipFree(ctx->mlp_w16);
    hipFree(ctx->mlp_mfma);
    for (uint32_t i = 0; i < ctx->ev_created; ++i) {
        hipEventDestroy(ctx->ev_a[i]);
        hipEventDestroy(ctx->ev_b[i]);
    }
    delete ctx;
    return BFSC_OK;
}

int bfsc_workspace_size(const bfsc_ctx *ctx, int op, uint64_t max_ids, uint32_t nseg, size_t *bytes) {
    if (!ctx || !bytes) return BFSC_E_INVAL;
    switch (op) {
        case BFSC_OP_SELECT:
        case BFSC_OP_ENCODE:
        case BFSC_OP_FEATURES:
            *bytes = plan_layout(nullptr, max_ids, nseg, op == BFSC_OP_ENCODE, nullptr);
            return BFSC_OK;
        case BFSC_OP_DECODE:
            *bytes = decode_ws_bytes(max_ids, nseg);
            return BFSC_OK;
        case BFSC_OP_MLP:
            *bytes = mlp_ws_bytes((uint32_t)(max_ids ? max_ids : 1));
            return BFSC_OK;
        case BFSC_OP_BITMAP_ENCODE:
        case BFSC_OP_BITMAP_DECODE:
            *bytes = bitmap_ws_bytes(max_ids, nseg);
            return BFSC_OK;
        default:
            return BFSC_E_INVAL;
    }
}

int bfsc_bfs_workspace_size(const bfsc_csr *g, size_t *bytes) {
    if (!g || !bytes || g->n_vertices == 0) return BFSC_E_INVAL;
    *bytes = bfs_ws_bytes_arcs(g->n_vertices, g->n_arcs);
    return BFSC_OK;
}

int bfsc_bfs_init(bfsc_ctx *ctx, const bfsc_csr *g, uint32_t root, int32_t *level, int32_t *parent,
                  uint32_t *frontier, uint32_t *frontier_len_dev, void *ws, void *stream) {
    if (!ctx || !g || !level || !parent || !frontier || !frontier_len_dev || !ws) return BFSC_E_INVAL;
    if (g->n_vertices == 0 || root >= g->n_vertices || g->n_vertices > 0x7FFFFFFFu) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_bfs_init(ctx, g, root, level, parent, frontier, frontier_len_dev, ws, S(stream));
}

int bfsc_bfs_level(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *frontier,
                   const uint32_t *frontier_len_dev, int32_t *level, int32_t *parent, uint32_t *next,
                   uint32_t *next_len_dev, void *ws, void *stream) {
    if (!ctx || !g || !g->row_ptr || !g->col_idx || !frontier || !frontier_len_dev || !level ||
        !parent || !next || !next_len_dev || !ws || cur_level < 0)
        return BFSC_E_INVAL;
    if (g->n_vertices == 0 || g->n_vertices > 0x7FFFFFFFu) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_bfs_level(ctx, g, cur_level, frontier, frontier_len_dev, level, parent, next,
                            next_len_dev, ws, S(stream));
}

int bfsc_bfs_set_direction(bfsc_ctx *ctx, float alpha, float beta) {
    if (!ctx || !(alpha >= 0.f) || (alpha > 0.f && !(beta > 0.f))) return BFSC_E_INVAL;
    ctx->bfs_alpha = alpha;
    ctx->bfs_beta = beta;
    return BFSC_OK;
}

// the candidate exchange: the owners' bitmaps together are indexed by 32-bit
// word numbers (nseg * ceil(V/32) words, with room for the last compaction
// chunk), and the nseg * nseg segments form one batch
static bool ex_ok(const bfsc_csr *g, uint32_t nseg) {
    return g && g->n_vertices > 0 && g->n_vertices <= 0x7FFFFFFFu && nseg > 0 && nseg <= 65535u &&
           (uint64_t)nseg * ((g->n_vertices + 31ull) / 32ull) <= 0xFFFFFFFFull - 65536ull;
}

int bfsc_exchange_workspace_size(const bfsc_csr *g, uint32_t nseg, size_t *bytes) {
    if (!bytes || !ex_ok(g, nseg)) return BFSC_E_INVAL;
    *bytes = ex_ws_bytes(g->n_vertices, g->n_arcs, nseg);
    return BFSC_OK;
}

int bfsc_exchange_init(bfsc_ctx *ctx, const bfsc_csr *g, uint32_t nseg, void *ws, void *stream) {
    if (!ctx || !ws || !ex_ok(g, nseg)) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_ex_init(ctx, g->n_vertices, g->n_arcs, nseg, ws, S(stream));
}

int bfsc_candidates(bfsc_ctx *ctx, const bfsc_csr *g, const uint32_t *frontier, const uint32_t *frontier_len_dev,
                    const uint32_t *bounds, uint32_t nseg, uint32_t *ids, uint64_t cap, uint64_t *seg_off,
                    uint32_t *seg_lo, uint32_t *seg_hi, void *ws, void *stream) {
    if (!ctx || !ex_ok(g, nseg) || !g->row_ptr || !g->col_idx || !frontier || !frontier_len_dev || !bounds ||
        !ids || !seg_off || !seg_lo || !seg_hi || !ws)
        return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_candidates(ctx, g, frontier, frontier_len_dev, bounds, nseg, ids, cap, seg_off, seg_lo, seg_hi,
                             ws, S(stream));
}

int bfsc_merge_filter(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *ids,
                      const uint64_t *n_dev, int32_t *level, uint32_t *next, uint32_t *next_len_dev, void *bfs_ws,
                      void *ws, void *stream) {
    if (!ctx || !ex_ok(g, 1) || !ids || !n_dev || !level || !next || !next_len_dev || !bfs_ws || !ws ||
        cur_level < 0)
        return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_merge_filter(ctx, g, cur_level, ids, n_dev, level, next, next_len_dev, bfs_ws, ws, S(stream));
}

int bfsc_partition(const uint32_t *ids, const uint32_t *n_dev, const uint32_t *bounds, uint32_t nseg,
                   uint64_t *seg_off, void *stream) {
    if (!ids || !n_dev || !bounds || !seg_off || nseg == 0) return BFSC_E_INVAL;
    return launch_partition(ids, n_dev, bounds, nseg, seg_off, S(stream));
}

int bfsc_select(bfsc_ctx *ctx, const bfsc_batch *b, int mode, uint8_t *classes,
                uint64_t *fallbacks_dev, void *ws, void *stream) {
    if (!ctx || !batch_ok(b) || !classes || !ws) return BFSC_E_INVAL;
    mode = sel_mode(ctx, mode);
    if (mode < BFSC_SEL_PLAIN_BP || mode > BFSC_SEL_LEARNED) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    Plan p;
    plan_layout(ws, b->max_ids, b->nseg, false, &p);
    int st = launch_plan_prep(b, p, ctx->err, false, S(stream));
    if (st) return st;
    return launch_select(ctx, b, mode, classes, fallbacks_dev, nullptr, p, S(stream));
}

int bfsc_features(bfsc_ctx *ctx, const bfsc_batch *b, uint16_t *feat, void *ws, void *stream) {
    if (!ctx || !batch_ok(b) || !feat || !ws) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    Plan p;
    plan_layout(ws, b->max_ids, b->nseg, false, &p);
    int st = launch_plan_prep(b, p, ctx->err, false, S(stream));
    if (st) return st;
    return launch_select(ctx, b, BFSC_SEL_EXHAUSTIVE, nullptr, nullptr, feat, p, S(stream));
}

int bfsc_encode_bound(uint64_t n_ids, uint32_t nseg, size_t *bytes) {
    if (!bytes) return BFSC_E_INVAL;
    const uint64_t nb = (n_ids + kBlock - 1) / kBlock + nseg;
    const uint64_t ng = (n_ids + kBlock * kGroup - 1) / (kBlock * kGroup) + nseg;
    *bytes = (size_t)(16ull * nseg + nb * (8ull + 4ull * kBlock) + 4ull * ng);
    return BFSC_OK;
}

int bfsc_encode(bfsc_ctx *ctx, const bfsc_batch *b, const uint8_t *classes, int mode, uint8_t *out,
                size_t out_cap, uint64_t *seg_byte_off, void *ws, void *stream) {
    if (!ctx || !batch_ok(b) || !out || !seg_byte_off || !ws) return BFSC_E_INVAL;
    mode = sel_mode(ctx, mode);
    if (((uintptr_t)out & 3) || mode < BFSC_SEL_PLAIN_BP || mode > BFSC_SEL_LEARNED) return BFSC_E_INVAL;
    if (mode == BFSC_SEL_LEARNED && !classes && !b->seg_level) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    Plan p;
    plan_layout(ws, b->max_ids, b->nseg, true, &p);
    p.raw_below = ctx->cfg.raw_below;
    int st = launch_plan_prep(b, p, ctx->err, true, S(stream));
    if (st) return st;
    if (mode == BFSC_SEL_LEARNED && !classes && ctx->cfg.resolve_literal) {
        // literal widths are not a selection kind of the fused pass: select
        // into the workspace first
        st = launch_select(ctx, b, BFSC_SEL_LEARNED, p.cls_buf, nullptr, nullptr, p, S(stream));
        if (st) return st;
        classes = p.cls_buf;
    }
    return launch_encode(ctx, b, classes, mode, out, out_cap, seg_byte_off, p, S(stream));
}

int bfsc_decode(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                uint64_t max_ids, uint32_t *out_ids, uint64_t out_cap, uint64_t *out_off, void *ws,
                void *stream) {
    if (!ctx || !in || !seg_byte_off || !out_ids || !out_off || !ws || nseg == 0) return BFSC_E_INVAL;
    if ((uintptr_t)in & 3) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_decode(ctx, in, seg_byte_off, nseg, max_ids, out_ids, out_cap, out_off, ws, S(stream));
}

int bfsc_decode_noalloc(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                        uint64_t max_ids, uint32_t *out_ids, uint64_t out_cap, uint64_t *out_off,
                        void *stream) {
    if (!ctx || !in || !seg_byte_off || !out_ids || !out_off || nseg == 0) return BFSC_E_INVAL;
    if (nseg > BFSC_DECODE_NOALLOC_MAX_SEGS || (uintptr_t)in & 3) return BFSC_E_INVAL;
    if (dec_ws_bytes(nseg) > kNoAllocScratchBytes || !ctx->noalloc_scratch) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    // every word of the plan that the decoder reads is written by its first
    // kernel, so the array needs no clearing between calls; no timing events
    // either (creating one may allocate); the array holds the per-segment
    // plan only, so the decoder finds each tile's segment by search
    return launch_decode(ctx, in, seg_byte_off, nseg, max_ids, out_ids, out_cap, out_off, ctx->noalloc_scratch,
                         S(stream), false, false);
}

int bfsc_bitmap_encode_bound(uint64_t n_words, uint32_t nseg, size_t *bytes) {
    if (!bytes) return BFSC_E_INVAL;
    *bytes = (size_t)bitmap_encode_bound(n_words, nseg);
    return BFSC_OK;
}

int bfsc_bitmap_encode(bfsc_ctx *ctx, const uint32_t *bits, const uint64_t *seg_w, uint32_t nseg, uint64_t max_words,
                       uint8_t *out, size_t out_cap, uint64_t *seg_byte_off, void *ws, void *stream) {
    if (!ctx || !bits || !seg_w || !out || !seg_byte_off || !ws || nseg == 0 || max_words >= (1ull << 40))
        return BFSC_E_INVAL;
    if ((uintptr_t)out & 3) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_bitmap_encode(ctx, bits, seg_w, nseg, max_words, out, out_cap, seg_byte_off, ws, S(stream));
}

int bfsc_bitmap_decode(bfsc_ctx *ctx, const uint8_t *in, const uint64_t *seg_byte_off, uint32_t nseg,
                       uint64_t max_words, uint32_t *out, uint64_t out_cap, uint64_t *out_off, void *ws,
                       void *stream) {
    if (!ctx || !in || !seg_byte_off || !out || !out_off || !ws || nseg == 0 || max_words >= (1ull << 40))
        return BFSC_E_INVAL;
    if ((uintptr_t)in & 3) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_bitmap_decode(ctx, in, seg_byte_off, nseg, max_words, out, out_cap, out_off, ws, S(stream));
}

int bfsc_mlp_param_count(void) { return kNParams; }

// Counter-based SplitMix64 draw (Steele, Lea & Flood, OOPSLA 2014): the
// finaliser applied to seed + G (stream + 1), then to that key + G (idx + 1).
static uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t ctr64(uint64_t seed, uint64_t stream, uint64_t idx) {
    const uint64_t G = 0x9E3779B97F4A7C15ull;
    return mix64(mix64(seed + G * (stream + 1)) + G * (idx + 1));
}

int bfsc_mlp_init(bfsc_ctx *ctx, uint64_t seed) {
    if (!ctx) return BFSC_E_INVAL;
    static const int dims[4] = {kIn, kH, kH, kOut};
    float *h = (float *)calloc(kNParams, sizeof(float));
    if (!h) return BFSC_E_HIP;
    size_t k = 0;
    for (int l = 0; l < 3; ++l) {
        const uint64_t nw = (uint64_t)dims[l] * dims[l + 1];
        const float lim = (float)sqrt(6.0 / dims[l]);
        for (uint64_t i = 0; i < nw; ++i) {
            const double u = (double)(ctr64(seed, 100 + l, i) >> 40) * 0x1.0p-24;
            h[k++] = (float)((double)lim * (2.0 * u - 1.0));
        }
        k += dims[l + 1];  // biases stay 0
    }
    const int st = bfsc_mlp_set_weights(ctx, h);
    free(h);
    return st;
}

int bfsc_mlp_set_weights(bfsc_ctx *ctx, const float *host_params) {
    if (!ctx || !host_params) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    HIP_OK(hipMemcpy(ctx->mlp_params, host_params, kNParams * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemset(ctx->adam_m, 0, kNParams * 4));
    HIP_OK(hipMemset(ctx->adam_v, 0, kNParams * 4));
    ctx->adam_t = 0;
    if (launch_round16(ctx, nullptr)) return BFSC_E_HIP;
    HIP_OK(hipDeviceSynchronize());
    return BFSC_OK;
}

int bfsc_mlp_get_weights(bfsc_ctx *ctx, float *host_params) {
    if (!ctx || !host_params) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(host_params, ctx->mlp_params, kNParams * 4, hipMemcpyDeviceToHost));
    return BFSC_OK;
}

int bfsc_mlp_forward(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, void *ws,
                     void *stream) {
    (void)ws;
    if (!ctx || (!X && n) || (!logits && n)) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_mlp_forward(ctx, X, n, logits, S(stream));
}

int bfsc_mlp_infer(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, uint8_t *classes,
                   void *stream) {
    if (!ctx || (!X && n)) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_mlp_infer(ctx, X, n, logits, classes, S(stream));
}

int bfsc_mlp_grad(bfsc_ctx *ctx, const uint16_t *X, const uint8_t *y, uint32_t n, float *grads,
                  float *loss_dev, void *ws, void *stream) {
    if (!ctx || !X || !y || !grads || !ws || n == 0) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    return launch_mlp_grad(ctx, X, y, n, grads, loss_dev, ws, S(stream));
}

int bfsc_mlp_train_step(bfsc_ctx *ctx, const uint16_t *X, const uint8_t *y, uint32_t n,
                        const bfsc_adam *opt, float *loss_dev, void *ws, void *stream) {
    if (!ctx || !X || !y || !opt || !ws || n == 0) return BFSC_E_INVAL;
    if (!(opt->lr > 0.0f) || !(opt->beta1 >= 0.0f && opt->beta1 < 1.0f) ||
        !(opt->beta2 >= 0.0f && opt->beta2 < 1.0f) || !(opt->eps > 0.0f))
        return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    int st = launch_mlp_grad(ctx, X, y, n, ctx->mlp_grad, loss_dev, ws, S(stream));
    if (st) return st;
    return launch_adam(ctx, ctx->mlp_grad, opt, S(stream));
}

int bfsc_get_tune(const bfsc_ctx *ctx, bfsc_tune *out) {
    if (!ctx || !out) return BFSC_E_INVAL;
    *out = ctx->tune;
    return BFSC_OK;
}

int bfsc_set_tune(bfsc_ctx *ctx, const bfsc_tune *t) {
    if (!ctx || !t || !tune_valid(t)) return BFSC_E_INVAL;
    ctx->tune = *t;
    return BFSC_OK;
}

int bfsc_timing_enable(bfsc_ctx *ctx, int enable) {
    if (!ctx) return BFSC_E_INVAL;
    ctx->timing = enable ? 1 : 0;
    ctx->n_timed = 0;
    return BFSC_OK;
}

int bfsc_timing_read(bfsc_ctx *ctx, int op, double *total_ms, uint64_t *count) {
    if (!ctx || !total_ms || !count) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    double tot = 0.0;
    uint64_t cnt = 0;
    uint32_t keep = 0;
    for (uint32_t i = 0; i < ctx->n_timed; ++i) {
        if (ctx->timed_op[i] != op) {
            // compact the slots of other operations to the front
            if (keep != i) {
                hipEvent_t a = ctx->ev_a[keep], b = ctx->ev_b[keep];
                ctx->ev_a[keep] = ctx->ev_a[i];
                ctx->ev_b[keep] = ctx->ev_b[i];
                ctx->ev_a[i] = a;
                ctx->ev_b[i] = b;
                ctx->timed_op[keep] = ctx->timed_op[i];
            }
            ++keep;
            continue;
        }
        HIP_OK(hipEventSynchronize(ctx->ev_b[i]));
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, ctx->ev_a[i], ctx->ev_b[i]));
        tot += ms;
        ++cnt;
    }
    ctx->n_timed = keep;
    *total_ms = tot;
    *count = cnt;
    return BFSC_OK;
}

int bfsc_sync_status(bfsc_ctx *ctx, void *stream) {
    if (!ctx) return BFSC_E_INVAL;
    if (set_device(ctx)) return BFSC_E_HIP;
    HIP_OK(hipStreamSynchronize(S(stream)));
    uint32_t e = 0;
    HIP_OK(hipMemcpy(&e, ctx->err, 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemset(ctx->err, 0, 4));
    HIP_OK(hipDeviceSynchronize());
    if (e & kErrCorrupt) return BFSC_E_CORRUPT;
    if (e & kErrCapacity) return BFSC_E_CAPACITY;
    if (e & kErrInval) return BFSC_E_INVAL;
    return BFSC_OK;
}

const char *bfsc_status_string(int status) {
    switch (status) {
        case BFSC_OK: return "ok";
        case BFSC_E_INVAL: return "invalid argument or input";
        case BFSC_E_CAPACITY: return "output capacity exceeded";
        case BFSC_E_CORRUPT: return "corrupt compressed stream";
        case BFSC_E_HIP: return "HIP runtime error";
        case BFSC_E_UNIMPLEMENTED: return "not implemented";
        default: return "unknown status";
    }
}

}  // extern "C"
