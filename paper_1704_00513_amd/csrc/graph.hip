// Runtime around the kernels: a per-level BFS + compression pipeline
// captured into HIP graphs, and the launch-shape autotuner.
//
// One pipeline step compresses the current frontier F_L by destination range
// and decompresses it (the compress -> exchange -> decompress of the paper's
// BFS-with-compression algorithm, with the exchange left out on one GPU),
// then expands F_L into F_{L+1}.  The level number lives on the device, so
// one graph per frontier buffer parity (even / odd level) replays every
// level; the host reads back one 4-byte frontier length per level.
#include <stdlib.h>
#include <string.h>

#include <new>

#include "common.hpp"

namespace bfsc {
size_t bfs_ws_bytes_arcs(uint32_t V, uint64_t n_arcs);
}

using namespace bfsc;

struct bfsc_pipeline {
    bfsc_ctx *ctx;
    bfsc_csr g;
    uint32_t nseg;
    int mode;
    uint32_t *front[2];
    uint32_t *flen;        // [2]
    int32_t *level, *parent, *level_dev;
    uint32_t *bounds, *seg_lo, *seg_hi;
    int32_t *seg_level;
    uint64_t *seg_off, *sbo, *doff;
    uint8_t *out, *classes;
    size_t out_cap;
    uint32_t *dec;
    void *bfs_ws, *enc_ws, *dec_ws;
    hipStream_t cap;
    hipGraph_t graph[2];
    hipGraphExec_t exec[2];
    int parity;
    int captured;
};

namespace {

__global__ void k_pipe_setup(const uint32_t *bounds, uint32_t nseg, uint32_t *seg_lo,
                             uint32_t *seg_hi, int32_t *level_dev) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nseg; r += gridDim.x * blockDim.x) {
        seg_lo[r] = bounds[r];
        seg_hi[r] = bounds[r + 1];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *level_dev = 0;
}

__global__ void k_fill_level(int32_t *seg_level, uint32_t nseg, const int32_t *level_dev) {
    const int32_t L = *level_dev;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < nseg; r += gridDim.x * blockDim.x)
        seg_level[r] = L;
}

template <typename T>
int dalloc(T **p, size_t bytes) {
    return hipMalloc((void **)p, bytes ? bytes : 4) == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

// The launches of one step, on stream s, for frontier parity p.
int enqueue_step(bfsc_pipeline *P, int p, hipStream_t s) {
    bfsc_ctx *ctx = P->ctx;
    const uint32_t V = P->g.n_vertices;
    int st = launch_partition(P->front[p], P->flen + p, P->bounds, P->nseg, P->seg_off, s);
    if (st) return st;
    hipLaunchKernelGGL(k_fill_level, dim3(1), dim3(256), 0, s, P->seg_level, P->nseg, P->level_dev);
    bfsc_batch b;
    b.ids = P->front[p];
    b.seg_off = P->seg_off;
    b.seg_lo = P->seg_lo;
    b.seg_hi = P->seg_hi;
    b.seg_level = P->seg_level;
    b.nseg = P->nseg;
    b.max_ids = V;
    Plan plan;
    plan_layout(P->enc_ws, V, P->nseg, true, &plan);
    plan.raw_below = ctx->cfg.raw_below;
    st = launch_plan_prep(&b, plan, ctx->err, false, s);
    if (st) return st;
    const uint8_t *cls = nullptr;
    if (P->mode == BFSC_SEL_LEARNED && ctx->cfg.resolve_literal) {
        // literal widths: a separate selection pass (the fused pack pass
        // snaps widths to the minimal one)
        st = launch_select(ctx, &b, BFSC_SEL_LEARNED, P->classes, nullptr, nullptr, plan, s);
        if (st) return st;
        cls = P->classes;
    }
    // learned choice otherwise inside the pack pass, on the matrix cores
    st = launch_encode(ctx, &b, cls, P->mode, P->out, P->out_cap, P->sbo, plan, s);
    if (st) return st;
    st = launch_decode(ctx, P->out, P->sbo, P->nseg, V, P->dec, V, P->doff, P->dec_ws, s);
    if (st) return st;
    st = launch_bfs_level(ctx, &P->g, 0, P->front[p], P->flen + p, P->level, P->parent,
                          P->front[p ^ 1], P->flen + (p ^ 1), P->bfs_ws, s, P->level_dev);
    if (st) return st;
    st = launch_level_inc(P->level_dev, s);
    if (st) return st;
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

void free_pipeline(bfsc_pipeline *P) {
    for (int i = 0; i < 2; ++i) {
        if (P->exec[i]) hipGraphExecDestroy(P->exec[i]);
        if (P->graph[i]) hipGraphDestroy(P->graph[i]);
        hipFree(P->front[i]);
    }
    if (P->cap) hipStreamDestroy(P->cap);
    hipFree(P->flen);
    hipFree(P->level);
    hipFree(P->parent);
    hipFree(P->level_dev);
    hipFree(P->bounds);
    hipFree(P->seg_lo);
    hipFree(P->seg_hi);
    hipFree(P->seg_level);
    hipFree(P->seg_off);
    hipFree(P->sbo);
    hipFree(P->doff);
    hipFree(P->out);
    hipFree(P->classes);
    hipFree(P->dec);
    hipFree(P->bfs_ws);
    hipFree(P->enc_ws);
    hipFree(P->dec_ws);
    delete P;
}

}  // namespace

extern "C" {

int bfsc_pipeline_create(bfsc_ctx *ctx, const bfsc_csr *g, const uint32_t *bounds_host, uint32_t nseg,
                         int mode, int use_graph, bfsc_pipeline **out) {
    if (ctx && mode == BFSC_SEL_DEFAULT) mode = ctx->cfg.selector;
    if (!ctx || !g || !bounds_host || !out || nseg == 0 || g->n_vertices == 0 ||
        g->n_vertices > 0x7FFFFFFFu || mode < BFSC_SEL_PLAIN_BP || mode > BFSC_SEL_LEARNED)
        return BFSC_E_INVAL;
    for (uint32_t r = 0; r < nseg; ++r)
        if (bounds_host[r] > bounds_host[r + 1]) return BFSC_E_INVAL;
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return BFSC_E_HIP;
    bfsc_pipeline *P = new (std::nothrow) bfsc_pipeline();
    if (!P) return BFSC_E_HIP;
    memset(P, 0, sizeof(*P));
    P->ctx = ctx;
    P->g = *g;
    P->nseg = nseg;
    P->mode = mode;
    const uint64_t V = g->n_vertices;
    size_t cap = 0;
    bfsc_encode_bound(V, nseg, &cap);
    P->out_cap = cap;
    int st = BFSC_OK;
    st |= dalloc(&P->front[0], V * 4);
    st |= dalloc(&P->front[1], V * 4);
    st |= dalloc(&P->flen, 16);
    st |= dalloc(&P->level, V * 4);
    st |= dalloc(&P->parent, V * 4);
    st |= dalloc(&P->level_dev, 16);
    st |= dalloc(&P->bounds, ((size_t)nseg + 1) * 4);
    st |= dalloc(&P->seg_lo, (size_t)nseg * 4);
    st |= dalloc(&P->seg_hi, (size_t)nseg * 4);
    st |= dalloc(&P->seg_level, (size_t)nseg * 4);
    st |= dalloc(&P->seg_off, ((size_t)nseg + 1) * 8);
    st |= dalloc(&P->sbo, ((size_t)nseg + 1) * 8);
    st |= dalloc(&P->doff, ((size_t)nseg + 1) * 8);
    st |= dalloc(&P->out, cap);
    st |= dalloc(&P->classes, (V + kBlock - 1) / kBlock + nseg);
    st |= dalloc(&P->dec, V * 4);
    st |= dalloc((char **)&P->bfs_ws, bfs_ws_bytes_arcs(g->n_vertices, g->n_arcs));
    st |= dalloc((char **)&P->enc_ws, plan_layout(nullptr, V, nseg, true, nullptr));
    st |= dalloc((char **)&P->dec_ws, decode_ws_bytes(V, nseg));
    if (st != BFSC_OK ||
        hipMemcpy(P->bounds, bounds_host, ((size_t)nseg + 1) * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess) {
        free_pipeline(P);
        return BFSC_E_HIP;
    }
    hipLaunchKernelGGL(k_pipe_setup, dim3(1), dim3(256), 0, P->cap, P->bounds, nseg, P->seg_lo,
                       P->seg_hi, P->level_dev);
    if (hipStreamSynchronize(P->cap) != hipSuccess) {
        free_pipeline(P);
        return BFSC_E_HIP;
    }
    if (use_graph) {
        // event timing stays out of the captured graphs
        const int timing = ctx->timing;
        ctx->timing = 0;
        for (int p = 0; p < 2 && st == BFSC_OK; ++p) {
            if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                st = BFSC_E_HIP;
                break;
            }
            const int est = enqueue_step(P, p, P->cap);
            const hipError_t ce = hipStreamEndCapture(P->cap, &P->graph[p]);
            if (est != BFSC_OK || ce != hipSuccess) {
                st = est != BFSC_OK ? est : BFSC_E_HIP;
                break;
            }
            if (hipGraphInstantiate(&P->exec[p], P->graph[p], nullptr, nullptr, 0) != hipSuccess)
                st = BFSC_E_HIP;
        }
        ctx->timing = timing;
        if (st != BFSC_OK) {
            free_pipeline(P);
            return st;
        }
        P->captured = 1;
    }
    *out = P;
    return BFSC_OK;
}

int bfsc_pipeline_destroy(bfsc_pipeline *P) {
    if (!P) return BFSC_E_INVAL;
    hipSetDevice(P->ctx->device);
    hipDeviceSynchronize();
    free_pipeline(P);
    return BFSC_OK;
}

int bfsc_pipeline_start(bfsc_pipeline *P, uint32_t root, void *stream) {
    if (!P || root >= P->g.n_vertices) return BFSC_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    int st = launch_bfs_init(P->ctx, &P->g, root, P->level, P->parent, P->front[0], P->flen + 0,
                             P->bfs_ws, s);
    if (st) return st;
    hipLaunchKernelGGL(k_pipe_setup, dim3(1), dim3(256), 0, s, P->bounds, P->nseg, P->seg_lo,
                       P->seg_hi, P->level_dev);
    P->parity = 0;
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int bfsc_pipeline_step(bfsc_pipeline *P, void *stream, uint32_t *next_len_host) {
    if (!P) return BFSC_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const int p = P->parity;
    int st;
    if (P->captured) {
        const int slot = timing_begin(P->ctx, BFSC_OP_PIPELINE, s);
        st = hipGraphLaunch(P->exec[p], s) == hipSuccess ? BFSC_OK : BFSC_E_HIP;
        timing_end(P->ctx, slot, s);
    } else {
        const int slot = timing_begin(P->ctx, BFSC_OP_PIPELINE, s);
        st = enqueue_step(P, p, s);
        timing_end(P->ctx, slot, s);
    }
    if (st) return st;
    P->parity = p ^ 1;
    if (next_len_host) {
        if (hipMemcpyAsync(next_len_host, P->flen + (p ^ 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return BFSC_E_HIP;
    }
    return BFSC_OK;
}

int bfsc_pipeline_buffers(const bfsc_pipeline *P, bfsc_pipeline_bufs *b) {
    if (!P || !b) return BFSC_E_INVAL;
    const int cur = P->parity;  // holds the frontier the next step compresses
    b->frontier = P->front[cur];
    b->frontier_len = P->flen + cur;
    b->prev_frontier = P->front[cur ^ 1];
    b->prev_frontier_len = P->flen + (cur ^ 1);
    b->level = P->level;
    b->parent = P->parent;
    b->seg_off = P->seg_off;
    b->stream = P->out;
    b->stream_cap = P->out_cap;
    b->seg_byte_off = P->sbo;
    b->decoded = P->dec;
    b->decoded_off = P->doff;
    b->classes = P->classes;
    return BFSC_OK;
}

int bfsc_memcpy(void *dst, const void *src, size_t bytes) {
    if ((!dst || !src) && bytes) return BFSC_E_INVAL;
    if (!bytes) return BFSC_OK;
    return hipMemcpy(dst, src, bytes, hipMemcpyDefault) == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

// Tries encode and decode launch shapes on a sample batch and keeps the
// fastest (event-timed on `stream`).  Allocates and frees its own buffers.
int bfsc_autotune(bfsc_ctx *ctx, const bfsc_batch *sample, void *ws, void *stream) {
    if (!ctx || !sample || !ws || !sample->ids || sample->nseg == 0) return BFSC_E_INVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return BFSC_E_HIP;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t N = sample->max_ids;
    size_t cap = 0;
    bfsc_encode_bound(N, sample->nseg, &cap);
    uint8_t *out = nullptr;
    uint64_t *sbo = nullptr, *doff = nullptr;
    uint32_t *dec = nullptr;
    void *dws = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = BFSC_OK;
    st |= dalloc(&out, cap);
    st |= dalloc(&sbo, ((size_t)sample->nseg + 1) * 8);
    st |= dalloc(&doff, ((size_t)sample->nseg + 1) * 8);
    st |= dalloc(&dec, N * 4 + 4);
    st |= dalloc((char **)&dws, decode_ws_bytes(N, sample->nseg));
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = BFSC_E_HIP;
    const bfsc_tune keep = ctx->tune;
    const int timing = ctx->timing;
    ctx->timing = 0;
    // {waves per workgroup, workgroups per CU, pack variant}
    static const uint32_t kEnc[][3] = {{4, 8, 6}, {4, 8, 4}, {4, 8, 2}, {4, 8, 7}, {2, 16, 6},
                                       {8, 4, 6}, {4, 8, 0}};
    // {waves per workgroup, workgroups per CU, decoder variant}
    static const uint32_t kDec[][3] = {{4, 8, 3}, {4, 8, 2}, {4, 8, 1}, {2, 16, 3}, {8, 4, 3},
                                       {4, 8, 0}, {4, 8, 6}};
    bfsc_tune best = keep;
    float best_e = 1e30f, best_d = 1e30f;
    for (const auto &c : kEnc) {
        if (st) break;
        ctx->tune.enc_waves = c[0];
        ctx->tune.enc_wg_per_cu = c[1];
        ctx->tune.enc_pack = c[2];
        float tot = 0.0f;
        for (int rep = 0; rep < 4 && !st; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess) st = BFSC_E_HIP;
            st |= bfsc_encode(ctx, sample, nullptr, BFSC_SEL_EXHAUSTIVE, out, cap, sbo, ws, s);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) st = BFSC_E_HIP;
            float ms = 0.0f;
            hipEventElapsedTime(&ms, e0, e1);
            if (rep) tot += ms;  // first run warms up
        }
        if (!st && tot < best_e) {
            best_e = tot;
            best.enc_waves = c[0];
            best.enc_wg_per_cu = c[1];
            best.enc_pack = c[2];
        }
    }
    ctx->tune.enc_waves = best.enc_waves;
    ctx->tune.enc_wg_per_cu = best.enc_wg_per_cu;
    ctx->tune.enc_pack = best.enc_pack;
    if (!st) st |= bfsc_encode(ctx, sample, nullptr, BFSC_SEL_EXHAUSTIVE, out, cap, sbo, ws, s);
    for (const auto &c : kDec) {
        if (st) break;
        ctx->tune.dec_waves = c[0];
        ctx->tune.dec_wg_per_cu = c[1];
        ctx->tune.dec_mode = c[2];
        float tot = 0.0f;
        for (int rep = 0; rep < 4 && !st; ++rep) {
            if (hipEventRecord(e0, s) != hipSuccess) st = BFSC_E_HIP;
            st |= bfsc_decode(ctx, out, sbo, sample->nseg, N, dec, N + 1, doff, dws, s);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) st = BFSC_E_HIP;
            float ms = 0.0f;
            hipEventElapsedTime(&ms, e0, e1);
            if (rep) tot += ms;
        }
        if (!st && tot < best_d) {
            best_d = tot;
            best.dec_waves = c[0];
            best.dec_wg_per_cu = c[1];
            best.dec_mode = c[2];
        }
    }
    ctx->timing = timing;
    ctx->tune = st ? keep : best;
    if (!st) tune_cache_store(ctx);
    hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(out);
    hipFree(sbo);
    hipFree(doff);
    hipFree(dec);
    hipFree(dws);
    return st ? BFSC_E_HIP : BFSC_OK;
}

}  // extern "C"
