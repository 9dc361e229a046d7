// Top-down BFS level on gfx950: the frontier expansion t = A (x) f followed by
// the visited filter of the baseline BFS algorithm (Romera, arXiv 1704.00513,
// "Our Baseline algorithm": SpMV step, then the element-wise product with the
// complement of the visited list), producing the next frontier as a sorted
// vertex list without sorting: winners mark a next-level bitmap, which is
// compacted in vertex order.
//
// Load balance: each workgroup takes 256 frontier vertices; high-degree
// vertices are expanded by the whole wave (64 <= deg < 2048) or workgroup
// (2048 <= deg < 16384), the rest by a workgroup-wide gather over the
// concatenated small adjacency lists; vertices of degree >= 16384 are cut
// into 8192-edge chunks and queued for a second, grid-wide kernel.
#include "common.hpp"

namespace bfsc {

constexpr uint32_t kExpandThreads = 256;
constexpr uint32_t kMedium = 64, kLarge = 2048, kHuge = 16384, kHugeChunk = 8192;
constexpr uint32_t kCompactWords = 1024;  // bitmap words per compaction chunk

struct BfsWs {
    uint32_t *visited;   // V/32 words
    uint32_t *next_bm;   // V/32 words
    uint32_t *chunk;     // [nchunks + 1] counts then offsets
    uint32_t *qcount;    // [4] huge queue count
    uint4 *queue;        // huge chunks {u, start_lo, start_hi, len}
    uint32_t words, nchunks, qcap;
};

static inline BfsWs bfs_ws_layout(void *ws, uint32_t V, uint64_t n_arcs, size_t *bytes) {
    BfsWs w;
    char *b = (char *)ws;
    size_t off = 0;
    w.words = (V + 31) / 32;
    w.nchunks = (w.words + kCompactWords - 1) / kCompactWords;
    w.qcap = (uint32_t)(n_arcs / kHugeChunk + n_arcs / kHuge + 16);
    w.visited = (uint32_t *)(b + off);
    off = align256(off + (size_t)w.words * 4);
    w.next_bm = (uint32_t *)(b + off);
    off = align256(off + (size_t)w.words * 4);
    w.chunk = (uint32_t *)(b + off);
    off = align256(off + ((size_t)w.nchunks + 1) * 4);
    w.qcount = (uint32_t *)(b + off);
    off = align256(off + 16);
    w.queue = (uint4 *)(b + off);
    off = align256(off + (size_t)w.qcap * 16);
    if (bytes) *bytes = off;
    return w;
}

size_t bfs_ws_bytes_arcs(uint32_t V, uint64_t n_arcs) {
    size_t bytes;
    bfs_ws_layout(nullptr, V, n_arcs, &bytes);
    return bytes;
}

// The arbiter of a visit: the atomic OR on the visited bitmap has exactly one
// winner per vertex; the winner records level and parent and marks the next
// frontier.  A plain read first skips most atomics (bits only ever get set).
__device__ __forceinline__ void visit(uint32_t w, uint32_t u, int32_t nl, const BfsWs &ws,
                                      int32_t *level, int32_t *parent) {
    const uint32_t word = w >> 5, bit = 1u << (w & 31);
    if (ws.visited[word] & bit) return;
    const uint32_t old = atomicOr(&ws.visited[word], bit);
    if (old & bit) return;
    level[w] = nl;
    parent[w] = (int32_t)u;
    atomicOr(&ws.next_bm[word], bit);
}

__global__ __launch_bounds__(kExpandThreads) void k_bfs_expand(
    const uint64_t *row_ptr, const uint32_t *col_idx, const uint32_t *frontier,
    const uint32_t *frontier_len, int32_t *level, int32_t *parent, int32_t nl_host, const int32_t *level_dev, BfsWs ws) {
    // the new level: from the host, or one past the level kept on the device
    const int32_t nl = level_dev ? *level_dev + 1 : nl_host;
    __shared__ uint32_t s_deg_scan[kExpandThreads];
    __shared__ uint32_t s_u[kExpandThreads];
    __shared__ uint64_t s_start[kExpandThreads];
    __shared__ uint32_t s_total;
    __shared__ uint32_t s_big_u, s_big_len;
    __shared__ uint64_t s_big_start;
    __shared__ int s_big_owner;
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint32_t n = *frontier_len;
    for (uint64_t base = (uint64_t)blockIdx.x * kExpandThreads; base < n;
         base += (uint64_t)gridDim.x * kExpandThreads) {
        const uint64_t i = base + tid;
        uint32_t u = 0, deg = 0;
        uint64_t start = 0;
        if (i < n) {
            u = frontier[i];
            start = row_ptr[u];
            deg = (uint32_t)(row_ptr[u + 1] - start);
        }
        // huge: queue 8192-edge chunks for the grid-wide pass
        if (deg >= kHuge) {
            const uint32_t nch = (deg + kHugeChunk - 1) / kHugeChunk;
            const uint32_t q = atomicAdd(ws.qcount, nch);
            for (uint32_t c = 0; c < nch; ++c) {
                if (q + c < ws.qcap) {
                    const uint64_t s = start + (uint64_t)c * kHugeChunk;
                    const uint32_t len = min(kHugeChunk, deg - c * kHugeChunk);
                    ws.queue[q + c] = make_uint4(u, (uint32_t)s, (uint32_t)(s >> 32), len);
                }
            }
            deg = 0;
        }
        // large: whole workgroup, one vertex at a time
        for (;;) {
            if (tid == 0) s_big_owner = -1;
            __syncthreads();
            if (deg >= kLarge) s_big_owner = (int)tid;  // any writer wins
            __syncthreads();
            const int owner = s_big_owner;
            if (owner < 0) break;
            if ((int)tid == owner) {
                s_big_u = u;
                s_big_start = start;
                s_big_len = deg;
                deg = 0;
            }
            __syncthreads();
            const uint32_t bu = s_big_u, blen = s_big_len;
            const uint64_t bs = s_big_start;
            for (uint32_t e = tid; e < blen; e += kExpandThreads) visit(col_idx[bs + e], bu, nl, ws, level, parent);
            __syncthreads();
        }
        // medium: whole wave, one vertex at a time
        for (;;) {
            const uint64_t m = ballot(deg >= kMedium);
            if (!m) break;
            const uint32_t src = (uint32_t)__builtin_ctzll(m);
            const uint32_t mu = readlane(u, src), mlen = readlane(deg, src);
            const uint64_t ms = ((uint64_t)readlane((uint32_t)(start >> 32), src) << 32) |
                                readlane((uint32_t)start, src);
            if (lane == src) deg = 0;
            for (uint32_t e = lane; e < mlen; e += 64) visit(col_idx[ms + e], mu, nl, ws, level, parent);
        }
        // small: gather over the concatenated lists
        uint32_t tot;
        {
            // workgroup exclusive scan of deg (4 waves)
            const uint32_t incl = wave_incl_scan(deg);
            __shared__ uint32_t s_wt[4];
            if (lane == 63) s_wt[tid >> 6] = incl;
            __syncthreads();
            uint32_t wb = 0;
            for (uint32_t q = 0; q < (tid >> 6); ++q) wb += s_wt[q];
            tot = s_wt[0] + s_wt[1] + s_wt[2] + s_wt[3];
            s_deg_scan[tid] = wb + incl - deg;
            s_u[tid] = u;
            s_start[tid] = start;
            if (tid == 0) s_total = tot;
        }
        __syncthreads();
        tot = s_total;
        for (uint32_t e = tid; e < tot; e += kExpandThreads) {
            // owner: last thread whose scan start <= e
            uint32_t lo = 0, hi = kExpandThreads;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s_deg_scan[mid] <= e) lo = mid; else hi = mid;
            }
            visit(col_idx[s_start[lo] + (e - s_deg_scan[lo])], s_u[lo], nl, ws, level, parent);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_bfs_huge(const uint32_t *col_idx, int32_t *level,
                                                  int32_t *parent, int32_t nl_host,
                                                  const int32_t *level_dev, BfsWs ws) {
    const int32_t nl = level_dev ? *level_dev + 1 : nl_host;
    const uint32_t nq = min(*ws.qcount, ws.qcap);
    for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const uint4 c = ws.queue[q];
        const uint64_t s = ((uint64_t)c.z << 32) | c.y;
        for (uint32_t e = threadIdx.x; e < c.w; e += blockDim.x) visit(col_idx[s + e], c.x, nl, ws, level, parent);
    }
}

// Compaction, pass 1: set bits per chunk of the next-level bitmap.
__global__ __launch_bounds__(256) void k_bfs_count(BfsWs ws) {
    __shared__ uint32_t s_w[4];
    const uint32_t c = blockIdx.x, tid = threadIdx.x;
    const uint32_t w0 = c * kCompactWords;
    uint32_t cnt = 0;
    for (uint32_t k = tid; k < kCompactWords; k += 256) {
        const uint32_t wi = w0 + k;
        if (wi < ws.words) cnt += __popc(ws.next_bm[wi]);
    }
    cnt = wave_sum(cnt);
    if ((tid & 63) == 0) s_w[tid >> 6] = cnt;
    __syncthreads();
    if (tid == 0) ws.chunk[c] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Pass 2: exclusive scan of the chunk counts (one workgroup); total -> next_len.
__global__ __launch_bounds__(1024) void k_bfs_scan(BfsWs ws, uint32_t *next_len) {
    __shared__ uint32_t s_wt[16];
    __shared__ uint32_t s_carry;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < ws.nchunks; base += 1024) {
        const uint32_t i = base + tid;
        const uint32_t v = i < ws.nchunks ? ws.chunk[i] : 0u;
        const uint32_t incl = wave_incl_scan(v);
        if (lane == 63) s_wt[w] = incl;
        __syncthreads();
        uint32_t wb = 0, tot = 0;
        for (uint32_t q = 0; q < 16; ++q) {
            wb += q < w ? s_wt[q] : 0u;
            tot += s_wt[q];
        }
        const uint32_t carry = s_carry;
        if (i < ws.nchunks) ws.chunk[i] = carry + wb + incl - v;
        __syncthreads();
        if (tid == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (tid == 0) {
        ws.chunk[ws.nchunks] = s_carry;
        *next_len = s_carry;
        *ws.qcount = 0;  // huge queue is empty for the next level
    }
}

// Pass 3: write the set bits' vertex IDs in order and clear the bitmap.
__global__ __launch_bounds__(256) void k_bfs_emit(BfsWs ws, uint32_t *next) {
    __shared__ uint32_t s_wt[4];
    const uint32_t c = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const uint32_t w0 = c * kCompactWords + tid * 4;  // 4 consecutive words per thread
    uint32_t x[4], cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = (w0 + k < ws.words) ? ws.next_bm[w0 + k] : 0u;
        cnt += __popc(x[k]);
    }
    const uint32_t incl = wave_incl_scan(cnt);
    if (lane == 63) s_wt[tid >> 6] = incl;
    __syncthreads();
    uint32_t wb = 0;
    for (uint32_t q = 0; q < (tid >> 6); ++q) wb += s_wt[q];
    uint32_t pos = ws.chunk[c] + wb + incl - cnt;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t v = x[k];
        while (v) {
            const uint32_t b = __builtin_ctz(v);
            v &= v - 1;
            next[pos++] = (w0 + k) * 32 + b;
        }
        if (x[k]) ws.next_bm[w0 + k] = 0u;
    }
}

__global__ void k_bfs_fill(int32_t *level, int32_t *parent, uint32_t V, BfsWs ws) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
        level[i] = -1;
        parent[i] = -1;
    }
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ws.words; i += stride) {
        ws.visited[i] = 0u;
        ws.next_bm[i] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *ws.qcount = 0;
}

__global__ void k_bfs_root(uint32_t root, int32_t *level, int32_t *parent, uint32_t *frontier,
                           uint32_t *frontier_len, BfsWs ws) {
    level[root] = 0;
    parent[root] = (int32_t)root;
    ws.visited[root >> 5] |= 1u << (root & 31);
    frontier[0] = root;
    *frontier_len = 1;
}

int launch_bfs_init(bfsc_ctx *ctx, const bfsc_csr *g, uint32_t root, int32_t *level,
                    int32_t *parent, uint32_t *frontier, uint32_t *frontier_len, void *wsp,
                    hipStream_t s) {
    BfsWs ws = bfs_ws_layout(wsp, g->n_vertices, g->n_arcs, nullptr);
    const uint32_t grid = (uint32_t)ctx->n_cu * 8;
    hipLaunchKernelGGL(k_bfs_fill, dim3(grid), dim3(256), 0, s, level, parent, g->n_vertices, ws);
    hipLaunchKernelGGL(k_bfs_root, dim3(1), dim3(1), 0, s, root, level, parent, frontier,
                       frontier_len, ws);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

// Increments the device-side level (end of a captured pipeline step).
__global__ void k_level_inc(int32_t *level_dev) { *level_dev += 1; }

int launch_level_inc(int32_t *level_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_level_inc, dim3(1), dim3(1), 0, s, level_dev);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

// cur_level_dev != NULL: the current level is read on the device (for
// replayed graphs); otherwise cur_level is used.
int launch_bfs_level(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *frontier,
                     const uint32_t *frontier_len, int32_t *level, int32_t *parent, uint32_t *next,
                     uint32_t *next_len, void *wsp, hipStream_t s, const int32_t *cur_level_dev) {
    BfsWs ws = bfs_ws_layout(wsp, g->n_vertices, g->n_arcs, nullptr);
    const int32_t nl = cur_level + 1;
    const uint32_t grid = (uint32_t)ctx->n_cu * 8;
    const int slot = timing_begin(ctx, BFSC_OP_BFS, s);
    hipLaunchKernelGGL(k_bfs_expand, dim3(grid), dim3(kExpandThreads), 0, s, g->row_ptr, g->col_idx,
                       frontier, frontier_len, level, parent, nl, cur_level_dev, ws);
    hipLaunchKernelGGL(k_bfs_huge, dim3((uint32_t)ctx->n_cu * 4), dim3(256), 0, s, g->col_idx, level,
                       parent, nl, cur_level_dev, ws);
    hipLaunchKernelGGL(k_bfs_count, dim3(ws.nchunks), dim3(256), 0, s, ws);
    hipLaunchKernelGGL(k_bfs_scan, dim3(1), dim3(1024), 0, s, ws, next_len);
    hipLaunchKernelGGL(k_bfs_emit, dim3(ws.nchunks), dim3(256), 0, s, ws, next);
    timing_end(ctx, slot, s);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

}  // namespace bfsc
