// BFS level on gfx950.  Top-down: the frontier expansion t = A (x) f followed
// by the visited filter of the baseline BFS algorithm (Romera, arXiv
// 1704.00513, "Our Baseline algorithm": SpMV step, then the element-wise
// product with the complement of the visited list).  Bottom-up, on the levels
// the direction rule picks (the paper's related work, "Direction
// optimization"): each unvisited vertex looks for a frontier neighbour.  The
// next frontier comes out as a sorted vertex list without sorting: winners
// mark a next-level bitmap, which is compacted in vertex order.  The
// candidate exchange of the compressed 2D BFS (end of this file) reuses the
// top-down expansion.
//
// Load balance: each workgroup takes 256 frontier vertices; vertices of
// degree < 512 are expanded by a workgroup-wide gather over their
// concatenated adjacency lists; vertices of degree >= 512 are cut into
// 2048-edge chunks and queued for a second, grid-wide kernel (a small
// frontier of hubs then still fills the chip).
#include "common.hpp"
#include "exchange.hpp"

namespace bfsc {

constexpr uint32_t kExpandThreads = 256;
constexpr uint32_t kHuge = 512, kHugeChunk = 2048;
constexpr uint32_t kCompactWords = 1024;  // bitmap words per compaction chunk

struct BfsWs {
    uint32_t *visited;   // V/32 words
    uint32_t *next_bm;   // V/32 words
    uint32_t *chunk;     // [nchunks + 1] counts then offsets
    uint32_t *qcount;    // [4] huge queue count
    uint4 *queue;        // huge chunks {u, start_lo, start_hi, len}
    uint32_t *front_bm;  // V/32 words: the current frontier as a bitmap (bottom-up levels read it)
    unsigned long long *stat;  // direction state, see k_bfs_decide
    unsigned long long *part;  // [kParts] per-workgroup sums of the new frontier's arcs
    uint32_t words, nchunks, qcap;
};

// Workgroups of the kernels that sum the new frontier's arcs (k_bfs_bu,
// k_bfs_arcs): each writes its own partial sum, since same-address atomics
// from every workgroup of the chip serialise.
constexpr uint32_t kParts = 4096;

// Direction state (stat[]): [0] arcs of the unvisited vertices, [1] the
// previous frontier's size, [2] this level's direction (0 top-down, 1
// bottom-up), [3] the root's arcs (later frontiers' arcs come as partial sums).
enum { kStatMu = 0, kStatPrevN = 1, kStatDir = 2, kStatMf = 3 };

static inline BfsWs bfs_ws_layout(void *ws, uint32_t V, uint64_t n_arcs, size_t *bytes) {
    BfsWs w;
    char *b = (char *)ws;
    size_t off = 0;
    w.words = (V + 31) / 32;
    w.nchunks = (w.words + kCompactWords - 1) / kCompactWords;
    // a vertex of degree d >= kHuge gives at most d / kHugeChunk + 1 chunks,
    // and fewer than n_arcs / kHuge such vertices exist
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
    w.front_bm = (uint32_t *)(b + off);
    off = align256(off + (size_t)w.words * 4);
    w.stat = (unsigned long long *)(b + off);
    off = align256(off + 32);
    w.part = (unsigned long long *)(b + off);
    off = align256(off + (size_t)kParts * 8);
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

// What an arc (u, w) of the frontier does, for the expansion kernels below:
// tag(u) is computed once per frontier vertex and handed to every one of its
// arcs, visit(w, tag) handles one arc.
struct BfsVisit {  // a BFS level: the visited filter, level and parent
    BfsWs ws;
    int32_t *level, *parent;
    int32_t nl;                // the new level, from the host ...
    const int32_t *level_dev;  // ... or one past the level kept on the device
    const unsigned long long *dir;  // the level's direction (null: always top-down)
    __device__ void begin() {
        if (level_dev) nl = *level_dev + 1;
    }
    // false on a bottom-up level: the expansion kernels then do nothing
    __device__ bool active() const { return !dir || *dir == 0ull; }
    __device__ uint32_t tag(uint32_t u) const { return u; }
    __device__ void operator()(uint32_t w, uint32_t u) const { visit(w, u, nl, ws, level, parent); }
};

struct CandVisit {  // the candidate exchange: bit w of the owner's bitmap, visited or not
    const uint32_t *bounds;
    uint32_t R, words;
    uint32_t *cand;  // R bitmaps of `words` words each
    __device__ void begin() {}
    __device__ bool active() const { return true; }
    __device__ uint32_t tag(uint32_t u) const { return upper_bound_m1(bounds, R, u) * words; }
    __device__ void operator()(uint32_t w, uint32_t base) const {
        uint32_t *p = cand + base + (w >> 5);
        const uint32_t bit = 1u << (w & 31);
        if (*p & bit) return;  // bits only get set: skip most atomics
        atomicOr(p, bit);
    }
};

template <class Visit>
__global__ __launch_bounds__(kExpandThreads) void k_bfs_expand(
    const uint64_t *row_ptr, const uint32_t *col_idx, const uint32_t *frontier,
    const uint32_t *frontier_len, Visit vis, BfsWs ws) {
    if (!vis.active()) return;  // uniform over the grid
    vis.begin();
    __shared__ uint32_t s_deg_scan[kExpandThreads];
    __shared__ uint32_t s_u[kExpandThreads];
    __shared__ uint64_t s_start[kExpandThreads];
    __shared__ uint32_t s_total;
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint32_t n = *frontier_len;
    for (uint64_t base = (uint64_t)blockIdx.x * kExpandThreads; base < n;
         base += (uint64_t)gridDim.x * kExpandThreads) {
        const uint64_t i = base + tid;
        uint32_t u = 0, deg = 0;
        uint64_t start = 0;
        if (i < n) {
            const uint32_t f = frontier[i];
            start = row_ptr[f];
            deg = (uint32_t)(row_ptr[f + 1] - start);
            u = vis.tag(f);
        }
        // huge: queue 2048-edge chunks for the grid-wide pass, one atomic per wave
        {
            const uint32_t nch = deg >= kHuge ? (deg + kHugeChunk - 1) / kHugeChunk : 0u;
            const uint32_t cincl = wave_incl_scan(nch);
            const uint32_t ctot = readlane(cincl, 63);
            if (ctot) {  // uniform over the wave
                uint32_t qb = 0;
                if (lane == 0) qb = atomicAdd(ws.qcount, ctot);
                const uint32_t q = readlane(qb, 0) + cincl - nch;
                for (uint32_t c = 0; c < nch; ++c) {
                    if (q + c < ws.qcap) {  // never false: qcap bounds the chunks of distinct vertices
                        const uint64_t s = start + (uint64_t)c * kHugeChunk;
                        const uint32_t len = min(kHugeChunk, deg - c * kHugeChunk);
                        ws.queue[q + c] = make_uint4(u, (uint32_t)s, (uint32_t)(s >> 32), len);
                    }
                }
                if (nch) deg = 0;
            }
        }
        // the rest: a workgroup-wide gather over the concatenated lists
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
        // four arcs per thread per step, their loads issued together
        for (uint32_t e0 = tid; e0 < tot; e0 += 4 * kExpandThreads) {
            uint32_t x[4], tg[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t e = e0 + k * kExpandThreads;
                x[k] = 0u;
                tg[k] = 0u;
                if (e < tot) {
                    // owner: the last thread whose scan start is <= e
                    uint32_t lo = 0;
#pragma unroll
                    for (uint32_t st = kExpandThreads / 2; st > 0; st >>= 1)
                        if (s_deg_scan[lo + st] <= e) lo += st;
                    tg[k] = s_u[lo];
                    x[k] = col_idx[s_start[lo] + (e - s_deg_scan[lo])];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (e0 + k * kExpandThreads < tot) vis(x[k], tg[k]);
        }
        __syncthreads();
    }
}

template <class Visit>
__global__ __launch_bounds__(256) void k_bfs_huge(const uint32_t *col_idx, Visit vis, BfsWs ws) {
    if (!vis.active()) return;
    vis.begin();
    const uint32_t nq = min(*ws.qcount, ws.qcap);
    for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const uint4 c = ws.queue[q];
        const uint64_t s = ((uint64_t)c.z << 32) | c.y;
        for (uint32_t e = threadIdx.x; e < c.w; e += blockDim.x) vis(col_idx[s + e], c.x);
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

// Pass 3: write the set bits' vertex IDs in order and clear the bitmap; the
// bitmap becomes the frontier bitmap of the next level.
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
        if (w0 + k < ws.words) ws.front_bm[w0 + k] = x[k];
    }
}

// Sum over a 256-thread workgroup (every thread calls it).
__device__ __forceinline__ unsigned long long block_sum64(unsigned long long x) {
    __shared__ unsigned long long s_w[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    return s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// The new frontier's arcs after a top-down level, summed for the direction
// choice of the next level (one ID per thread, a partial sum per workgroup);
// a bottom-up level sums its winners' arcs itself.
__global__ __launch_bounds__(256) void k_bfs_arcs(const uint32_t *next, const uint32_t *next_len,
                                                  const uint64_t *row_ptr, BfsWs ws) {
    if (ws.stat[kStatDir] != 0ull) return;  // uniform over the grid
    const uint32_t n = *next_len;
    unsigned long long arcs = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t v = next[i];
        arcs += row_ptr[v + 1] - row_ptr[v];
    }
    arcs = block_sum64(arcs);
    if (threadIdx.x == 0) ws.part[blockIdx.x] = arcs;
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
        ws.front_bm[i] = 0u;
    }
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kParts; i += stride) ws.part[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ws.qcount = 0;
}

__global__ void k_bfs_root(uint32_t root, int32_t *level, int32_t *parent, uint32_t *frontier,
                           uint32_t *frontier_len, BfsWs ws, const uint64_t *row_ptr, uint64_t n_arcs) {
    level[root] = 0;
    parent[root] = (int32_t)root;
    ws.visited[root >> 5] |= 1u << (root & 31);
    ws.front_bm[root >> 5] |= 1u << (root & 31);
    frontier[0] = root;
    *frontier_len = 1;
    ws.stat[kStatMu] = n_arcs;
    ws.stat[kStatPrevN] = 0ull;
    ws.stat[kStatDir] = 0ull;
    ws.stat[kStatMf] = row_ptr[root + 1] - row_ptr[root];
}

// Direction of the coming level (direction-optimizing BFS, Beamer, Asanovic
// and Patterson, SC 2012): with m_f the frontier's arcs and m_u the arcs of
// the unvisited vertices, a top-down traversal turns bottom-up when
// m_f > m_u / alpha while the frontier grows, and a bottom-up one turns back
// when the frontier holds fewer than V / beta vertices while it shrinks.
// One workgroup of 256 threads: it first adds up the partial sums of the
// new frontier's arcs left by the previous level (nparts of them).
__global__ __launch_bounds__(256) void k_bfs_decide(BfsWs ws, const uint32_t *frontier_len, uint32_t V,
                                                    float alpha, float beta, uint32_t nparts) {
    unsigned long long part = 0;
    for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) part += ws.part[i];
    part = block_sum64(part);
    if (threadIdx.x != 0) return;
    unsigned long long *st = ws.stat;
    const unsigned long long mf = st[kStatMf] + part;
    const unsigned long long mu = st[kStatMu] - min(mf, st[kStatMu]);  // the frontier is visited now
    const unsigned long long nf = *frontier_len, prev = st[kStatPrevN];
    unsigned long long dir = st[kStatDir];
    if (dir == 0ull) {
        if ((double)mf * alpha > (double)mu && nf > prev) dir = 1ull;
    } else if ((double)nf * beta < (double)V && nf < prev) {
        dir = 0ull;
    }
    st[kStatMu] = mu;
    st[kStatMf] = 0ull;  // only the root's arcs come this way
    st[kStatPrevN] = nf;
    st[kStatDir] = dir;
}

// A bottom-up level: every unvisited vertex looks through its own
// neighbours for one on the frontier (the frontier bitmap) and stops at the
// first.  A wave owns 64 consecutive vertices, i.e. two bitmap words, so the
// visited and next-level words are written by one lane without atomics.
__global__ __launch_bounds__(256) void k_bfs_bu(const uint64_t *row_ptr, const uint32_t *col_idx, int32_t *level,
                                                int32_t *parent, int32_t nl_host, const int32_t *level_dev,
                                                BfsWs ws, uint32_t V) {
    if (ws.stat[kStatDir] == 0ull) return;  // uniform over the grid
    const int32_t nl = level_dev ? *level_dev + 1 : nl_host;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    unsigned long long acc = 0;  // the winners' arcs, for the next direction choice
    for (uint64_t wv = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); wv * 64 < V; wv += nwaves) {
        const uint32_t v = (uint32_t)(wv * 64) + lane;
        bool found = false;
        uint32_t par = 0;
        if (v < V && !((ws.visited[v >> 5] >> (v & 31)) & 1u)) {
            const uint64_t e0 = row_ptr[v], e1 = row_ptr[v + 1];
            for (uint64_t e = e0; e < e1; ++e) {
                const uint32_t u = col_idx[e];
                if ((ws.front_bm[u >> 5] >> (u & 31)) & 1u) {
                    found = true;
                    par = u;
                    acc += e1 - e0;
                    break;
                }
            }
        }
        if (found) {
            level[v] = nl;
            parent[v] = (int32_t)par;
        }
        const uint64_t m = ballot(found);
        const uint32_t wi = (uint32_t)(wv * 2) + (lane >> 5), bits = lane < 32 ? (uint32_t)m : (uint32_t)(m >> 32);
        if ((lane & 31) == 0 && bits) {
            ws.visited[wi] |= bits;
            ws.next_bm[wi] = bits;  // cleared by the previous emit pass
        }
    }
    acc = block_sum64(acc);
    if (threadIdx.x == 0) ws.part[blockIdx.x] = acc;
}

int launch_bfs_init(bfsc_ctx *ctx, const bfsc_csr *g, uint32_t root, int32_t *level,
                    int32_t *parent, uint32_t *frontier, uint32_t *frontier_len, void *wsp,
                    hipStream_t s) {
    BfsWs ws = bfs_ws_layout(wsp, g->n_vertices, g->n_arcs, nullptr);
    const uint32_t grid = (uint32_t)ctx->n_cu * 8;
    hipLaunchKernelGGL(k_bfs_fill, dim3(grid), dim3(256), 0, s, level, parent, g->n_vertices, ws);
    hipLaunchKernelGGL(k_bfs_root, dim3(1), dim3(1), 0, s, root, level, parent, frontier,
                       frontier_len, ws, g->row_ptr, g->n_arcs);
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
    const bool dopt = ctx->bfs_alpha > 0.f;
    // k_bfs_bu and k_bfs_arcs run on the same grid, so whichever ran last
    // level wrote every partial sum that k_bfs_decide adds up
    const uint32_t dgrid = min(grid, kParts);
    if (dopt)
        hipLaunchKernelGGL(k_bfs_decide, dim3(1), dim3(256), 0, s, ws, frontier_len, g->n_vertices, ctx->bfs_alpha,
                           ctx->bfs_beta, dgrid);
    const BfsVisit vis{ws, level, parent, nl, cur_level_dev, dopt ? ws.stat + kStatDir : nullptr};
    hipLaunchKernelGGL(k_bfs_expand<BfsVisit>, dim3(grid), dim3(kExpandThreads), 0, s, g->row_ptr, g->col_idx,
                       frontier, frontier_len, vis, ws);
    hipLaunchKernelGGL(k_bfs_huge<BfsVisit>, dim3((uint32_t)ctx->n_cu * 4), dim3(256), 0, s, g->col_idx, vis, ws);
    if (dopt)
        hipLaunchKernelGGL(k_bfs_bu, dim3(dgrid), dim3(256), 0, s, g->row_ptr, g->col_idx, level, parent, nl,
                           cur_level_dev, ws, g->n_vertices);
    hipLaunchKernelGGL(k_bfs_count, dim3(ws.nchunks), dim3(256), 0, s, ws);
    hipLaunchKernelGGL(k_bfs_scan, dim3(1), dim3(1024), 0, s, ws, next_len);
    hipLaunchKernelGGL(k_bfs_emit, dim3(ws.nchunks), dim3(256), 0, s, ws, next);
    if (dopt)
        hipLaunchKernelGGL(k_bfs_arcs, dim3(dgrid), dim3(256), 0, s, next, next_len, g->row_ptr, ws);
    timing_end(ctx, slot, s);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

// ------------------------------------------------------------------ candidate exchange

// The row exchange of the compressed 2D BFS (the candidate vector t = A x f,
// compressed and sent to the owners before the element-wise filter with the
// complement of the visited list, in the paper's algorithm with compression
// integrated), on one GPU.  The vertex range is split by bounds[0..R] into R
// owners.  Owner p's frontier vertices (those in [bounds[p], bounds[p+1]))
// expand into owner p's candidate bitmap, visited or not (the expansion
// kernels of a BFS level, with the candidate visitor); the R bitmaps are
// compacted as one, owner after owner, which is the order of the segments
// (p, d) of the batch; the receiver ORs every decoded candidate
// into one bitmap and keeps what is not yet visited.

// Workspace: the merge bitmap (first, so that its place does not depend on
// R), R candidate bitmaps of ceil(V/32) words (compacted through a BfsWs
// view), the candidate count.
struct ExWs {
    uint32_t *merged;
    BfsWs cb;        // next_bm: the R bitmaps back to back (words = R * V/32)
    uint32_t *count; // [4] [0]: candidates found, [1]: kept (capacity)
    uint32_t words;  // V/32 (rounded up)
};

static inline ExWs ex_ws_layout(void *ws, uint32_t V, uint64_t n_arcs, uint32_t nseg, size_t *bytes) {
    ExWs w;
    char *b = (char *)ws;
    size_t off = 0;
    w.words = (V + 31) / 32;
    w.merged = (uint32_t *)(b + off);
    off = align256(off + (size_t)w.words * 4);
    const uint64_t cw = (uint64_t)w.words * nseg;
    w.cb.visited = nullptr;
    w.cb.next_bm = (uint32_t *)(b + off);
    off = align256(off + cw * 4);
    w.cb.words = (uint32_t)cw;
    w.cb.nchunks = (uint32_t)((cw + kCompactWords - 1) / kCompactWords);
    w.cb.chunk = (uint32_t *)(b + off);
    off = align256(off + ((size_t)w.cb.nchunks + 1) * 4);
    w.cb.qcap = (uint32_t)(n_arcs / kHugeChunk + n_arcs / kHuge + 16);
    w.cb.qcount = (uint32_t *)(b + off);  // the expansion's queue of huge vertices
    off = align256(off + 16);
    w.cb.queue = (uint4 *)(b + off);
    off = align256(off + (size_t)w.cb.qcap * 16);
    w.cb.front_bm = nullptr;  // the candidate compaction uses k_ex_emit, which has no frontier bitmap
    w.cb.stat = nullptr;
    w.cb.part = nullptr;
    w.count = (uint32_t *)(b + off);
    off = align256(off + 16);
    if (bytes) *bytes = off;
    return w;
}

size_t ex_ws_bytes(uint32_t V, uint64_t n_arcs, uint32_t nseg) {
    size_t bytes;
    ex_ws_layout(nullptr, V, n_arcs, nseg, &bytes);
    return bytes;
}

__global__ void k_ex_zero(uint32_t *a, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0u;
}

// The owners must cover [0, V) in order (else the batch is flagged invalid).
__global__ void k_ex_check(const uint32_t *bounds, uint32_t R, uint32_t V, uint32_t *err) {
    bool ok = bounds[0] == 0 && bounds[R] == V;
    for (uint32_t r = 0; r < R; ++r) ok = ok && bounds[r] <= bounds[r + 1];
    if (!ok) raise_err(err, kErrInval);
}

// Owner p's bitmap is words [p W, (p + 1) W) of the concatenation (W =
// ceil(V/32)), so segment p R + d, owner p's candidates in receiver d's range,
// starts at bit p 32 W + bounds[d]: its offset in the batch is the number of
// candidates before that bit, the chunk's prefix (k_bfs_scan) plus the set
// bits of the chunk's words before it.  One wave per boundary (i = R R is the
// end); offsets past the capacity are clamped to it.  Runs before the
// compaction clears the bitmaps.
__global__ __launch_bounds__(256) void k_ex_segoff(BfsWs ws, const uint32_t *bounds, uint32_t R, uint32_t W,
                                                   uint64_t cap, uint64_t *seg_off) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t RR = (uint64_t)R * R;
    const uint64_t NW = (uint64_t)gridDim.x * 4;
    for (uint64_t i = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i <= RR; i += NW) {
        const uint64_t p = i / R, d = i % R;
        const uint64_t bit = i == RR ? 32ull * W * R : p * 32ull * W + bounds[d];
        const uint64_t word = bit >> 5;
        const uint64_t c = word / kCompactWords;
        uint32_t cnt = 0;
        for (uint64_t q = c * kCompactWords + lane; q < word; q += 64) cnt += __popc(ws.next_bm[q]);
        if (lane == 0 && (bit & 31)) cnt += __popc(ws.next_bm[word] & ((1u << (bit & 31)) - 1u));
        cnt = wave_sum(cnt);
        const uint64_t before = (uint64_t)ws.chunk[c] + cnt;  // chunk[nchunks] holds the total
        if (lane == 0) seg_off[i] = before < cap ? before : cap;
    }
}

// The candidates' vertex IDs in order (k_bfs_emit with a capacity: IDs past
// cap are dropped), the bitmaps cleared for the next call.  Word q of the
// concatenation is word q mod W of owner q / W.
__global__ __launch_bounds__(256) void k_ex_emit(BfsWs ws, uint32_t W, uint32_t *ids, uint64_t cap) {
    __shared__ uint32_t s_wt[4];
    const uint32_t c = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const uint32_t w0 = c * kCompactWords + tid * 4;
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
    uint64_t pos = (uint64_t)ws.chunk[c] + wb + incl - cnt;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t v = x[k];
        const uint32_t vbase = ((w0 + k) % W) * 32u;
        while (v) {
            const uint32_t b = __builtin_ctz(v);
            v &= v - 1;
            if (pos < cap) ids[pos] = vbase + b;
            ++pos;
        }
        if (x[k]) ws.next_bm[w0 + k] = 0u;
    }
}

__global__ void k_ex_clamp(uint32_t *count, uint64_t cap, uint32_t *err) {
    const uint32_t n = count[0];
    count[1] = (uint64_t)n > cap ? (uint32_t)cap : n;
    if ((uint64_t)n > cap) raise_err(err, kErrCapacity);
}

// Each segment's range: receiver d's [bounds[d], bounds[d+1]).
__global__ void k_ex_finish(const uint32_t *bounds, uint32_t R, uint32_t *seg_lo, uint32_t *seg_hi) {
    const uint64_t RR = (uint64_t)R * R;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < RR; i += stride) {
        seg_lo[i] = bounds[i % R];
        seg_hi[i] = bounds[i % R + 1];
    }
}

// Receiver: every decoded candidate into one bitmap (IDs outside [0, V) are
// ignored: a damaged stream is reported by the decoder).  The segments are
// sorted, so neighbouring lanes mostly hit the same word: lanes first OR
// their bits over runs of equal words (a segmented scan across the wave) and
// only the last lane of a run issues the atomic.  Lanes combine only bits of
// their own word, and every lane's bits reach the last lane of its run.
__global__ __launch_bounds__(256) void k_ex_merge(const uint32_t *ids, const uint64_t *n_dev, uint32_t V,
                                                  uint32_t *merged) {
    const uint64_t n = *n_dev, stride = (uint64_t)gridDim.x * blockDim.x;
    const int lane = (int)(threadIdx.x & 63);
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n; base += stride) {  // wave-uniform
        const uint64_t i = base + threadIdx.x;
        uint32_t wd = 0xFFFFFFFFu, bits = 0u;  // no valid word is all ones (V < 2^31)
        if (i < n) {
            const uint32_t w = ids[i];
            if (w < V) {
                wd = w >> 5;
                bits = 1u << (w & 31);
            }
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t ow = (uint32_t)__shfl_up((int)wd, d, 64), ob = (uint32_t)__shfl_up((int)bits, d, 64);
            if (lane >= d && ow == wd) bits |= ob;
        }
        const uint32_t nw = (uint32_t)__shfl_down((int)wd, 1, 64);
        if (bits && (lane == 63 || nw != wd)) atomicOr(&merged[wd], bits);
    }
}

// ... less the visited vertices: the rest are marked visited, get level nl,
// and go to the next-level bitmap (compacted as in a BFS level).  One thread
// per word, so the visited word is updated without atomics.
__global__ void k_ex_filter(uint32_t *merged, BfsWs ws, int32_t *level, int32_t nl) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ws.words; i += stride) {
        const uint32_t m = merged[i];
        if (!m) continue;
        merged[i] = 0u;
        const uint32_t nb = m & ~ws.visited[i];
        if (!nb) continue;
        ws.visited[i] |= nb;
        ws.next_bm[i] |= nb;
        uint32_t v = nb;
        while (v) {
            const uint32_t b = __builtin_ctz(v);
            v &= v - 1;
            level[i * 32 + b] = nl;
        }
    }
}

int launch_ex_init(bfsc_ctx *ctx, uint32_t V, uint64_t n_arcs, uint32_t nseg, void *wsp, hipStream_t s) {
    ExWs ws = ex_ws_layout(wsp, V, n_arcs, nseg, nullptr);
    const uint32_t grid = (uint32_t)ctx->n_cu * 8;
    hipLaunchKernelGGL(k_ex_zero, dim3(grid), dim3(256), 0, s, ws.cb.next_bm, (uint64_t)ws.cb.words);
    hipLaunchKernelGGL(k_ex_zero, dim3(grid), dim3(256), 0, s, ws.merged, (uint64_t)ws.words);
    hipLaunchKernelGGL(k_ex_zero, dim3(1), dim3(64), 0, s, ws.cb.qcount, (uint64_t)4);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_candidates(bfsc_ctx *ctx, const bfsc_csr *g, const uint32_t *frontier, const uint32_t *frontier_len,
                      const uint32_t *bounds, uint32_t nseg, uint32_t *ids, uint64_t cap, uint64_t *seg_off,
                      uint32_t *seg_lo, uint32_t *seg_hi, void *wsp, hipStream_t s) {
    const uint32_t V = g->n_vertices;
    ExWs ws = ex_ws_layout(wsp, V, g->n_arcs, nseg, nullptr);
    const uint32_t grid = (uint32_t)ctx->n_cu * 8;
    const uint64_t RR = (uint64_t)nseg * nseg;
    hipLaunchKernelGGL(k_ex_check, dim3(1), dim3(1), 0, s, bounds, nseg, V, ctx->err);
    const CandVisit vis{bounds, nseg, ws.words, ws.cb.next_bm};
    hipLaunchKernelGGL(k_bfs_expand<CandVisit>, dim3(grid), dim3(kExpandThreads), 0, s, g->row_ptr, g->col_idx,
                       frontier, frontier_len, vis, ws.cb);
    hipLaunchKernelGGL(k_bfs_huge<CandVisit>, dim3((uint32_t)ctx->n_cu * 4), dim3(256), 0, s, g->col_idx, vis, ws.cb);
    hipLaunchKernelGGL(k_bfs_count, dim3(ws.cb.nchunks), dim3(256), 0, s, ws.cb);
    hipLaunchKernelGGL(k_bfs_scan, dim3(1), dim3(1024), 0, s, ws.cb, ws.count);
    const uint64_t sw = (RR + 1 + 3) / 4;
    hipLaunchKernelGGL(k_ex_segoff, dim3((uint32_t)(sw < (uint64_t)grid * 4 ? sw : (uint64_t)grid * 4)), dim3(256), 0,
                       s, ws.cb, bounds, nseg, ws.words, cap, seg_off);
    hipLaunchKernelGGL(k_ex_emit, dim3(ws.cb.nchunks), dim3(256), 0, s, ws.cb, ws.words, ids, cap);
    hipLaunchKernelGGL(k_ex_clamp, dim3(1), dim3(1), 0, s, ws.count, cap, ctx->err);
    hipLaunchKernelGGL(k_ex_finish, dim3(grid), dim3(256), 0, s, bounds, nseg, seg_lo, seg_hi);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_merge_filter(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *ids,
                        const uint64_t *n_dev, int32_t *level, uint32_t *next, uint32_t *next_len, void *bfs_wsp,
                        void *wsp, hipStream_t s) {
    const uint32_t V = g->n_vertices;
    BfsWs bws = bfs_ws_layout(bfs_wsp, V, g->n_arcs, nullptr);
    ExWs ws = ex_ws_layout(wsp, V, g->n_arcs, 1, nullptr);  // the merge bitmap's place does not depend on R
    const uint32_t grid = (uint32_t)ctx->n_cu * 8;
    hipLaunchKernelGGL(k_ex_merge, dim3(grid), dim3(256), 0, s, ids, n_dev, V, ws.merged);
    hipLaunchKernelGGL(k_ex_filter, dim3(grid), dim3(256), 0, s, ws.merged, bws, level, cur_level + 1);
    hipLaunchKernelGGL(k_bfs_count, dim3(bws.nchunks), dim3(256), 0, s, bws);
    hipLaunchKernelGGL(k_bfs_scan, dim3(1), dim3(1024), 0, s, bws, next_len);
    hipLaunchKernelGGL(k_bfs_emit, dim3(bws.nchunks), dim3(256), 0, s, bws, next);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

}  // namespace bfsc
