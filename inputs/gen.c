/*
 * Seeded synthetic inputs for the BFS-frontier codec: graphs, BFS roots and
 * destination-segment bounds.  This file holds none of the codec's or the
 * BFS's arithmetic; both the CPU oracle and the GPU path consume what it
 * produces, as plain arrays.
 *
 * Workload shapes follow the paper's benchmark setting (Graph 500 style
 * Kronecker/R-MAT graphs with 2^scale vertices and edgefactor*2^scale edge
 * samples; "Synthetic data" section and the problem-size table of the
 * Graph 500 background section).
 *
 * Random numbers: one counter-based generator, the SplitMix64 finaliser of
 * Steele, Lea and Flood (OOPSLA 2014) applied to (seed, stream, index), so
 * every draw is a pure function of its coordinates and any thread can make
 * any draw.
 *
 * Graph construction: R-MAT quadrant recursion with integer thresholds
 * floor(p * 2^32), most significant bit first, no noise and no vertex-label
 * scrambling; or uniform endpoints with the same number of samples.
 * Self-loops are dropped, every sample u-v gives arcs u->v and v->u, rows are
 * sorted ascending and duplicates removed, giving a symmetric CSR
 * (row_ptr u64[V+1], col_idx u32[arcs]).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define STREAM_RMAT 1ull
#define STREAM_UNIF 2ull
#define STREAM_ROOT 3ull
#define STREAM_ZIPF 4ull
#define GOLDEN 0x9E3779B97F4A7C15ull

uint64_t bfsgen_mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

/* Counter-based draw: mix(mix(seed + G*(stream+1)) + G*(idx+1)). */
uint64_t bfsgen_ctr(uint64_t seed, uint64_t stream, uint64_t idx)
{
    uint64_t key = bfsgen_mix64(seed + GOLDEN * (stream + 1ull));
    return bfsgen_mix64(key + GOLDEN * (idx + 1ull));
}

typedef struct {
    uint32_t n_vertices;
    uint64_t n_arcs;
    uint64_t *row_ptr;
    uint32_t *col_idx;
} bfsgen_graph;

typedef struct {
    int kind; /* 0 = R-MAT, 1 = uniform */
    int scale;
    uint64_t seed;
    uint32_t ta, tab, tabc; /* cumulative quadrant thresholds */
} genparams;

static inline void gen_edge(const genparams *p, uint64_t e, uint32_t *pu, uint32_t *pv)
{
    uint32_t u = 0, v = 0;
    if (p->kind == 0) {
        uint64_t r64 = 0;
        for (int lvl = 0; lvl < p->scale; ++lvl) {
            if ((lvl & 1) == 0)
                r64 = bfsgen_ctr(p->seed, STREAM_RMAT, e * 16ull + (uint64_t)(lvl >> 1));
            uint32_t r = (lvl & 1) ? (uint32_t)(r64 >> 32) : (uint32_t)r64;
            uint32_t bit = 1u << (p->scale - 1 - lvl);
            if (r < p->ta) {
                /* quadrant a: neither bit */
            } else if (r < p->tab) {
                v |= bit;            /* quadrant b */
            } else if (r < p->tabc) {
                u |= bit;            /* quadrant c */
            } else {
                u |= bit;            /* quadrant d */
                v |= bit;
            }
        }
    } else {
        uint32_t sh = 32 - (uint32_t)p->scale;
        uint64_t a = bfsgen_ctr(p->seed, STREAM_UNIF, 2ull * e);
        uint64_t b = bfsgen_ctr(p->seed, STREAM_UNIF, 2ull * e + 1ull);
        u = sh >= 32 ? 0u : (uint32_t)(a >> 32) >> sh;
        v = sh >= 32 ? 0u : (uint32_t)(b >> 32) >> sh;
    }
    *pu = u;
    *pv = v;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

static void sort_u32(uint32_t *a, uint64_t n)
{
    if (n < 2) return;
    if (n <= 32) {
        for (uint64_t i = 1; i < n; ++i) {
            uint32_t x = a[i];
            uint64_t j = i;
            while (j > 0 && a[j - 1] > x) { a[j] = a[j - 1]; --j; }
            a[j] = x;
        }
        return;
    }
    qsort(a, n, sizeof(uint32_t), cmp_u32);
}

static uint32_t thresh(double p)
{
    double t = floor(p * 4294967296.0);
    if (t >= 4294967295.0) return 0xFFFFFFFFu;
    if (t < 0) return 0;
    return (uint32_t)t;
}

/* Builds the graph; returns NULL on allocation failure or bad arguments. */
void *bfsgen_graph_create(int kind, int scale, int edgefactor, uint64_t seed,
                          double a, double b, double c)
{
    if (scale < 1 || scale > 31 || edgefactor < 1 || (kind != 0 && kind != 1)) return NULL;
    genparams p;
    p.kind = kind;
    p.scale = scale;
    p.seed = seed;
    p.ta = thresh(a);
    p.tab = thresh(a + b);
    p.tabc = thresh(a + b + c);

    const uint64_t V = 1ull << scale;
    const uint64_t M = (uint64_t)edgefactor << scale;

    uint64_t *deg = (uint64_t *)calloc(V + 1, sizeof(uint64_t));
    if (!deg) return NULL;

    /* pass 1: degrees with multiplicity */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)M; ++e) {
        uint32_t u, v;
        gen_edge(&p, (uint64_t)e, &u, &v);
        if (u == v) continue;
        #pragma omp atomic
        deg[u]++;
        #pragma omp atomic
        deg[v]++;
    }
    uint64_t *start = (uint64_t *)malloc((V + 1) * sizeof(uint64_t));
    if (!start) { free(deg); return NULL; }
    uint64_t acc = 0;
    for (uint64_t i = 0; i < V; ++i) { start[i] = acc; acc += deg[i]; }
    start[V] = acc;
    const uint64_t raw_arcs = acc;
    uint32_t *tmp = (uint32_t *)malloc((raw_arcs ? raw_arcs : 1) * sizeof(uint32_t));
    if (!tmp) { free(deg); free(start); return NULL; }
    /* cursors reuse deg[] */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)V; ++i) deg[i] = start[i];

    /* pass 2: scatter arcs (order inside a row is fixed by the sort below) */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)M; ++e) {
        uint32_t u, v;
        gen_edge(&p, (uint64_t)e, &u, &v);
        if (u == v) continue;
        uint64_t pu, pv;
        #pragma omp atomic capture
        pu = deg[u]++;
        #pragma omp atomic capture
        pv = deg[v]++;
        tmp[pu] = v;
        tmp[pv] = u;
    }

    /* sort and dedup every row; new degree into deg[] */
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < (int64_t)V; ++i) {
        uint32_t *row = tmp + start[i];
        uint64_t n = start[i + 1] - start[i];
        sort_u32(row, n);
        uint64_t k = 0;
        for (uint64_t j = 0; j < n; ++j)
            if (k == 0 || row[j] != row[k - 1]) row[k++] = row[j];
        deg[i] = k;
    }

    bfsgen_graph *g = (bfsgen_graph *)calloc(1, sizeof(bfsgen_graph));
    uint64_t *row_ptr = (uint64_t *)malloc((V + 1) * sizeof(uint64_t));
    if (!g || !row_ptr) { free(g); free(row_ptr); free(tmp); free(deg); free(start); return NULL; }
    acc = 0;
    for (uint64_t i = 0; i < V; ++i) { row_ptr[i] = acc; acc += deg[i]; }
    row_ptr[V] = acc;
    uint32_t *col = (uint32_t *)malloc((acc ? acc : 1) * sizeof(uint32_t));
    if (!col) { free(g); free(row_ptr); free(tmp); free(deg); free(start); return NULL; }
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < (int64_t)V; ++i)
        memcpy(col + row_ptr[i], tmp + start[i], deg[i] * sizeof(uint32_t));
    free(tmp);
    free(deg);
    free(start);
    g->n_vertices = (uint32_t)V;
    g->n_arcs = acc;
    g->row_ptr = row_ptr;
    g->col_idx = col;
    return g;
}

void bfsgen_graph_info(void *h, uint32_t *n_vertices, uint64_t *n_arcs,
                       uint64_t **row_ptr, uint32_t **col_idx)
{
    bfsgen_graph *g = (bfsgen_graph *)h;
    *n_vertices = g->n_vertices;
    *n_arcs = g->n_arcs;
    *row_ptr = g->row_ptr;
    *col_idx = g->col_idx;
}

void bfsgen_graph_free(void *h)
{
    bfsgen_graph *g = (bfsgen_graph *)h;
    if (!g) return;
    free(g->row_ptr);
    free(g->col_idx);
    free(g);
}

/* Raw R-MAT / uniform edge samples (for statistics tests): writes M pairs. */
void bfsgen_samples(int kind, int scale, uint64_t seed, double a, double b, double c,
                    uint64_t first, uint64_t count, uint32_t *u_out, uint32_t *v_out)
{
    genparams p;
    p.kind = kind;
    p.scale = scale;
    p.seed = seed;
    p.ta = thresh(a);
    p.tab = thresh(a + b);
    p.tabc = thresh(a + b + c);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        gen_edge(&p, first + (uint64_t)i, &u_out[i], &v_out[i]);
}

/* k distinct roots of positive degree, by rejection sampling on the draw
 * stream high32(ctr(seed, ROOT, i)) >> (32 - scale).  Returns the number found. */
int bfsgen_roots(const uint64_t *row_ptr, int scale, uint64_t seed, int k, uint32_t *out)
{
    int found = 0;
    const uint32_t sh = 32u - (uint32_t)scale;
    for (uint64_t i = 0; found < k && i < (1ull << 32); ++i) {
        uint32_t v = (uint32_t)(bfsgen_ctr(seed, STREAM_ROOT, i) >> 32) >> sh;
        if (row_ptr[v + 1] == row_ptr[v]) continue;
        int dup = 0;
        for (int j = 0; j < found; ++j) dup |= (out[j] == v);
        if (dup) continue;
        out[found++] = v;
    }
    return found;
}

/* Equal ranges: b_r = floor(r * V / R). */
void bfsgen_bounds_equal(uint64_t V, uint32_t R, uint32_t *out)
{
    for (uint32_t r = 0; r <= R; ++r)
        out[r] = (uint32_t)(((unsigned __int128)r * V) / R);
}

/* Zipf(s) sizes on {1..kmax} by inverse CDF (fp64 table summed ascending,
 * u = (draw >> 11) * 2^-53), then normalised cumulative bounds tiling [0, V).
 * Also returns the raw draws in k_out (may be NULL). */
int bfsgen_bounds_zipf(uint64_t V, uint32_t R, double s, uint32_t kmax, uint64_t seed,
                       uint32_t *out, uint32_t *k_out)
{
    double *cdf = (double *)malloc((size_t)kmax * sizeof(double));
    if (!cdf) return -1;
    double acc = 0.0;
    for (uint32_t k = 1; k <= kmax; ++k) {
        acc += pow((double)k, -s);
        cdf[k - 1] = acc;
    }
    uint64_t *ks = (uint64_t *)malloc((size_t)R * sizeof(uint64_t));
    if (!ks) { free(cdf); return -1; }
    unsigned __int128 total = 0;
    for (uint32_t r = 0; r < R; ++r) {
        double u = (double)(bfsgen_ctr(seed, STREAM_ZIPF, r) >> 11) * 0x1.0p-53;
        double target = u * acc;
        uint32_t lo = 0, hi = kmax - 1;
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] >= target) hi = mid; else lo = mid + 1;
        }
        ks[r] = (uint64_t)lo + 1u;
        if (k_out) k_out[r] = (uint32_t)ks[r];
        total += ks[r];
    }
    unsigned __int128 run = 0;
    for (uint32_t r = 0; r < R; ++r) {
        out[r] = (uint32_t)(((unsigned __int128)V * run) / total);
        run += ks[r];
    }
    out[R] = (uint32_t)V;
    free(ks);
    free(cdf);
    return 0;
}

/* Zipf draw only (for distribution tests). */
void bfsgen_zipf_draws(double s, uint32_t kmax, uint64_t seed, uint64_t count, uint32_t *out)
{
    double *cdf = (double *)malloc((size_t)kmax * sizeof(double));
    double acc = 0.0;
    for (uint32_t k = 1; k <= kmax; ++k) {
        acc += pow((double)k, -s);
        cdf[k - 1] = acc;
    }
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)count; ++r) {
        double u = (double)(bfsgen_ctr(seed, STREAM_ZIPF, (uint64_t)r) >> 11) * 0x1.0p-53;
        double target = u * acc;
        uint32_t lo = 0, hi = kmax - 1;
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] >= target) hi = mid; else lo = mid + 1;
        }
        out[r] = lo + 1u;
    }
    free(cdf);
}

/* Uniform fp32 values in [-lim, lim) from the counter stream, for weight
 * initialisation: x_i = lim * (2 * ((draw >> 40) * 2^-24) - 1). */
void bfsgen_uniform_f32(uint64_t seed, uint64_t stream, uint64_t count, float lim, float *out)
{
    for (uint64_t i = 0; i < count; ++i) {
        double u = (double)(bfsgen_ctr(seed, stream, i) >> 40) * 0x1.0p-24;
        out[i] = (float)((double)lim * (2.0 * u - 1.0));
    }
}
