/*
 * Seeded synthetic graph inputs shared by the oracle and the GPU path.
 *
 * This file holds input generation only: random draws, CSR assembly,
 * symmetrisation, de-duplication and edge weights.  None of the traversal
 * arithmetic (distances, parents, frontiers, buckets) lives here.
 *
 * Inputs stand in for the paper's datasets (Experiments, "Graph Data" and the
 * graph-input table): RMAT graphs for the low-diameter skewed social and web
 * graphs, the 3-D torus that the paper itself uses as its high-diameter
 * family, and Erdos-Renyi graphs as a non-skewed contrast.  Weighted inputs
 * draw integral weights uniformly from [1, W) as the Experiments section does
 * with W = log n.
 *
 * Random numbers come from a counter-based generator (SplitMix64 applied to a
 * seed-derived key xor a counter), so the output is bit-identical for any
 * thread count.  Every graph is returned in CSR form: int64 offsets[n+1],
 * int32 neighbours sorted strictly ascending per vertex, no self loops, no
 * duplicate edges, symmetric (each undirected edge stored in both lists).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014). */
static inline uint64_t sm64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

/* Uniform integer in [0, range) from a 64-bit draw (multiply-high). */
static inline uint64_t draw_below(uint64_t x, uint64_t range) {
    return (uint64_t)(((unsigned __int128)x * range) >> 64);
}

static void set_threads(int threads) {
    if (threads > 0) omp_set_num_threads(threads);
}

/* ------------------------------------------------------------------ */
/* Raw RMAT edge list.                                                  */
/* Edge e, level l (0 = most significant bit) draws r = high 32 bits of  */
/* sm64(key ^ (e*64 + l)); quadrant thresholds are the cumulative        */
/* probabilities (a, a+b, a+b+c) scaled to 2^32.  No noise, no vertex    */
/* relabelling.                                                          */
/* ------------------------------------------------------------------ */
void gg_rmat_edges(int scale, int64_t nedges, double a, double b, double c,
                   uint64_t seed, uint32_t* us, uint32_t* vs, int threads) {
    set_threads(threads);
    const uint64_t key = sm64(seed ^ 0x524D4154ULL);
    const uint64_t tA = (uint64_t)(a * 4294967296.0);
    const uint64_t tB = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tC = (uint64_t)((a + b + c) * 4294967296.0);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nedges; ++e) {
        uint32_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            uint64_t r = sm64(key ^ ((uint64_t)e * 64u + (uint64_t)l)) >> 32;
            uint32_t bit = 1u << (scale - 1 - l);
            if (r < tA) {
            } else if (r < tB) {
                v |= bit;
            } else if (r < tC) {
                u |= bit;
            } else {
                u |= bit;
                v |= bit;
            }
        }
        us[e] = u;
        vs[e] = v;
    }
}

/* Raw Erdos-Renyi edge list: pair e draws u and v independently. */
void gg_er_edges(int64_t n, int64_t npairs, uint64_t seed, uint32_t* us,
                 uint32_t* vs, int threads) {
    set_threads(threads);
    const uint64_t key = sm64(seed ^ 0x45524552ULL);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < npairs; ++e) {
        us[e] = (uint32_t)draw_below(sm64(key ^ ((uint64_t)e * 2u)), (uint64_t)n);
        vs[e] = (uint32_t)draw_below(sm64(key ^ ((uint64_t)e * 2u + 1u)), (uint64_t)n);
    }
}

/* ------------------------------------------------------------------ */
/* Symmetric CSR from an undirected edge list.                          */
/* Self loops are dropped, every edge is stored in both directions, and */
/* each adjacency list is sorted and de-duplicated.                     */
/* ------------------------------------------------------------------ */
static int cmp_u32(const void* x, const void* y) {
    uint32_t a = *(const uint32_t*)x, b = *(const uint32_t*)y;
    return (a > b) - (a < b);
}

static void sort_u32(uint32_t* p, int64_t len) {
    if (len < 24) {
        for (int64_t i = 1; i < len; ++i) {
            uint32_t x = p[i];
            int64_t j = i - 1;
            while (j >= 0 && p[j] > x) {
                p[j + 1] = p[j];
                --j;
            }
            p[j + 1] = x;
        }
    } else {
        qsort(p, (size_t)len, sizeof(uint32_t), cmp_u32);
    }
}

/* Pass 1: returns the number of directed entries before de-duplication
 * and fills deg_raw[n] (int64).  The caller allocates tmp[that count]. */
int64_t gg_csr_count(int64_t n, int64_t ne, const uint32_t* us,
                     const uint32_t* vs, int64_t* deg_raw, int threads) {
    set_threads(threads);
    memset(deg_raw, 0, sizeof(int64_t) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        uint32_t u = us[e], v = vs[e];
        if (u == v) continue;
        __atomic_fetch_add(&deg_raw[u], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&deg_raw[v], 1, __ATOMIC_RELAXED);
    }
    int64_t tot = 0;
    for (int64_t i = 0; i < n; ++i) tot += deg_raw[i];
    return tot;
}

/* Pass 2: scatter into tmp (size = pass-1 total) using raw offsets, sort and
 * de-duplicate each list; writes the final degree of each vertex into
 * deg_out[n] and returns the final number of directed entries m. */
int64_t gg_csr_fill(int64_t n, int64_t ne, const uint32_t* us,
                    const uint32_t* vs, const int64_t* deg_raw, uint32_t* tmp,
                    int64_t* raw_off, int64_t* deg_out, int threads) {
    set_threads(threads);
    raw_off[0] = 0;
    for (int64_t i = 0; i < n; ++i) raw_off[i + 1] = raw_off[i] + deg_raw[i];
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    memcpy(cur, raw_off, sizeof(int64_t) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        uint32_t u = us[e], v = vs[e];
        if (u == v) continue;
        int64_t pu = __atomic_fetch_add(&cur[u], 1, __ATOMIC_RELAXED);
        tmp[pu] = v;
        int64_t pv = __atomic_fetch_add(&cur[v], 1, __ATOMIC_RELAXED);
        tmp[pv] = u;
    }
    free(cur);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        uint32_t* p = tmp + raw_off[i];
        int64_t len = raw_off[i + 1] - raw_off[i];
        sort_u32(p, len);
        int64_t k = 0;
        for (int64_t j = 0; j < len; ++j)
            if (k == 0 || p[k - 1] != p[j]) p[k++] = p[j];
        deg_out[i] = k;
    }
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) m += deg_out[i];
    return m;
}

/* Pass 3: compact the de-duplicated lists into the final CSR. */
void gg_csr_compact(int64_t n, const uint32_t* tmp, const int64_t* raw_off,
                    const int64_t* deg, int64_t* offsets, int32_t* nbrs,
                    int threads) {
    set_threads(threads);
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + deg[i];
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i)
        memcpy(nbrs + offsets[i], tmp + raw_off[i], sizeof(uint32_t) * (size_t)deg[i]);
}

/* ------------------------------------------------------------------ */
/* 3-D torus k x k x k: id = x + k*y + k*k*z, neighbours at +-1 (mod k) */
/* in each dimension, lists sorted ascending and de-duplicated (k <= 2  */
/* merges the two directions).  Returns m.                              */
/* ------------------------------------------------------------------ */
int64_t gg_torus_degree(int64_t k) {
    if (k <= 1) return 0;
    return k == 2 ? 3 : 6;
}

void gg_torus3d(int64_t k, int64_t* offsets, int32_t* nbrs, int threads) {
    set_threads(threads);
    const int64_t n = k * k * k;
    const int64_t d = gg_torus_degree(k);
    for (int64_t i = 0; i <= n; ++i) offsets[i] = i * d;
    if (d == 0) return;
#pragma omp parallel for schedule(static)
    for (int64_t id = 0; id < n; ++id) {
        int64_t x = id % k, y = (id / k) % k, z = id / (k * k);
        uint32_t c[6];
        c[0] = (uint32_t)(((x + 1) % k) + k * y + k * k * z);
        c[1] = (uint32_t)(((x + k - 1) % k) + k * y + k * k * z);
        c[2] = (uint32_t)(x + k * ((y + 1) % k) + k * k * z);
        c[3] = (uint32_t)(x + k * ((y + k - 1) % k) + k * k * z);
        c[4] = (uint32_t)(x + k * y + k * k * ((z + 1) % k));
        c[5] = (uint32_t)(x + k * y + k * k * ((z + k - 1) % k));
        sort_u32(c, 6);
        int64_t w = 0;
        for (int j = 0; j < 6; ++j)
            if (w == 0 || c[w - 1] != c[j]) c[w++] = c[j];
        for (int64_t j = 0; j < w; ++j) nbrs[id * d + j] = (int32_t)c[j];
    }
}

/* ------------------------------------------------------------------ */
/* Symmetric integral weights in [1, W): w(u,v) depends only on the     */
/* unordered pair, so the two stored copies of an edge agree.           */
/* ------------------------------------------------------------------ */
void gg_weights(int64_t n, const int64_t* offsets, const int32_t* nbrs,
                int64_t W, uint64_t seed, int32_t* w, int threads) {
    set_threads(threads);
    const uint64_t key = sm64(seed ^ 0x57454947ULL);
    const uint64_t range = (uint64_t)(W - 1);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; ++u) {
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            uint64_t v = (uint64_t)(uint32_t)nbrs[e];
            uint64_t lo = (uint64_t)u < v ? (uint64_t)u : v;
            uint64_t hi = (uint64_t)u < v ? v : (uint64_t)u;
            w[e] = (int32_t)(1 + draw_below(sm64(key ^ ((lo << 32) | hi)), range));
        }
    }
}

/* ------------------------------------------------------------------ */
/* Seeded sources: draw i picks sm64(key ^ i) scaled to [0,n); vertices */
/* of degree 0 and repeats are rejected.  Returns how many were found   */
/* (fewer than k only if the graph has fewer non-isolated vertices).    */
/* ------------------------------------------------------------------ */
int64_t gg_sources(int64_t n, const int64_t* offsets, int64_t k, uint64_t seed,
                   int32_t* out) {
    const uint64_t key = sm64(seed ^ 0x53524353ULL);
    int64_t got = 0;
    uint64_t limit = (uint64_t)(64 * n + 1024);
    for (uint64_t i = 0; got < k && i < limit; ++i) {
        int64_t v = (int64_t)draw_below(sm64(key ^ i), (uint64_t)n);
        if (offsets[v + 1] == offsets[v]) continue;
        int dup = 0;
        for (int64_t j = 0; j < got; ++j)
            if (out[j] == (int32_t)v) { dup = 1; break; }
        if (dup) continue;
        out[got++] = (int32_t)v;
    }
    return got;
}
