/* Drives the input generator (graphgen.c) and every oracle function
 * (oracle.c) on small graphs, for a build under address and
 * undefined-behaviour sanitizers (test_host_sanitized.py).  Also checks two
 * reductions that need no second solver: weighted BFS with unit weights
 * equals BFS, and the component labels agree with BFS reachability.
 * Exits non-zero on a failed check; the sanitizers abort on a memory or
 * undefined-behaviour error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void gg_rmat_edges(int scale, int64_t nedges, double a, double b, double c, uint64_t seed,
                   uint32_t* us, uint32_t* vs, int threads);
void gg_er_edges(int64_t n, int64_t npairs, uint64_t seed, uint32_t* us, uint32_t* vs,
                 int threads);
int64_t gg_csr_count(int64_t n, int64_t ne, const uint32_t* us, const uint32_t* vs,
                     int64_t* deg_raw, int threads);
int64_t gg_csr_fill(int64_t n, int64_t ne, const uint32_t* us, const uint32_t* vs,
                    const int64_t* deg_raw, uint32_t* tmp, int64_t* raw_off, int64_t* deg_out,
                    int threads);
void gg_csr_compact(int64_t n, const uint32_t* tmp, const int64_t* raw_off, const int64_t* deg,
                    int64_t* offsets, int32_t* nbrs, int threads);
int64_t gg_torus_degree(int64_t k);
void gg_torus3d(int64_t k, int64_t* offsets, int32_t* nbrs, int threads);
void gg_weights(int64_t n, const int64_t* offsets, const int32_t* nbrs, int64_t W, uint64_t seed,
                int32_t* w, int threads);
int64_t gg_sources(int64_t n, const int64_t* offsets, int64_t k, uint64_t seed, int32_t* out);

int oracle_bfs(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t src,
               int32_t* dist, int32_t* parent);
int oracle_wbfs(int64_t n, const int64_t* offsets, const int32_t* nbrs, const int32_t* w,
                int32_t src, uint32_t* dist, int32_t* parent);
int oracle_bellman_ford(int64_t n, const int64_t* offsets, const int32_t* nbrs,
                        const int32_t* w, int32_t src, int64_t* dist);
int oracle_widest_path(int64_t n, const int64_t* offsets, const int32_t* nbrs,
                       const int32_t* w, int32_t src, uint32_t* width);
int oracle_betweenness(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t src,
                       double* dep);
int oracle_ldd(int64_t n, const int64_t* offsets, const int32_t* nbrs, double beta,
               uint64_t seed, uint32_t level, int32_t* cluster);
int oracle_components(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t* label);

typedef struct {
    int64_t n, m;
    int64_t* off;
    int32_t* nbr;
    int32_t* w;
} Graph;

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            printf("FAIL line %d: %s\n", __LINE__, #c);                   \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static Graph from_raw(int64_t n, int64_t ne, uint32_t* us, uint32_t* vs) {
    Graph g;
    g.n = n;
    int64_t* deg_raw = malloc(sizeof(int64_t) * (size_t)n);
    int64_t tot = gg_csr_count(n, ne, us, vs, deg_raw, 2);
    uint32_t* tmp = malloc(sizeof(uint32_t) * (size_t)(tot > 0 ? tot : 1));
    int64_t* raw_off = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* deg = malloc(sizeof(int64_t) * (size_t)n);
    g.m = gg_csr_fill(n, ne, us, vs, deg_raw, tmp, raw_off, deg, 2);
    g.off = malloc(sizeof(int64_t) * (size_t)(n + 1));
    g.nbr = malloc(sizeof(int32_t) * (size_t)(g.m > 0 ? g.m : 1));
    gg_csr_compact(n, tmp, raw_off, deg, g.off, g.nbr, 2);
    free(deg_raw);
    free(tmp);
    free(raw_off);
    free(deg);
    g.w = NULL;
    return g;
}

static void add_weights(Graph* g, int W) {
    g->w = malloc(sizeof(int32_t) * (size_t)(g->m > 0 ? g->m : 1));
    gg_weights(g->n, g->off, g->nbr, W, 2, g->w, 2);
}

static void free_graph(Graph* g) {
    free(g->off);
    free(g->nbr);
    free(g->w);
}

static void exercise(const Graph* g, const char* name) {
    const int64_t n = g->n;
    int32_t srcs[4];
    const int64_t k = gg_sources(n, g->off, 4, 3, srcs);
    int32_t* dist = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* par = malloc(sizeof(int32_t) * (size_t)n);
    uint32_t* wd = malloc(sizeof(uint32_t) * (size_t)n);
    int32_t* wp = malloc(sizeof(int32_t) * (size_t)n);
    int64_t* bf = malloc(sizeof(int64_t) * (size_t)n);
    uint32_t* wide = malloc(sizeof(uint32_t) * (size_t)n);
    double* dep = malloc(sizeof(double) * (size_t)n);
    int32_t* cl = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* lab = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* ones = malloc(sizeof(int32_t) * (size_t)(g->m > 0 ? g->m : 1));
    for (int64_t e = 0; e < g->m; ++e) ones[e] = 1;
    CHECK(oracle_components(n, g->off, g->nbr, lab) == 0);
    CHECK(oracle_ldd(n, g->off, g->nbr, 0.2, 1, 0, cl) == 0);
    CHECK(oracle_ldd(n, g->off, g->nbr, 0.5, 7, 1, cl) == 0);
    for (int64_t i = 0; i < k; ++i) {
        const int32_t s = srcs[i];
        CHECK(oracle_bfs(n, g->off, g->nbr, s, dist, par) == 0);
        CHECK(oracle_wbfs(n, g->off, g->nbr, ones, s, wd, wp) == 0);
        for (int64_t v = 0; v < n; ++v) {
            const int reached = dist[v] != INT32_MAX;
            CHECK(reached ? wd[v] == (uint32_t)dist[v] : wd[v] == 0xFFFFFFFFu);
            CHECK(wp[v] == par[v]);
            CHECK(reached == (lab[v] == lab[s]));
        }
        CHECK(oracle_betweenness(n, g->off, g->nbr, s, dep) == 0);
        if (g->w) {
            CHECK(oracle_wbfs(n, g->off, g->nbr, g->w, s, wd, wp) == 0);
            CHECK(oracle_bellman_ford(n, g->off, g->nbr, g->w, s, bf) == 0);
            CHECK(oracle_widest_path(n, g->off, g->nbr, g->w, s, wide) == 0);
            for (int64_t v = 0; v < n; ++v)
                CHECK(wd[v] == 0xFFFFFFFFu ? bf[v] == INT64_MAX : bf[v] == (int64_t)wd[v]);
        }
        if (failures) break;
    }
    /* argument errors are reported, not acted on */
    CHECK(oracle_bfs(n, g->off, g->nbr, -1, dist, par) != 0);
    CHECK(oracle_bfs(n, g->off, g->nbr, (int32_t)n, dist, par) != 0);
    printf("%s: n=%lld m=%lld sources=%lld\n", name, (long long)n, (long long)g->m, (long long)k);
    free(dist); free(par); free(wd); free(wp); free(bf); free(wide); free(dep); free(cl);
    free(lab); free(ones);
}

int main(void) {
    {
        const int scale = 10;
        const int64_t n = 1 << scale, ne = 16 * n;
        uint32_t* us = malloc(sizeof(uint32_t) * (size_t)ne);
        uint32_t* vs = malloc(sizeof(uint32_t) * (size_t)ne);
        gg_rmat_edges(scale, ne, 0.57, 0.19, 0.19, 1, us, vs, 2);
        Graph g = from_raw(n, ne, us, vs);
        add_weights(&g, 10);
        exercise(&g, "rmat10");
        free_graph(&g);
        free(us);
        free(vs);
    }
    {
        const int64_t n = 3000, ne = n * 2;
        uint32_t* us = malloc(sizeof(uint32_t) * (size_t)ne);
        uint32_t* vs = malloc(sizeof(uint32_t) * (size_t)ne);
        gg_er_edges(n, ne, 5, us, vs, 2);
        Graph g = from_raw(n, ne, us, vs);
        add_weights(&g, 11);
        exercise(&g, "er3000");
        free_graph(&g);
        free(us);
        free(vs);
    }
    for (int64_t kk = 2; kk <= 7; kk += 5) {
        Graph g;
        g.n = kk * kk * kk;
        g.m = g.n * gg_torus_degree(kk);
        g.off = malloc(sizeof(int64_t) * (size_t)(g.n + 1));
        g.nbr = malloc(sizeof(int32_t) * (size_t)g.m);
        gg_torus3d(kk, g.off, g.nbr, 2);
        CHECK(g.off[g.n] == g.m);
        g.w = NULL;
        add_weights(&g, 24);
        exercise(&g, kk == 2 ? "torus2" : "torus7");
        free_graph(&g);
    }
    if (failures) {
        printf("%d checks failed\n", failures);
        return 1;
    }
    printf("generator and oracle checks passed\n");
    return 0;
}
