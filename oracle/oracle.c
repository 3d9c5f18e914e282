/*
 * Oracle for single-source BFS and integral-weight SSSP (weighted BFS).
 *
 * TEST INFRASTRUCTURE ONLY.  This plain, sequential, single-threaded CPU code
 * defines the expected results.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call it; the GPU library never does, and
 * the two share no code.
 *
 * What is computed (problem statements of the Benchmark section, "Shortest
 * Path Problems"):
 *   BFS:  D[v] = hop distance from src, infinity when unreachable.
 *   wBFS: D[v] = shortest-path distance from src with integral weights,
 *         infinity when unreachable.
 * Both are reached exactly by the paper's frontier algorithms (BFS and wBFS
 * algorithm boxes), so the oracle computes the plain definitions with
 * textbook methods: a FIFO-queue BFS, and Dial's bucketed Dijkstra (buckets
 * indexed by tentative distance, stale entries skipped when popped).
 *
 * The paper's BFS leaves the discovering parent to whichever test-and-set
 * wins, so it is not unique.  Here the parent is fixed by definition:
 *   BFS:  parent[v] = min { u in N(v) : D[u] + 1      == D[v] }
 *   wBFS: parent[v] = min { u in N(v) : D[u] + w(u,v) == D[v] }
 * with parent[src] = src and parent = -1 for unreachable vertices.
 *
 * Encodings of infinity: BFS int32 INT32_MAX, wBFS uint32 0xFFFFFFFF.
 *
 * Two more problems of the same section are computed from their definitions
 * (distances / widths only; the statements ask for no parents):
 *   General-weight SSSP: D[v] = shortest-path distance from src over int32
 *         weights of any sign (int64), INT64_MAX when unreachable, INT64_MIN
 *         (minus infinity) when a negative cycle reachable from src reaches
 *         v.  Textbook Bellman-Ford: passes over every edge until none
 *         lowers a distance (at most n - 1), one more pass to find the
 *         vertices a negative cycle still lowers, then every vertex reachable
 *         from those gets minus infinity.
 *   Single-source betweenness: S[v] = sum over targets t != src, v of
 *         sigma_st(v) / sigma_st (sigma_st = number of shortest src-t paths,
 *         sigma_st(v) = those through v), double; S[src] = 0 and S = 0 for
 *         unreachable vertices.  Textbook Brandes: a FIFO BFS counting
 *         shortest paths, then dependencies accumulated in reverse BFS order,
 *         delta(v) = sum over children w of sigma(v) / sigma(w) * (1 +
 *         delta(w)).
 *   Widest path: W[v] = maximum over src-v paths of the smallest weight on
 *         the path (weights >= 1, uint32).  The source's width is that of the
 *         empty path, 0xFFFFFFFF; an unreachable vertex gets 0, the maximum
 *         over no paths (the statement's "infinity when unreachable" would
 *         collide with the source's own width).  Textbook method: Dijkstra's
 *         algorithm on a max-heap of widths.
 *   Low-diameter decomposition (Miller-Peng-Xu, the paper's LDD algorithm
 *         box): every vertex draws a shift g(v); start(v) = max g - g(v);
 *         rounds r = 0, 1, ...: unvisited vertices with start(v) = r become
 *         centres of their own clusters and join the frontier, then the
 *         frontier claims its unvisited neighbours, which take the cluster of
 *         their smallest-ID frontier neighbour and form the next frontier.
 *         The shifts are the floored Exp(beta) shifts of the box, drawn as
 *         geometric variables: g(v) = number of leading SplitMix64 draws
 *         below q * 2^64, q = exp(-beta), counter seed ^ (level << 40 |
 *         v << 6 | i), at most 63.
 *   Connectivity: label[v] = smallest vertex id of v's component (a FIFO
 *         BFS from each unlabelled vertex in increasing id order).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define BFS_INF INT32_MAX
#define WBFS_INF 0xFFFFFFFFu

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_bfs(int64_t n, const int64_t* offsets, const int32_t* nbrs,
               int32_t src, int32_t* dist, int32_t* parent) {
    if (n <= 0 || src < 0 || src >= n) return -1;
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) return -2;
    for (int64_t v = 0; v < n; ++v) {
        dist[v] = BFS_INF;
        parent[v] = -1;
    }
    /* FIFO breadth-first search: D[src] = 0, each vertex enqueued once, at
     * the first time it is seen, with the distance of its discoverer + 1. */
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            int32_t v = nbrs[e];
            if (dist[v] == BFS_INF) {
                dist[v] = dist[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    /* Parent rule: smallest neighbour one hop closer to the source. */
    for (int64_t v = 0; v < n; ++v) {
        if (dist[v] == BFS_INF || v == src) continue;
        int32_t best = -1;
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
            int32_t u = nbrs[e];
            if (dist[u] != BFS_INF && dist[u] + 1 == dist[v] && (best < 0 || u < best))
                best = u;
        }
        parent[v] = best;
    }
    parent[src] = src;
    return 0;
}

/* Growable int32 list used as one Dial bucket. */
typedef struct {
    int32_t* a;
    int64_t len, cap;
} ilist;

static int ilist_push(ilist* l, int32_t x) {
    if (l->len == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 16;
        int32_t* na = (int32_t*)realloc(l->a, sizeof(int32_t) * (size_t)nc);
        if (!na) return -1;
        l->a = na;
        l->cap = nc;
    }
    l->a[l->len++] = x;
    return 0;
}

/* Returns 0 on success, -1 on bad arguments (weights < 1), -2 on allocation
 * failure.  Distances are accumulated in 64 bits and must stay below
 * 0xFFFFFFFF (guaranteed when max_w * (n - 1) < 2^32 - 1). */
int oracle_wbfs(int64_t n, const int64_t* offsets, const int32_t* nbrs,
                const int32_t* w, int32_t src, uint32_t* dist, int32_t* parent) {
    if (n <= 0 || src < 0 || src >= n) return -1;
    int64_t m = offsets[n];
    int64_t maxw = 1;
    for (int64_t e = 0; e < m; ++e) {
        if (w[e] < 1) return -1;
        if (w[e] > maxw) maxw = w[e];
    }
    /* Dial's algorithm: tentative distances lie in [cur, cur + maxw], so a
     * circular array of maxw + 1 buckets holds every pending entry. */
    const int64_t C = maxw + 1;
    ilist* bucket = (ilist*)calloc((size_t)C, sizeof(ilist));
    uint64_t* d = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    unsigned char* settled = (unsigned char*)calloc((size_t)n, 1);
    if (!bucket || !d || !settled) {
        free(bucket); free(d); free(settled);
        return -2;
    }
    const uint64_t INF64 = UINT64_MAX;
    for (int64_t v = 0; v < n; ++v) d[v] = INF64;
    d[src] = 0;
    int64_t pending = 0;
    int rc = 0;
    if (ilist_push(&bucket[0], src)) rc = -2;
    pending = 1;
    uint64_t cur = 0;
    while (pending > 0 && rc == 0) {
        ilist* b = &bucket[cur % (uint64_t)C];
        /* Entries appended while scanning this bucket carry larger
         * distances (weights >= 1), so they never land in this bucket. */
        for (int64_t i = 0; i < b->len; ++i) {
            int32_t u = b->a[i];
            --pending;
            if (settled[u] || d[u] != cur) continue; /* stale entry */
            settled[u] = 1;
            for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
                int32_t v = nbrs[e];
                uint64_t nd = cur + (uint64_t)w[e];
                if (!settled[v] && nd < d[v]) {
                    d[v] = nd;
                    if (ilist_push(&bucket[nd % (uint64_t)C], v)) { rc = -2; break; }
                    ++pending;
                }
            }
        }
        b->len = 0;
        ++cur;
    }
    for (int64_t i = 0; i < C; ++i) free(bucket[i].a);
    free(bucket);
    free(settled);
    if (rc) { free(d); return rc; }
    for (int64_t v = 0; v < n; ++v) {
        dist[v] = d[v] == INF64 ? WBFS_INF : (uint32_t)d[v];
        parent[v] = -1;
    }
    /* Parent rule: smallest neighbour u with D[u] + w(u,v) == D[v]; the
     * weights are symmetric, so w(u,v) is read from v's own list. */
    for (int64_t v = 0; v < n; ++v) {
        if (d[v] == INF64 || v == src) continue;
        int32_t best = -1;
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
            int32_t u = nbrs[e];
            if (d[u] != INF64 && d[u] + (uint64_t)w[e] == d[v] && (best < 0 || u < best))
                best = u;
        }
        parent[v] = best;
    }
    parent[src] = src;
    free(d);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* General-weight SSSP (Bellman-Ford).                                      */
/* ------------------------------------------------------------------------ */

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 * The CSR may be directed here (edge e goes from its list's owner to
 * nbrs[e]); distances of simple paths fit in int64 for any int32 weights. */
int oracle_bellman_ford(int64_t n, const int64_t* offsets, const int32_t* nbrs,
                        const int32_t* w, int32_t src, int64_t* dist) {
    if (n <= 0 || src < 0 || src >= n) return -1;
    /* With a negative cycle, in-place passes can follow walks of up to n
     * edges per pass, n^2 * 2^31 in all: negative weights are accepted on
     * graphs small enough for that to fit in int64. */
    if (n > 65536) {
        for (int64_t e = 0; e < offsets[n]; ++e)
            if (w[e] < 0) return -1;
    }
    const int64_t INF = INT64_MAX;
    for (int64_t v = 0; v < n; ++v) dist[v] = INF;
    dist[src] = 0;
    /* passes over all edges until a pass changes nothing; a graph without a
     * reachable negative cycle settles within n - 1 passes */
    int changed = 1;
    for (int64_t pass = 0; pass < n - 1 && changed; ++pass) {
        changed = 0;
        for (int64_t u = 0; u < n; ++u) {
            if (dist[u] == INF) continue;
            for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
                const int64_t nd = dist[u] + (int64_t)w[e];
                if (nd < dist[nbrs[e]]) {
                    dist[nbrs[e]] = nd;
                    changed = 1;
                }
            }
        }
    }
    if (!changed) return 0;
    /* one more pass: every vertex that can still be lowered lies on or
     * behind a negative cycle reachable from src */
    unsigned char* neg = (unsigned char*)calloc((size_t)n, 1);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!neg || !queue) {
        free(neg);
        free(queue);
        return -2;
    }
    int64_t tail = 0;
    for (int64_t u = 0; u < n; ++u) {
        if (dist[u] == INF) continue;
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            const int32_t v = nbrs[e];
            if (dist[u] + (int64_t)w[e] < dist[v] && !neg[v]) {
                neg[v] = 1;
                queue[tail++] = v;
            }
        }
    }
    /* minus infinity spreads to everything reachable from those vertices */
    for (int64_t head = 0; head < tail; ++head) {
        const int32_t u = queue[head];
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            const int32_t v = nbrs[e];
            if (!neg[v]) {
                neg[v] = 1;
                queue[tail++] = v;
            }
        }
    }
    for (int64_t v = 0; v < n; ++v)
        if (neg[v]) dist[v] = INT64_MIN;
    free(neg);
    free(queue);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Widest (bottleneck) path.                                                */
/* ------------------------------------------------------------------------ */

/* Binary max-heap of vertices keyed by their current width, with the
 * position of every vertex so that a width can be raised in place. */
typedef struct {
    int32_t* v;     /* heap slots */
    int64_t* pos;   /* slot of each vertex, -1 when not in the heap */
    const uint32_t* key;
    int64_t len;
} maxheap;

static void mh_swap(maxheap* h, int64_t i, int64_t j) {
    int32_t t = h->v[i];
    h->v[i] = h->v[j];
    h->v[j] = t;
    h->pos[h->v[i]] = i;
    h->pos[h->v[j]] = j;
}

static void mh_up(maxheap* h, int64_t i) {
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->key[h->v[p]] >= h->key[h->v[i]]) break;
        mh_swap(h, i, p);
        i = p;
    }
}

static void mh_down(maxheap* h, int64_t i) {
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, b = i;
        if (l < h->len && h->key[h->v[l]] > h->key[h->v[b]]) b = l;
        if (r < h->len && h->key[h->v[r]] > h->key[h->v[b]]) b = r;
        if (b == i) break;
        mh_swap(h, i, b);
        i = b;
    }
}

/* Returns 0 on success, -1 on bad arguments (weights < 1), -2 on
 * allocation failure. */
int oracle_widest_path(int64_t n, const int64_t* offsets, const int32_t* nbrs,
                       const int32_t* w, int32_t src, uint32_t* width) {
    if (n <= 0 || src < 0 || src >= n) return -1;
    const int64_t m = offsets[n];
    for (int64_t e = 0; e < m; ++e)
        if (w[e] < 1) return -1;
    maxheap h;
    h.v = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    h.pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char* done = (unsigned char*)calloc((size_t)n, 1);
    if (!h.v || !h.pos || !done) {
        free(h.v);
        free(h.pos);
        free(done);
        return -2;
    }
    for (int64_t v = 0; v < n; ++v) {
        width[v] = 0;
        h.pos[v] = -1;
    }
    h.key = width;
    h.len = 0;
    width[src] = 0xFFFFFFFFu;
    h.v[0] = src;
    h.pos[src] = 0;
    h.len = 1;
    /* Dijkstra with the roles of min and + taken by max and min: the widest
     * unsettled vertex cannot be widened any more, since every path through
     * another unsettled vertex is at most that vertex's width. */
    while (h.len > 0) {
        const int32_t u = h.v[0];
        h.len--;
        if (h.len > 0) {
            h.v[0] = h.v[h.len];
            h.pos[h.v[0]] = 0;
            mh_down(&h, 0);
        }
        h.pos[u] = -1;
        done[u] = 1;
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            const int32_t v = nbrs[e];
            if (done[v]) continue;
            const uint32_t c = width[u] < (uint32_t)w[e] ? width[u] : (uint32_t)w[e];
            if (c > width[v]) {
                width[v] = c;
                if (h.pos[v] < 0) {
                    h.v[h.len] = v;
                    h.pos[v] = h.len;
                    h.len++;
                }
                mh_up(&h, h.pos[v]);
            }
        }
    }
    free(h.v);
    free(h.pos);
    free(done);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-source betweenness centrality (Brandes).                          */
/* ------------------------------------------------------------------------ */

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_betweenness(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t src,
                       double* dep) {
    if (n <= 0 || src < 0 || src >= n) return -1;
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* d = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double* sigma = (double*)calloc((size_t)n, sizeof(double));
    if (!order || !d || !sigma) {
        free(order);
        free(d);
        free(sigma);
        return -2;
    }
    for (int64_t v = 0; v < n; ++v) {
        d[v] = -1;
        dep[v] = 0.0;
    }
    /* FIFO BFS; a vertex's path count is complete when it is dequeued,
     * since all its predecessors were dequeued before it */
    int64_t head = 0, tail = 0;
    d[src] = 0;
    sigma[src] = 1.0;
    order[tail++] = src;
    while (head < tail) {
        const int32_t v = order[head++];
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
            const int32_t w = nbrs[e];
            if (d[w] < 0) {
                d[w] = d[v] + 1;
                order[tail++] = w;
            }
            if (d[w] == d[v] + 1) sigma[w] += sigma[v];
        }
    }
    /* reverse BFS order: every child of v is finished before v */
    for (int64_t i = tail - 1; i >= 0; --i) {
        const int32_t w = order[i];
        for (int64_t e = offsets[w]; e < offsets[w + 1]; ++e) {
            const int32_t v = nbrs[e];
            if (d[v] == d[w] - 1) dep[v] += sigma[v] / sigma[w] * (1.0 + dep[w]);
        }
    }
    dep[src] = 0.0;
    free(order);
    free(d);
    free(sigma);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Low-diameter decomposition and connectivity.                             */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output function (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", 2014, with the constants of Vigna's
 * reference code), applied to a counter. */
static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* q * 2^64 with q = exp(-beta): a draw below it is a success. */
uint64_t oracle_geo_threshold(double beta) {
    const double q = exp(-beta);
    if (q >= 1.0) return UINT64_MAX;
    return (uint64_t)ldexp(q, 64);
}

int32_t oracle_geo_shift(uint64_t seed, uint32_t level, uint32_t v, uint64_t thr) {
    int32_t g = 0;
    while (g < 63 &&
           splitmix64(seed ^ (((uint64_t)level << 40) | ((uint64_t)v << 6) | (uint64_t)g)) < thr)
        ++g;
    return g;
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_ldd(int64_t n, const int64_t* offsets, const int32_t* nbrs, double beta,
               uint64_t seed, uint32_t level, int32_t* cluster) {
    if (n <= 0 || !(beta > 0.0)) return -1;
    const uint64_t thr = oracle_geo_threshold(beta);
    int32_t* start = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* par = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* F = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* nxt = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t* bstart = (int64_t*)calloc(65, sizeof(int64_t));
    int32_t* byst = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!start || !par || !F || !nxt || !bstart || !byst) {
        free(start); free(par); free(F); free(nxt); free(bstart); free(byst);
        return -2;
    }
    int32_t gmax = 0;
    for (int64_t v = 0; v < n; ++v) {
        start[v] = oracle_geo_shift(seed, level, (uint32_t)v, thr);
        if (start[v] > gmax) gmax = start[v];
    }
    for (int64_t v = 0; v < n; ++v) {
        start[v] = gmax - start[v];
        cluster[v] = -1;
        par[v] = -1;
        bstart[start[v] + 1]++;
    }
    /* vertices listed by start round */
    for (int i = 1; i <= 64; ++i) bstart[i] += bstart[i - 1];
    {
        int64_t fill[64];
        for (int i = 0; i < 64; ++i) fill[i] = bstart[i];
        for (int64_t v = 0; v < n; ++v) byst[fill[start[v]]++] = (int32_t)v;
    }
    int64_t visited = 0, nf = 0;
    for (int64_t r = 0; visited < n; ++r) {
        /* new centres: still unvisited vertices whose start round is r */
        if (r <= gmax) {
            for (int64_t i = bstart[r]; i < bstart[r + 1]; ++i) {
                const int32_t v = byst[i];
                if (cluster[v] < 0) {
                    cluster[v] = v;
                    F[nf++] = v;
                }
            }
        }
        visited += nf;
        /* the frontier claims its unvisited neighbours; each takes the
         * cluster of its smallest-ID frontier neighbour */
        int64_t nn = 0;
        for (int64_t i = 0; i < nf; ++i) {
            const int32_t u = F[i];
            for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
                const int32_t d = nbrs[e];
                if (cluster[d] >= 0) continue;
                if (par[d] < 0) {
                    par[d] = u;
                    nxt[nn++] = d;
                } else if (u < par[d]) {
                    par[d] = u;
                }
            }
        }
        for (int64_t i = 0; i < nn; ++i) cluster[nxt[i]] = cluster[par[nxt[i]]];
        int32_t* t = F;
        F = nxt;
        nxt = t;
        nf = nn;
    }
    free(start); free(par); free(F); free(nxt); free(bstart); free(byst);
    return 0;
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_components(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t* label) {
    if (n <= 0) return -1;
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) return -2;
    for (int64_t v = 0; v < n; ++v) label[v] = -1;
    for (int64_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        int64_t head = 0, tail = 0;
        label[s] = (int32_t)s;
        queue[tail++] = (int32_t)s;
        while (head < tail) {
            const int32_t u = queue[head++];
            for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
                const int32_t v = nbrs[e];
                if (label[v] < 0) {
                    label[v] = (int32_t)s;
                    queue[tail++] = v;
                }
            }
        }
    }
    free(queue);
    return 0;
}
