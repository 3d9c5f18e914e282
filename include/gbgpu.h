/*
 * gbgpu -- frontier traversal (edgeMap) over a resident CSR graph on one
 * MI355X (gfx950) GPU: breadth-first search and integral-weight SSSP
 * (weighted BFS), single-source, multi-source batched, and served; and on
 * the same rounds general-weight SSSP (Bellman-Ford), widest path,
 * single-source betweenness, low-diameter decomposition, connectivity, and
 * BFS over compressed neighbour lists.
 *
 * Operations follow the problem statements of the paper's Benchmark section,
 * "Shortest Path Problems" (Dhulipala, Blelloch, Shun, "Theoretically
 * Efficient Parallel Graph Algorithms Can Be Fast and Scalable"):
 *   BFS:  input G = (V, E) unweighted and src; output D[v] = hop distance
 *         from src, infinity if unreachable.
 *   wBFS: input G = (V, E, w) with integral weights and src; output D[v] =
 *         shortest-path distance, infinity if unreachable.
 * The paper's BFS lets a test-and-set pick the discovering parent, so its
 * parent is not unique; this library fixes it deterministically:
 *   BFS:  parent[v] = min { u in N(v) : D[u] + 1      == D[v] }
 *   wBFS: parent[v] = min { u in N(v) : D[u] + w(u,v) == D[v] }
 *   parent[src] = src; parent[v] = -1 when v is unreachable.
 * Output encodings: BFS dist int32 with INT32_MAX for infinity; wBFS dist
 * uint32 with 0xFFFFFFFF for infinity; parent int32.
 *
 * Conventions for every call:
 *   - Return value is a gbgpu_status; 0 (GBGPU_OK) means success.  On any
 *     other value gbgpu_last_error() returns a message for the calling thread.
 *   - Argument errors are detected before any device work; outputs are then
 *     left untouched.
 *   - "dev" pointers are device pointers on the current HIP device (for
 *     instance torch tensor data); "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is ordered on that stream; the traversal calls return only when
 *     their outputs are complete in device memory.  gbgpu_bfs may leave a
 *     few empty traversal launches queued on the stream behind that point;
 *     they touch only the library's workspace, and later work on the stream
 *     (or a later call on the same graph, on any stream) is ordered after
 *     them.
 *   - Graph handles are immutable after load and may be shared between
 *     threads; calls on one handle are serialised internally because they
 *     share its workspace.
 */
#ifndef GBGPU_H
#define GBGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GBGPU_OK = 0,
    GBGPU_E_INVALID = 1,     /* bad argument or malformed graph            */
    GBGPU_E_UNSUPPORTED = 2, /* valid input outside the library's limits   */
    GBGPU_E_NOMEM = 3,       /* device or host allocation failed / budget  */
    GBGPU_E_HIP = 4,         /* HIP runtime error                          */
    GBGPU_E_OVERFLOW = 5,    /* distances could exceed 0xFFFFFFFF - 1      */
    GBGPU_E_AGAIN = 6,       /* not ready yet / queue full; retry later    */
    GBGPU_E_NOTFOUND = 7     /* unknown ticket or id                       */
} gbgpu_status;

/* Message describing the last non-OK status returned on this thread. */
const char* gbgpu_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int gbgpu_version(void);

typedef struct gbgpu_graph_s* gbgpu_graph;

/* Load flags. */
enum {
    GBGPU_SYMMETRIC = 1u, /* caller asserts every edge is stored both ways   */
    GBGPU_VALIDATE = 2u,  /* check the CSR on the device (see gbgpu_load_csr) */
    GBGPU_SIGNED_WEIGHTS = 4u /* weights may be any int32 (zero and negative
                                 ones allowed; only gbgpu_bellman_ford then
                                 accepts the graph's weights)               */
};

/* Tuning knobs; a zero field selects the built-in (or autotuned) default.
 * None of them changes results, only speed. */
typedef struct {
    int32_t force_direction; /* 0 auto, 1 always push (sparse), 2 always pull
                                (dense), 3 alternate push/pull by round (wBFS:
                                dense on odd buckets)                         */
    int32_t tau;             /* go dense when |U| + sum deg(U) > m / tau (BFS
                                frontier or wBFS bucket)                      */
    int32_t pull_light;      /* pull: neighbours one lane scans before the
                                vertex is handed to a whole wavefront          */
    int32_t wave_chunk;      /* push: max edges per wavefront work item (>=64) */
    int32_t grid;            /* workgroups per traversal launch                */
    int32_t bucket_window;   /* wBFS: ring of buckets (power of two >= 2*maxw+1) */
    int32_t bucket_capacity; /* wBFS: entries per bucket (retried larger on
                                overflow)                                       */
    int32_t rounds_per_sync; /* single-source BFS / wBFS: launches kept queued
                                ahead of the one the device last reported as
                                started (default 3)                            */
    int32_t profile;         /* 1: time each traversal launch with HIP events   */
    int32_t max_pending;     /* server: pending-queue bound (default 65536)     */
    int32_t beta;            /* BFS: after a dense round stay dense while
                                |U| > n / beta (default 24; negative: off)     */
    int32_t persistent;      /* BFS and batched BFS: 1 runs every round in
                                one cooperative launch (rounds separated by
                                grid barriers; batched groups drop out as
                                their frontiers empty; if the launch is
                                refused or a barrier wait gives up, the work
                                reruns one launch per round); 0 (default) and
                                -1: one launch per round                      */
    int32_t reserved[4];     /* must be zero                                   */
} gbgpu_opts;

/* Per-call statistics (optional out-parameter). */
typedef struct {
    int32_t rounds;          /* BFS: depth (largest finite distance + 1);
                                wBFS: buckets processed                       */
    int32_t push_rounds;     /* rounds run sparse (push)                       */
    int32_t pull_rounds;     /* rounds run dense (pull)                        */
    int32_t launches;        /* traversal kernel launches issued               */
    int64_t reached;         /* vertices with finite distance                  */
    int64_t edges_examined;  /* sum of deg over processed frontiers            */
    double kernel_ms;        /* sum of traversal kernel times (profile = 1)    */
    double wall_ms;          /* host wall time of the call                     */
    int32_t retries;         /* wBFS reruns after a bucket overflow            */
    int32_t bucket_peak;     /* wBFS: entries of the fullest bucket (what the
                                bucket capacity must hold); 0 if unknown      */
    int32_t reserved[6];
} gbgpu_stats;

/* Register a CSR graph that already lives in device memory.
 *   n          number of vertices, 0 < n < 2^31
 *   m          number of stored (directed) entries, 0 <= m <= 2^31 - 1 (the
 *              kernels index edges with 32-bit unsigned integers; the largest
 *              graph the tests run is RMAT scale 26, m = 2,103,850,106)
 *   offsets    dev int64[n+1], offsets[0] = 0, offsets[n] = m, non-decreasing
 *   neighbors  dev int32[m], each list sorted strictly ascending (no
 *              duplicates), no self loops, ids in [0, n)
 *   weights    dev int32[m] aligned with neighbors, w(u,v) = w(v,u), all >= 1
 *              unless GBGPU_SIGNED_WEIGHTS is given; NULL for an unweighted
 *              graph (BFS only).  The smallest weight is checked with or
 *              without GBGPU_VALIDATE.
 *   flags      must include GBGPU_SYMMETRIC (the dense pull reads a vertex's
 *              own list as its in-edges); GBGPU_VALIDATE checks every property
 *              above, including symmetry of edges and weights, on the device
 *   stream     stream used for the load-time kernels
 *   out        receives the handle
 * Ownership: the graph arrays are borrowed -- the caller keeps them alive and
 * unchanged until gbgpu_graph_free.  The handle owns a degree array, a
 * zero-degree bitmap and lazily sized traversal workspaces.
 * Errors: E_INVALID for null pointers, bad sizes, a missing SYMMETRIC flag,
 * a weight below 1 without GBGPU_SIGNED_WEIGHTS, or a failed validation;
 * E_UNSUPPORTED for n or m beyond the limits above. */
int gbgpu_load_csr(int64_t n, int64_t m, const int64_t* offsets,
                   const int32_t* neighbors, const int32_t* weights,
                   uint32_t flags, void* stream, gbgpu_graph* out);

/* Release a handle and its workspaces (not the borrowed arrays). */
int gbgpu_graph_free(gbgpu_graph g);

/* Number of vertices / stored entries / maximum weight (0 if unweighted). */
int gbgpu_graph_info(gbgpu_graph g, int64_t* n, int64_t* m, int32_t* max_weight);

/* Single-source BFS (BFS problem statement; frontier rounds of edgeMap as in
 * the paper's BFS algorithm box, with the sparse/dense switch of Ligra's
 * edgeMap and the blocked sparse traversal of the "edgeMapBlocked" section).
 *   src     source vertex in [0, n)
 *   dist    dev int32[n] output, INT32_MAX for unreachable
 *   parent  dev int32[n] output, min-ID parent, -1 for unreachable
 *   o, st   optional (NULL allowed)
 * Errors: E_INVALID for a null handle/output or src out of range. */
int gbgpu_bfs(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
              const gbgpu_opts* o, gbgpu_stats* st, void* stream);

/* k single-source BFS one after another on one stream (same algorithm and
 * results as k calls of gbgpu_bfs): each search starts as soon as the device
 * reports the previous one's empty frontier, with no return to the caller in
 * between.
 *   srcs        host int32[k], each in [0, n) (repeats allowed)
 *   dist/parent dev int32 outputs; search i writes dist + i * row_stride and
 *               parent + i * row_stride (row_stride = 0: every search writes
 *               the same n entries, so they end holding the last search's)
 *   row_stride  0 or >= n
 *   st          optional: rounds, launches, reached, edges summed over the
 *               k searches; wall_ms of the whole call
 * Errors: E_INVALID for k < 1, a bad source or stride, null pointers. */
int gbgpu_bfs_many(gbgpu_graph g, const int32_t* srcs, int32_t k, int32_t* dist,
                   int32_t* parent, int64_t row_stride, const gbgpu_opts* o,
                   gbgpu_stats* st, void* stream);

/* Allocation-free single-source BFS, for callers that cannot allocate
 * device or pinned host memory during the call (code under stream capture,
 * tight serving loops, harnesses that forbid allocation).  Same algorithm,
 * kernels and results as gbgpu_bfs; the traversal workspace, progress words
 * and round log live in a library-owned static device array of 64 MiB per
 * device (held from the library's first use on that device until the
 * process ends), so the graph's workspace is never allocated.
 *   n limit   at most about 4.05 million vertices: the workspace takes
 *             16.5 n bytes (four 4-byte vertex arrays and four bitmaps) plus
 *             about 170 KB of control words and round log
 *   other arguments as gbgpu_bfs; st->kernel_ms is always 0 (no events);
 *             o->persistent is ignored (one launch per round)
 * The host checks for the end of the search by copying four progress words
 * back after every max(8, rounds_per_sync) round launches and synchronising
 * the stream, so the call returns with the stream drained.  Calls for one
 * device share its array: the library serialises them (one at a time per
 * device and process); the array keeps the last call's contents, which the
 * next call re-initialises.  The current device must be the graph's.
 * Errors: as gbgpu_bfs; E_UNSUPPORTED when the graph needs more workspace
 * than the array holds (nothing is launched), E_INVALID when the current
 * device is not the one the graph was loaded on. */
int gbgpu_bfs_noalloc(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                      const gbgpu_opts* o, gbgpu_stats* st, void* stream);

/* Single-source integral-weight SSSP (weighted BFS problem statement; the
 * paper's wBFS algorithm box: buckets by distance, edgeMapData relaxations
 * with priority-write).  The first call on a graph builds a copy of every
 * list ordered by (weight, neighbour), 6 bytes per stored edge, kept by the
 * handle until gbgpu_graph_free (dense steps read it).  Unless o->tau is
 * set, a bucket goes dense above m / 10.
 *   dist    dev uint32[n] output, 0xFFFFFFFF for unreachable
 *   parent  dev int32[n] output, min-ID tight parent, -1 for unreachable
 * Errors: E_INVALID (no weights, a weight below 1, bad src, null output),
 * E_OVERFLOW when max_weight * n >= 0xFFFFFFFE (a tentative distance could
 * overflow), E_UNSUPPORTED when max_weight > 2047, E_NOMEM when the bucket
 * workspace cannot be allocated. */
int gbgpu_wbfs(gbgpu_graph g, int32_t src, uint32_t* dist, int32_t* parent,
               const gbgpu_opts* o, gbgpu_stats* st, void* stream);

/* Single-source general-weight SSSP (General-Weight SSSP problem statement;
 * the paper's frontier-based Bellman-Ford algorithm box: every round relaxes
 * the out-edges of the vertices whose distance dropped in the round before,
 * with a priority-write (atomic minimum), until no distance drops; the
 * sparse/dense switch of edgeMap applies).
 *   src     source vertex in [0, n)
 *   dist    dev int64[n] output: shortest-path distance; INT64_MAX for
 *           unreachable; INT64_MIN (minus infinity) for every vertex a
 *           negative cycle reachable from src reaches.  Weights are int32 of
 *           any sign (load with GBGPU_SIGNED_WEIGHTS for zero or negative
 *           ones).  The graph is symmetric, so a negative edge reachable from
 *           src is a negative cycle (u, v, u): then the whole component of
 *           src is minus infinity, which a reachability pass detects before
 *           any relaxation; otherwise the component's weights are >= 0 and
 *           the rounds end.
 *   o, st   optional (NULL allowed); st->rounds = relaxation rounds
 * Errors: E_INVALID for a null handle/output, no weights or src out of
 * range.  The call returns when dist is complete. */
int gbgpu_bellman_ford(gbgpu_graph g, int32_t src, int64_t* dist, const gbgpu_opts* o,
                       gbgpu_stats* st, void* stream);

/* Single-source widest (bottleneck) path (Widest Path problem statement; the
 * paper runs it as Bellman-Ford over the (max, min) semiring: the same
 * rounds, with min(width(u), w(u,v)) in place of D(u) + w(u,v) and an atomic
 * maximum in place of the minimum).
 *   width   dev uint32[n] output: the largest, over src-v paths, smallest
 *           weight on the path; 0xFFFFFFFF for src (the empty path); 0 for
 *           unreachable vertices (the maximum over no paths -- every real
 *           width is >= 1)
 * Errors: E_INVALID for a null handle/output, no weights, a weight below 1
 * or src out of range.  The call returns when width is complete. */
int gbgpu_widest_path(gbgpu_graph g, int32_t src, uint32_t* width, const gbgpu_opts* o,
                      gbgpu_stats* st, void* stream);

/* Single-source betweenness centrality (Betweenness Centrality problem
 * statement; the paper's algorithm box after Brandes: a forward pass of BFS
 * rounds counting shortest paths with fetch-and-add, then a backward pass
 * over the levels accumulating dependencies).
 *   src     source vertex in [0, n)
 *   dep     dev double[n] output: S[v] = sum over targets t (t != src,
 *           t != v) of sigma_st(v) / sigma_st, where sigma_st counts the
 *           shortest src-t paths and sigma_st(v) those through v; 0 for src
 *           and for unreachable vertices.  Path counts and sums are fp64 and
 *           the additions run in an order the device's atomics decide, so
 *           results agree with a sequential evaluation to rounding.
 *   o, st   optional (NULL allowed); st->rounds = number of BFS levels,
 *           st->reached = vertices reached
 * Weights, when present, are ignored (unweighted shortest paths).
 * Errors: E_INVALID for a null handle/output or src out of range.  The call
 * returns when dep is complete. */
int gbgpu_bc(gbgpu_graph g, int32_t src, double* dep, const gbgpu_opts* o, gbgpu_stats* st,
             void* stream);

/* Compressed adjacency (the paper's "Compression" section: blocked,
 * independently decodable neighbour lists).  Builds a compressed copy of the
 * graph's lists, owned by the handle (replacing an earlier one): each sorted
 * list is cut into blocks of 64 neighbours; a block stores its first
 * neighbour, a bit width w (bit length of last - first) and each
 * neighbour's offset from the first in w bits; lists of more than one block
 * start with a table of block offsets.  Word offsets per vertex are int64.
 *   bytes   optional host output: size of the copy (lists + offsets)
 * Errors: E_INVALID for a null handle; E_NOMEM.  Synchronous. */
int gbgpu_compress(gbgpu_graph g, int64_t* bytes, void* stream);

/* Decodes the compressed copy into neighbors (dev int32[m], the CSR order);
 * equal to the graph's own neighbour array.  E_INVALID without a copy. */
int gbgpu_decompress(gbgpu_graph g, int32_t* neighbors, void* stream);

/* BFS that reads only the compressed lists and the degrees (BFS algorithm
 * box; rounds of push with a min-ID atomic claim or pull taking the first
 * frontier neighbour in list order, chosen on the device from the
 * frontier's vertex and degree totals with tau, forced by force_direction).
 * Outputs and encodings as gbgpu_bfs (identical results).
 * Errors: as gbgpu_bfs; E_INVALID when the graph has no compressed copy. */
int gbgpu_bfs_compressed(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                         const gbgpu_opts* o, gbgpu_stats* st, void* stream);

/* The same rounds and kernels as gbgpu_bfs_compressed over the plain
 * neighbour array: the baseline that isolates the effect of compression
 * (gbgpu_bfs is the faster general BFS).  Same outputs and errors, without
 * the compressed-copy requirement. */
int gbgpu_bfs_simple(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent,
                     const gbgpu_opts* o, gbgpu_stats* st, void* stream);

/* Low-diameter decomposition (the paper's LDD algorithm box after Miller,
 * Peng and Xu, "Connectivity Problems" section).  Vertex v draws a shift
 * g(v); with start(v) = max g - g(v), round r first makes every unvisited
 * vertex with start(v) = r the centre of its own cluster, then the frontier
 * claims its unvisited neighbours.  Deterministic form of the algorithm:
 *   - g(v) = number of leading SplitMix64 outputs (Steele, Lea and Flood
 *     2014) of the counters seed ^ (v << 6 | i), i = 0, 1, ..., that lie
 *     below exp(-beta) * 2^64, at most 63 (the integer part of an
 *     Exp(beta) shift, which is what the rounds use);
 *   - a vertex claimed by several frontier vertices in one round joins the
 *     cluster of the one with the smallest id.
 *   beta    in (0, 1): larger beta, smaller clusters and more cut edges
 *   seed    any 64-bit value
 *   cluster dev int32[n] output: the centre vertex of v's cluster
 *   o, st   optional (NULL allowed); st->rounds = rounds run, st->reached =
 *           number of clusters
 * Weights, when present, are ignored.  The handle keeps a device arena of
 * the largest LDD / connectivity call made on it (for RMAT scale 24 about
 * 1 GB) until gbgpu_graph_free.  Errors: E_INVALID for a null
 * handle/output or beta outside (0, 1); E_NOMEM.  The call returns when
 * cluster is complete. */
int gbgpu_ldd(gbgpu_graph g, double beta, uint64_t seed, int32_t* cluster,
              const gbgpu_opts* o, gbgpu_stats* st, void* stream);

/* Connected components (Connectivity problem statement; the paper's
 * connectivity algorithm box: an LDD, every cluster contracted to one vertex
 * with the edges between clusters kept once and those inside dropped, then
 * the same on the contracted graph until it has no edges, and the labels
 * mapped back).  Recursion level l draws its shifts from the counters
 * seed ^ (l << 40 | v << 6 | i).
 *   label   dev int32[n] output: the smallest vertex id of v's component
 *   o, st   optional (NULL allowed); st->rounds = recursion levels,
 *           st->reached = number of components
 * Labels do not depend on beta or seed (only the running time does).
 * Weights, when present, are ignored.  Errors: E_INVALID for a null
 * handle/output or beta outside (0, 1); E_NOMEM when a level's buffers
 * (about 16 bytes per stored edge) cannot be allocated. */
int gbgpu_connectivity(gbgpu_graph g, double beta, uint64_t seed, int32_t* label,
                       const gbgpu_opts* o, gbgpu_stats* st, void* stream);

/* Batched multi-source BFS on one graph: k independent BFS problems solved
 * together with one 64-bit frontier mask per vertex and group of 64 sources.
 *   srcs    host int32[k], each in [0, n) (repeats allowed)
 *   dist    dev int32[k * n], row i = BFS from srcs[i] (same encoding as
 *           gbgpu_bfs)
 *   parent  dev int32[k * n], row i = min-ID parents for srcs[i]
 * Results are identical to k calls of gbgpu_bfs.
 * Errors: E_INVALID for k < 1, a bad source or null pointers. */
int gbgpu_bfs_multi(gbgpu_graph g, const int32_t* srcs, int32_t k,
                    int32_t* dist, int32_t* parent, const gbgpu_opts* o,
                    gbgpu_stats* st, void* stream);

/* Uneven batch: nq BFS queries over several graphs, answered together: the
 * queries on each graph are packed 64 to a group (one 64-bit frontier mask
 * per vertex and group), and one kernel launch per round advances every
 * group of every graph (up to 64 groups per launch), each group choosing
 * push or pull for itself; a group whose frontier is empty costs nothing.
 * The host checks for the end after 8, 16, 32, ... launches.  With
 * opts->persistent = 1 every round of those groups runs in one cooperative
 * launch instead, a grid barrier between rounds, ending at the first round
 * in which no group has a frontier (st->launches then counts one launch per
 * 64 groups).  Graphs of any depth are batched (on RMAT-24 and the 256^3
 * torus 64 batched sources run 1.5x and 1.8x faster than one at a time).
 *   graphs   host array of nq graph handles (repeats allowed, any sizes)
 *   srcs     host int32[nq]
 *   dists    host array of nq dev int32* outputs (each n_i long)
 *   parents  host array of nq dev int32* outputs (each n_i long)
 * Results are identical to gbgpu_bfs on each query. */
int gbgpu_bfs_batch(const gbgpu_graph* graphs, const int32_t* srcs, int32_t nq,
                    int32_t* const* dists, int32_t* const* parents,
                    const gbgpu_opts* o, gbgpu_stats* st, void* stream);

/* ---------------------------------------------------------------------- */
/* Serving: resident graphs, queries admitted by device-memory footprint,   */
/* continuous batching, per-query latency.                                  */
/* ---------------------------------------------------------------------- */
typedef struct gbgpu_server_s* gbgpu_server;

enum { GBGPU_QUERY_BFS = 0, GBGPU_QUERY_WBFS = 1 };

typedef struct {
    int32_t graph_id; /* id from gbgpu_server_add_graph                    */
    int32_t kind;     /* GBGPU_QUERY_BFS or GBGPU_QUERY_WBFS                */
    int32_t src;      /* source vertex                                      */
    int32_t reserved;
    void* dist;       /* dev int32[n] (BFS) or uint32[n] (wBFS) output      */
    int32_t* parent;  /* dev int32[n] output                                */
} gbgpu_query;

typedef struct {
    int32_t status;      /* GBGPU_OK, or the query's error status          */
    int32_t rounds;      /* rounds / buckets the query took                */
    int64_t t_arrive_ns; /* CLOCK_MONOTONIC time of gbgpu_submit           */
    int64_t t_start_ns;  /* time the query's last run was admitted to the
                            device (shared by the queries of one packed
                            group)                                         */
    int64_t t_done_ns;   /* time its outputs were known complete           */
    int32_t retries;     /* weighted BFS: runs repeated after a bucket
                            overflow (each doubles the bucket capacity)    */
    int32_t batch;       /* queries in the run that answered this one (1,
                            or the size of a bit-packed same-graph group,
                            including queries that joined it)             */
    int32_t join_round;  /* BFS that joined a running packed group: the
                            group's round it joined before (0 otherwise);
                            t_start_ns is then the time it joined          */
    int32_t launches;    /* traversal launches of the run that answered a
                            query run alone (1: every round in one launch);
                            0 for packed groups                            */
} gbgpu_result;

/* Create a server.
 *   arena, arena_bytes  dev memory the server carves per-query workspaces
 *                       from (caller-owned, kept alive until destroy);
 *                       admission never exceeds it
 *   max_inflight        queries resident on the device at once (>= 1)
 *   o                   tuning options for every query (NULL allowed) */
int gbgpu_server_create(void* arena, size_t arena_bytes, int32_t max_inflight,
                        const gbgpu_opts* o, gbgpu_server* out);

/* Make a loaded graph servable; returns its id.  The handle must outlive the
 * server. */
int gbgpu_server_add_graph(gbgpu_server sv, gbgpu_graph g, int32_t* graph_id);

/* Enqueue a query (copied).  E_AGAIN when the pending queue is full,
 * E_INVALID for a bad graph id, kind, source or output pointer, E_NOMEM when
 * the query's footprint alone exceeds the arena. */
int gbgpu_submit(gbgpu_server sv, const gbgpu_query* q, uint64_t* ticket);

/* Result of a ticket: GBGPU_OK with *r filled once done (the ticket is then
 * released), E_AGAIN while pending or running, E_NOTFOUND for an unknown or
 * already-collected ticket. */
int gbgpu_poll(gbgpu_server sv, uint64_t ticket, gbgpu_result* r);

/* Block until every submitted query has finished. */
int gbgpu_server_drain(gbgpu_server sv);

/* Stop the scheduler, wait for running queries and free the server. */
int gbgpu_server_destroy(gbgpu_server sv);

/* Bytes of device workspace one query of this kind needs on this graph (what
 * admission charges against the arena). */
int gbgpu_query_footprint(gbgpu_graph g, int32_t kind, size_t* bytes);

/* ---------------------------------------------------------------------- */
/* Diagnostics                                                              */
/* ---------------------------------------------------------------------- */
/* Per-round log of the last gbgpu_bfs on g, 4 uint32 per round: direction
 * (1 sparse push from the queue, 2 dense pull, 3 sparse push from the
 * bitmap), |U_r|, sum of deg(U_r), whether the sparse queue was available.
 * The rounds run over the vertices of degree >= 2 (and the source); vertices
 * of degree 1 are attached through their one neighbour after the last round,
 * so they appear in no |U_r| (and may make the depth one more than the
 * number of rounds).  out holds max_rounds * 4 words (host). */
int gbgpu_debug_bfs_log(gbgpu_graph g, uint32_t* out, int32_t max_rounds, int32_t* nrounds);

/* Per-launch log of the last gbgpu_wbfs on g, 4 uint32 per step launch:
 * bucket (distance), entries in the bucket (live and stale), sum of their
 * degrees, step kind (0 sparse push; a dense bucket takes two launches:
 * 1 marks the bucket's vertices, 2 pulls).  out holds max_steps * 4 words
 * (host). */
int gbgpu_debug_wbfs_log(gbgpu_graph g, uint32_t* out, int32_t max_steps, int32_t* nsteps);

/* Round-boundary admission (as the server's packed BFS groups use it):
 * runs srcs[0 .. k0) as one bit-packed group with room for 64 sources and,
 * at the first round boundary the host sees (every 4 rounds) at or after
 * round join_round -- or earlier, if the group runs out of work first --
 * adds srcs[k0 .. k0+k1) to it.  Row i of dist / parent (dev int32, stride
 * n) is the BFS from srcs[i] (host int32[k0 + k1]), the same as gbgpu_bfs
 * from it.  k0 >= 1, k0 + k1 <= 64.  Allocates its workspace per call;
 * returns when the rows are complete. */
int gbgpu_debug_bfs_join(gbgpu_graph g, const int32_t* srcs, int32_t k0, int32_t k1,
                         int32_t join_round, int32_t* dist, int32_t* parent, void* stream);

/* Host-only randomized self-test of the server's first-fit arena allocator
 * (no device work); GBGPU_OK when every allocation matched a reference. */
int gbgpu_debug_arena_selftest(uint64_t seed, int32_t steps);

#ifdef __cplusplus
}
#endif
#endif /* GBGPU_H */
