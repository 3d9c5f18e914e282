// Low-diameter decomposition (Miller-Peng-Xu) and connectivity.
//
// Method (paper: LDD and Connectivity algorithm boxes, "Connectivity
// Problems" section):
//   LDD: every vertex draws a shift g(v); start(v) = max g - g(v).  Round
//   r first makes every still unvisited vertex with start(v) = r the centre
//   of its own cluster and adds it to the frontier, then lets the frontier
//   claim its unvisited neighbours with edgeMap; the claimed vertices form
//   the next frontier.  The box's compare-and-swap leaves ties to a race;
//   here a vertex claimed by several frontier vertices takes the cluster of
//   the one with the smallest id (a 64-bit atomic minimum of (claimer id,
//   claimer's cluster)), so the clustering is deterministic.
//   Connectivity: LDD, contract every cluster to one vertex (inter-cluster
//   edges kept once, intra-cluster ones dropped), recurse on the contracted
//   graph until it has no edges, and map the labels back.  Labels are then
//   made canonical: the smallest vertex id of each component.
// Shifts: the box's Exp(beta) shifts matter only through their integer
// parts, which are geometric with success probability q = exp(-beta); g(v)
// is the number of leading SplitMix64 draws below q * 2^64 (counter
// seed ^ (level << 40 | v << 6 | i), at most 63), so any implementation of
// the published generator reproduces the clusters exactly.  Each recursion
// level draws with its own level number.

#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>  // unique
#include <rocprim/iterator/counting_iterator.hpp>

#include "common.h"
#include "emit.h"

namespace gb {

constexpr unsigned long long kUnclaimed = ~0ull;

// SplitMix64 output function (Steele, Lea and Flood 2014; the constants of
// Vigna's reference code) applied to a counter.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static uint64_t geo_threshold(double beta) {
    const double q = std::exp(-beta);
    if (q >= 1.0) return ~0ull;
    return (uint64_t)std::ldexp(q, 64);
}

// Device arena of the LDD and connectivity calls, cached on the graph
// handle: a stack (each recursion level releases what it took), so one
// allocation serves every level; what does not fit comes from hipMalloc for
// the rest of the call, and the next call starts with an arena as large as
// this call's peak.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, top = 0, peak = 0;
    std::vector<void*> extra;
};

void free_arena(Arena* a) {
    if (!a) return;
    if (a->base) (void)hipFree(a->base);
    for (void* p : a->extra) (void)hipFree(p);
    delete a;
}

static size_t b256(size_t x) { return (x + 255) & ~(size_t)255; }

// Readies the graph's arena for a call expected to need `need` bytes.
static int arena_begin(gbgpu_graph g, size_t need, Arena** out) {
    if (!g->cc) g->cc = new Arena();
    Arena* a = g->cc;
    need = std::max(need, a->peak);
    if (a->cap < need) {
        if (a->base) (void)hipFree(a->base);
        a->base = nullptr;
        a->cap = 0;
        if (hipMalloc(&a->base, need) != hipSuccess) {
            a->base = nullptr;
            return set_error(GBGPU_E_NOMEM, "LDD/connectivity arena of %zu bytes", need);
        }
        a->cap = need;
    }
    a->top = 0;
    *out = a;
    return GBGPU_OK;
}

// Ends a call: the overflow allocations go (the stream has been synchronised).
static void arena_end(Arena* a) {
    for (void* p : a->extra) (void)hipFree(p);
    a->extra.clear();
    a->top = 0;
}

template <typename T>
static int arena_alloc(Arena& a, size_t count, T** p) {
    const size_t bytes = b256(std::max<size_t>(count, 1) * sizeof(T));
    a.peak = std::max(a.peak, a.top + bytes);
    if (a.top + bytes <= a.cap) {
        *p = (T*)(a.base + a.top);
        a.top += bytes;
        return GBGPU_OK;
    }
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess)
        return set_error(GBGPU_E_NOMEM, "LDD/connectivity buffer of %zu bytes", bytes);
    a.extra.push_back(q);
    *p = (T*)q;
    return GBGPU_OK;
}

// A CSR as the rounds read it (the input graph or a contracted one).
struct GView {
    int64_t n, m;
    const int64_t* off;
    const int32_t* nbr;
    const uint32_t* deg;
};

struct LddWs {
    unsigned long long* key;  // (claimer id << 32 | cluster), kUnclaimed
    uint32_t* vis;            // visited bitmap (frontiers of earlier rounds)
    uint32_t* F[2];           // frontier bitmaps (current, next)
    uint32_t* start;          // start round of every vertex
    uint32_t* byst;           // vertices ordered by start round
    uint32_t* keys_sorted;    // sort scratch
    uint32_t* Q[2];
    uint32_t* P[2];
    unsigned long long* ctl;  // qcnt[2], qover[2], gmax, bucket bounds at +8, totals at +128
    void* tmp;
    size_t tmp_bytes;
};

static size_t ldd_ws_bytes(int64_t n) {
    const int64_t nwords = ((n + 63) / 64) * 2;
    return b256((size_t)n * 8) + 3 * b256((size_t)nwords * 4) + 7 * b256((size_t)(n + 64) * 4) +
           b256((128 + kSpread * kSpreadStride) * 8) + b256((size_t)n * 8) + (1u << 20);
}

static int new_ldd_ws(Arena& A, int64_t n, LddWs* w) {
    const int64_t nwords = ((n + 63) / 64) * 2;
    GB_TRY(arena_alloc(A, (size_t)n, &w->key));
    GB_TRY(arena_alloc(A, (size_t)nwords, &w->vis));
    for (int i = 0; i < 2; ++i) GB_TRY(arena_alloc(A, (size_t)nwords, &w->F[i]));
    GB_TRY(arena_alloc(A, (size_t)n + 64, &w->start));
    GB_TRY(arena_alloc(A, (size_t)n + 64, &w->byst));
    GB_TRY(arena_alloc(A, (size_t)n + 64, &w->keys_sorted));
    for (int i = 0; i < 2; ++i) GB_TRY(arena_alloc(A, (size_t)n + 64, &w->Q[i]));
    for (int i = 0; i < 2; ++i) GB_TRY(arena_alloc(A, (size_t)n + 64, &w->P[i]));
    GB_TRY(arena_alloc(A, (size_t)(128 + kSpread * kSpreadStride), &w->ctl));
    size_t ts = 0;
    GB_HIP(rocprim::radix_sort_pairs(nullptr, ts, w->start, w->keys_sorted,
                                     rocprim::counting_iterator<uint32_t>(0u), w->byst,
                                     (unsigned int)n, 0u, 6u));
    w->tmp_bytes = std::max<size_t>(ts, 256);
    char* t = nullptr;
    GB_TRY(arena_alloc(A, w->tmp_bytes, &t));
    w->tmp = t;
    return GBGPU_OK;
}

// g(v) into start[], max g into ctl[4]; keys and the visited and frontier
// bitmaps reset.
__global__ __launch_bounds__(kBlock) void ldd_shift_kernel(int64_t n, int64_t nwords, uint64_t seed,
                                                           uint32_t level, uint64_t thr,
                                                           uint32_t* start,
                                                           unsigned long long* key, uint32_t* vis,
                                                           uint32_t* F0, uint32_t* F1,
                                                           unsigned long long* ctl) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t gm = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        uint32_t g = 0;
        while (g < 63u &&
               splitmix64(seed ^ (((uint64_t)level << 40) | ((uint64_t)v << 6) | (uint64_t)g)) < thr)
            ++g;
        start[v] = g;
        gm = max(gm, g);
        key[v] = kUnclaimed;
    }
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        vis[w] = 0u;
        F0[w] = 0u;
        F1[w] = 0u;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) gm = max(gm, (uint32_t)__shfl_xor(gm, d, 64));
    if (lane_id() == 0) atomicMax(&ctl[4], (unsigned long long)gm);
}

__global__ __launch_bounds__(kBlock) void ldd_start_kernel(int64_t n, uint32_t* start,
                                                           const unsigned long long* ctl) {
    const uint32_t gm = (uint32_t)ctl[4];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        start[v] = gm - start[v];
}

// First position of every start round in the sorted order (ctl[8 + s]) and
// the end (ctl[8 + 64]).
__global__ __launch_bounds__(kBlock) void ldd_bucket_kernel(const uint32_t* skey, int64_t n,
                                                            unsigned long long* ctl) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t k = skey[i];
        const uint32_t kp = i == 0 ? 0u : skey[i - 1] + 1u;
        for (uint32_t s = kp; s <= k; ++s) ctl[8 + s] = (unsigned long long)i;
        if (i == n - 1)
            for (uint32_t s = k + 1; s <= 64u; ++s) ctl[8 + s] = (unsigned long long)n;
    }
}

struct LddArgs {
    const int64_t* off;
    const int32_t* nbr;
    const uint32_t* deg;
    unsigned long long* key;
    uint32_t* vis;
    uint32_t* Fc;       // frontier of this round (bitmap)
    uint32_t* Fn;       // vertices claimed this round (bitmap)
    const uint32_t* byst;
    uint32_t* Qc;
    uint32_t* Pc;
    uint32_t* Qn;
    uint32_t* Pn;
    unsigned long long* qcnt_c;
    unsigned long long* qcnt_n;
    unsigned long long* qover_c;
    unsigned long long* qover_n;
    unsigned long long* tot;
    uint32_t b0, b1;    // this round's start bucket in byst
    uint32_t nwords;
    uint32_t n;
    uint64_t dense_at;  // frontier size (vertices + edges) above which the round pulls
    uint32_t light;     // pull: neighbours one lane scans before its wavefront helps
};

// Round r, part 1: the vertices claimed in round r-1 (bitmap Fc) become
// visited; the still unvisited vertices whose start round is r become
// centres and join the frontier (queue Qc and bitmap Fc); Fn is cleared.
// A centre without edges is a cluster of its own and claims nothing, so it
// stays out of the queue (the late rounds inject every isolated vertex).
// Queue entries go through the workgroup's LDS buffer: one reservation per
// workgroup rather than one per wavefront.
__device__ __forceinline__ void ldd_inject_body(const LddArgs& a, WgQueue& q) {
    wgq_init(q);
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (tid == 0) {
        *a.qcnt_n = 0ull;
        *a.qover_n = 0ull;
    }
    for (uint32_t w = tid; w < a.nwords; w += stride) {
        const uint32_t f = a.Fc[w];
        if (f) atomicOr(&a.vis[w], f);  // atomic: centres below set bits of the same words
        a.Fn[w] = 0u;
    }
    __syncthreads();
    QueueOut out;
    out.Q = a.Qc;
    out.P = a.Pc;
    out.qcnt = a.qcnt_c;
    out.qover = a.qover_c;
    out.qlimit = ~0ull;
    out.tot = a.tot;
    const uint32_t span = a.b1 - a.b0;
    // workgroup-uniform trip count: the LDS queue is flushed between steps
    for (uint32_t b = blockIdx.x * (uint32_t)kRBlock; b < span; b += stride) {
        const uint32_t i = b + threadIdx.x;
        bool take = false;
        uint32_t v = 0, dv = 0;
        if (i < span) {
            v = a.byst[a.b0 + i];
            if (a.key[v] == kUnclaimed) {
                a.key[v] = ((unsigned long long)v << 32) | v;
                atomicOr(&a.vis[v >> 5], 1u << (v & 31));
                dv = a.deg[v];
                if (dv) {
                    take = true;
                    atomicOr(&a.Fc[v >> 5], 1u << (v & 31));
                }
            }
        }
        wgq_push(q, take, v, dv, out);
        wgq_maybe_flush(q, out, true, (uint32_t)kRBlock);
    }
    wgq_finish(q, out, true);
}

__global__ __launch_bounds__(kRBlock, 8) void ldd_inject_kernel(LddArgs a) {
    __shared__ WgQueue q;
    ldd_inject_body(a, q);
}

// Round r, part 2, sparse: the frontier queue claims its unvisited
// neighbours with a 64-bit atomic minimum of (claimer id, cluster); the
// smallest claimer id wins.  Visited bits are not touched during the round,
// so every claimer of a vertex competes.
struct LddPushPolicy {
    const LddArgs* a;
    WgQueue* q;
    const QueueOut* out;
    static constexpr bool kSkipDead = false;

    __device__ __forceinline__ uint32_t aux(uint32_t) const { return 1u; }

    __device__ __forceinline__ void edge(bool act, uint32_t u, uint32_t, int64_t e, bool) {
        bool take = false;
        uint32_t d = 0, dd = 0;
        if (act) {
            d = (uint32_t)a->nbr[e];
            if (!test_bit(a->vis, d)) {
                const unsigned long long cand =
                    ((unsigned long long)u << 32) | (a->key[u] & 0xFFFFFFFFull);
                if (cand < a->key[d]) {
                    const unsigned long long old = atomicMin(&a->key[d], cand);
                    if (old == kUnclaimed) {
                        take = true;
                        dd = a->deg[d];
                        atomicOr(&a->Fn[d >> 5], 1u << (d & 31));
                    }
                }
            }
        }
        wgq_push(*q, take, d, dd, *out);
    }

    __device__ __forceinline__ void window_done() {}
};

// Round r, part 2.  Sparse (small frontier): edge-balanced push over the
// queue.  Dense (frontier above dense_at): every unvisited vertex scans its
// sorted list for the first neighbour in the frontier bitmap -- the
// smallest claimer id, so the same result without atomics; a lane scans
// `light` neighbours, then its wavefront scans the rest 64 at a time.  Both
// emit the claimed vertices as the next queue and bitmap.
__device__ __forceinline__ void ldd_round_body(const LddArgs& a, uint32_t chunk_cap,
                                               WgQueue& q) {
    wgq_init(q);
    __syncthreads();
    const unsigned long long packed = *(volatile unsigned long long*)a.qcnt_c;
    const uint32_t count = (uint32_t)(packed >> 32);
    const uint32_t edges = (uint32_t)packed;
    QueueOut out;
    out.Q = a.Qn;
    out.P = a.Pn;
    out.qcnt = a.qcnt_n;
    out.qover = a.qover_n;
    out.qlimit = ~0ull;
    out.tot = a.tot;
    const uint32_t gwave = blockIdx.x * kRWaves + threadIdx.x / kWave;
    const uint32_t nwaves = gridDim.x * kRWaves;
    const int l = lane_id();
    if ((uint64_t)count + edges > a.dense_at) {
        // workgroup-uniform trip count: the LDS queue is flushed between steps
        for (uint32_t base = blockIdx.x * (uint32_t)kRBlock; base < a.n;
             base += gridDim.x * (uint32_t)kRBlock) {
            const uint32_t v = base + threadIdx.x;
            const bool valid = v < a.n;
            bool unvis = valid && !test_bit(a.vis, v);
            bool take = false;
            uint32_t u = 0;
            int64_t pos = 0, end = 0;
            if (unvis) {
                pos = a.off[v];
                end = a.off[v + 1];
                const int64_t lim = min(end, pos + (int64_t)a.light);
                for (; pos < lim; ++pos) {
                    const uint32_t x = (uint32_t)a.nbr[pos];
                    if (test_bit(a.Fc, x)) {
                        u = x;
                        take = true;
                        break;
                    }
                }
            }
            uint64_t heavy = ballot(unvis && !take && pos < end);
            while (heavy) {
                const int h = first_lane(heavy);
                heavy &= heavy - 1ull;
                const int64_t hs = (int64_t)shfl64((uint64_t)pos, h);
                const int64_t he = (int64_t)shfl64((uint64_t)end, h);
                uint32_t found = kNone;
                for (int64_t x0 = hs; x0 < he; x0 += kWave) {
                    const int64_t x = x0 + l;
                    uint32_t y = 0;
                    bool hit = false;
                    if (x < he) {
                        y = (uint32_t)a.nbr[x];
                        hit = test_bit(a.Fc, y);
                    }
                    const uint64_t hm = ballot(hit);
                    if (hm) {
                        found = __shfl(y, first_lane(hm), 64);
                        break;
                    }
                }
                if (l == h && found != kNone) {
                    u = found;
                    take = true;
                }
            }
            uint32_t dv = 0;
            if (take) {
                a.key[v] = ((unsigned long long)u << 32) | (a.key[u] & 0xFFFFFFFFull);
                dv = a.deg[v];
            }
            const uint64_t tm = ballot(take);
            if (l == 0 && (uint32_t)tm) a.Fn[v >> 5] = (uint32_t)tm;
            if (l == 32 && (uint32_t)(tm >> 32)) a.Fn[v >> 5] = (uint32_t)(tm >> 32);
            wgq_push(q, take, v, dv, out);
            wgq_maybe_flush(q, out, true, (uint32_t)kRBlock);
        }
    } else if (count && edges) {
        LddPushPolicy pol{&a, &q, &out};
        const uint32_t wc = wave_chunk(edges, nwaves, chunk_cap);
        const uint32_t nchunks = (edges + wc - 1) / wc;
        for (uint32_t c = gwave; c < nchunks; c += nwaves) {
            const uint32_t eb = c * wc;
            expand_range(a.Qc, a.Pc, count, edges, a.off, eb, min(edges, eb + wc), pol);
        }
    }
    wgq_finish(q, out, true);
}

__global__ __launch_bounds__(kRBlock, 8) void ldd_round_kernel(LddArgs a, uint32_t chunk_cap) {
    __shared__ WgQueue q;
    ldd_round_body(a, chunk_cap, q);
}

// Per-round arguments from the workspace (the pointers alternate by round).
__device__ __forceinline__ void ldd_round_args(LddArgs& a, uint32_t r, uint32_t* const F[2],
                                                        uint32_t* const Q[2], uint32_t* const P[2],
                                                        unsigned long long* ctl) {
    a.Fc = F[r & 1];
    a.Fn = F[(r + 1) & 1];
    a.Qc = Q[r & 1];
    a.Pc = P[r & 1];
    a.Qn = Q[(r + 1) & 1];
    a.Pn = P[(r + 1) & 1];
    a.qcnt_c = ctl + (r & 1);
    a.qcnt_n = ctl + ((r + 1) & 1);
    a.qover_c = ctl + 2 + (r & 1);
    a.qover_n = ctl + 2 + ((r + 1) & 1);
    a.tot = ctl + 128;
    a.b0 = (uint32_t)ctl[8 + r];
    a.b1 = (uint32_t)ctl[8 + r + 1];
}

struct LddSmall {
    LddArgs a;  // the round-invariant fields
    uint32_t* F[2];
    uint32_t* Q[2];
    uint32_t* P[2];
    unsigned long long* ctl;
};

// The whole decomposition of a small graph in one workgroup: the same
// injection and round steps, separated by workgroup barriers instead of
// launches, with the number of rounds and the start buckets read on the
// device (no host round trip).  Every loop is bounded: max g + 1 <= 64
// rounds.
__global__ __launch_bounds__(kRBlock, 1) void ldd_small_kernel(LddSmall S, uint32_t chunk_cap) {
    __shared__ WgQueue q;
    const uint32_t gmax = (uint32_t)S.ctl[4];
    for (uint32_t r = 0; r <= gmax; ++r) {
        LddArgs a = S.a;
        ldd_round_args(a, r, S.F, S.Q, S.P, S.ctl);
        ldd_inject_body(a, q);
        __syncthreads();
        if (r < gmax) ldd_round_body(a, chunk_cap, q);
        __syncthreads();
    }
}

// Number of v with x[v] == v (cluster centres; canonical component
// labels): one atomic per workgroup.
__global__ __launch_bounds__(kBlock) void count_self_kernel(const int32_t* x, int64_t n,
                                                            unsigned long long* count) {
    __shared__ uint32_t part[kBlock / kWave];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t c = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        c += x[v] == (int32_t)v ? 1u : 0u;
    c = wave_sum(c);
    if (lane_id() == 0) part[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < kBlock / kWave; ++i) t += part[i];
        if (t) atomicAdd(count, (unsigned long long)t);
    }
}

static int count_self(const int32_t* x, int64_t n, unsigned long long* dev_slot, hipStream_t s,
                      int64_t* out) {
    GB_HIP(hipMemsetAsync(dev_slot, 0, 8, s));
    hipLaunchKernelGGL(count_self_kernel, dim3(std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 1024))),
                       dim3(kBlock), 0, s, x, n, dev_slot);
    GB_HIP(hipGetLastError());
    unsigned long long h = 0;
    GB_HIP(hipMemcpyAsync(&h, dev_slot, 8, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    *out = (int64_t)h;
    return GBGPU_OK;
}

__global__ __launch_bounds__(kBlock) void ldd_label_kernel(const unsigned long long* key, int64_t n,
                                                           int32_t* label) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        label[v] = (int32_t)(key[v] & 0xFFFFFFFFull);
}

static int gridn(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((items + kBlock - 1) / kBlock, 4096));
}

// Graphs up to this size run the whole decomposition in one workgroup
// (ldd_small_kernel): at most 64 vertices of work per thread and round.
constexpr int64_t kSmallN = 1 << 16;
constexpr int64_t kSmallM = 1 << 20;

// One LDD of g into cluster[] (centre ids).  Returns the rounds run.
static int run_ldd(const GView& g, double beta, uint64_t seed, uint32_t level, int32_t* cluster,
                   const gbgpu_opts& o, hipStream_t s, LddWs* w, int32_t* rounds_out) {
    const int64_t n = g.n;
    const int64_t nwords = ((n + 63) / 64) * 2;
    GB_HIP(hipMemsetAsync(w->ctl, 0, 128 * 8, s));
    hipLaunchKernelGGL(ldd_shift_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, n, nwords, seed, level,
                       geo_threshold(beta), w->start, w->key, w->vis, w->F[0], w->F[1], w->ctl);
    hipLaunchKernelGGL(ldd_start_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, n, w->start, w->ctl);
    size_t tb = w->tmp_bytes;
    GB_HIP(rocprim::radix_sort_pairs(w->tmp, tb, w->start, w->keys_sorted,
                                     rocprim::counting_iterator<uint32_t>(0u), w->byst,
                                     (unsigned int)n, 0u, 6u, s));
    hipLaunchKernelGGL(ldd_bucket_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, w->keys_sorted, n,
                       w->ctl);
    GB_HIP(hipGetLastError());
    if (o.force_direction == 0 && n <= kSmallN && g.m <= kSmallM) {
        // small graph: every round in one workgroup, one launch
        LddSmall S;
        S.a.off = g.off;
        S.a.nbr = g.nbr;
        S.a.deg = g.deg;
        S.a.key = w->key;
        S.a.vis = w->vis;
        S.a.byst = w->byst;
        S.a.nwords = (uint32_t)nwords;
        S.a.n = (uint32_t)n;
        S.a.dense_at = (uint64_t)(g.m / std::max(1, o.tau));
        S.a.light = (uint32_t)o.pull_light;
        for (int i = 0; i < 2; ++i) {
            S.F[i] = w->F[i];
            S.Q[i] = w->Q[i];
            S.P[i] = w->P[i];
        }
        S.ctl = w->ctl;
        hipLaunchKernelGGL(ldd_small_kernel, dim3(1), dim3(kRBlock), 0, s, S,
                           (uint32_t)o.wave_chunk);
        hipLaunchKernelGGL(ldd_label_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, w->key, n,
                           cluster);
        GB_HIP(hipGetLastError());
        if (rounds_out) {
            unsigned long long gm = 0;
            GB_HIP(hipMemcpyAsync(&gm, w->ctl + 4, 8, hipMemcpyDeviceToHost, s));
            GB_HIP(hipStreamSynchronize(s));
            *rounds_out = (int32_t)gm + 1;
        }
        return GBGPU_OK;
    }
    unsigned long long hc[8 + 65];
    GB_HIP(hipMemcpyAsync(hc, w->ctl, sizeof(hc), hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    const uint32_t gmax = (uint32_t)hc[4];
    const int igrid = (int)std::max<int64_t>(1, std::min<int64_t>(n / (4 * kRBlock), o.grid));
    const int64_t work = std::max<int64_t>(1, std::max<int64_t>(n / kRBlock, g.m / 4096));
    const int egrid = (int)std::min<int64_t>(work, o.grid);
    // After round gmax's injection every vertex is in a cluster (a vertex
    // still unvisited at round start(v) becomes a centre then), so the rounds
    // are exactly 0..gmax and the last needs no expansion.
    for (uint32_t r = 0; r <= gmax; ++r) {
        LddArgs a;
        a.off = g.off;
        a.nbr = g.nbr;
        a.deg = g.deg;
        a.key = w->key;
        a.vis = w->vis;
        a.Fc = w->F[r & 1];
        a.Fn = w->F[(r + 1) & 1];
        a.byst = w->byst;
        a.Qc = w->Q[r & 1];
        a.Pc = w->P[r & 1];
        a.Qn = w->Q[(r + 1) & 1];
        a.Pn = w->P[(r + 1) & 1];
        a.qcnt_c = w->ctl + (r & 1);
        a.qcnt_n = w->ctl + ((r + 1) & 1);
        a.qover_c = w->ctl + 2 + (r & 1);
        a.qover_n = w->ctl + 2 + ((r + 1) & 1);
        a.tot = w->ctl + 128;
        a.b0 = (uint32_t)hc[8 + r];
        a.b1 = (uint32_t)hc[8 + r + 1];
        a.nwords = (uint32_t)nwords;
        a.n = (uint32_t)n;
        a.dense_at = o.force_direction == 1   ? ~0ull
                     : o.force_direction == 2 ? 0ull
                                              : (uint64_t)(g.m / std::max(1, o.tau));
        a.light = (uint32_t)o.pull_light;
        hipLaunchKernelGGL(ldd_inject_kernel, dim3(igrid), dim3(kRBlock), 0, s, a);
        if (r < gmax)
            hipLaunchKernelGGL(ldd_round_kernel, dim3(egrid), dim3(kRBlock), 0, s, a,
                               (uint32_t)o.wave_chunk);
        GB_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(ldd_label_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, w->key, n, cluster);
    GB_HIP(hipGetLastError());
    if (rounds_out) *rounds_out = (int32_t)gmax + 1;
    return GBGPU_OK;
}

// ---------------------------------------------------------------------------
// contraction
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void cc_iota_kernel(int64_t n, const int64_t* off,
                                                         uint32_t* iota, uint32_t* off32) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
        if (v < n) iota[v] = (uint32_t)v;
        off32[v] = (uint32_t)off[v];
    }
}

// Inter-cluster edges as keys (centre(u) << bits | centre(v)), compacted
// in any order (they are sorted next): a wavefront appends its keys to the
// workgroup's LDS buffer, and the workgroup copies the buffer out with one
// reservation when it is half full.  Most inter-cluster edges repeat a key
// (a few large clusters share many edges), so each workgroup first drops the
// keys it has already emitted, found in an LDS hash set (linear probing; a
// key whose probes all fail is emitted anyway -- the sort and unique that
// follow remove what duplicates remain).
constexpr int kKeyCap = 4096;
constexpr uint32_t kCrossChunk = 128;  // edges per wavefront step: a step adds <= kKeyCap / 2
constexpr int kHashSlots = 4096;
constexpr int kHashProbes = 8;

struct KeyBuf {
    unsigned long long k[kKeyCap];
    unsigned long long set[kHashSlots];
    uint32_t cnt;
    unsigned long long base;
};

__device__ __forceinline__ unsigned long long shfl_up64(unsigned long long x, int d) {
    const uint32_t lo = __shfl_up((uint32_t)x, d, 64);
    const uint32_t hi = __shfl_up((uint32_t)(x >> 32), d, 64);
    return ((unsigned long long)hi << 32) | lo;
}

// true when `key` was not in the set (and is now, if a slot was free)
__device__ __forceinline__ bool key_first_seen(KeyBuf* b, unsigned long long key) {
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 52);
#pragma unroll 1
    for (int p = 0; p < kHashProbes; ++p) {
        const uint32_t slot = (h + (uint32_t)p) & (kHashSlots - 1);
        const unsigned long long cur = b->set[slot];
        if (cur == key) return false;
        if (cur == kUnclaimed) {
            const unsigned long long old = atomicCAS(&b->set[slot], kUnclaimed, key);
            if (old == kUnclaimed) return true;
            if (old == key) return false;
        }
    }
    return true;
}

struct CrossPolicy {
    const int32_t* nbr;
    const int32_t* cluster;
    KeyBuf* buf;
    uint32_t bits;
    static constexpr bool kSkipDead = false;
    __device__ __forceinline__ uint32_t aux(uint32_t) const { return 1u; }
    __device__ __forceinline__ void edge(bool act, uint32_t u, uint32_t, int64_t e, bool) {
        bool cross = false;
        unsigned long long key = kUnclaimed;
        if (act) {
            const uint32_t a = (uint32_t)cluster[u], b = (uint32_t)cluster[nbr[e]];
            cross = a != b;
            if (cross) key = ((unsigned long long)a << bits) | b;
        }
        // the previous lane's equal key stands for this one (edges of one
        // vertex are adjacent)
        const unsigned long long prev = shfl_up64(key, 1);
        const bool take = cross && (lane_id() == 0 || prev != key) && key_first_seen(buf, key);
        const uint64_t m = ballot(take);
        if (!m) return;
        const int ld = first_lane(m);
        uint32_t pos = 0;
        if (lane_id() == ld) pos = atomicAdd(&buf->cnt, (uint32_t)__popcll(m));
        pos = __shfl(pos, ld, 64);
        if (take) buf->k[pos + mbcnt(m)] = key;
    }
    __device__ __forceinline__ void window_done() {}
};

// Workgroup-uniform: copies the buffered keys to out[] at a reserved range
// (keys past `cap` are counted, not written: the caller then retries with a
// larger buffer).
__device__ __forceinline__ void keybuf_flush(KeyBuf& b, unsigned long long* count,
                                             unsigned long long* out, uint64_t cap) {
    __syncthreads();
    const uint32_t n = b.cnt;
    if (threadIdx.x == 0 && n) b.base = atomicAdd(count, (unsigned long long)n);
    __syncthreads();
    const unsigned long long base = b.base;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        if (base + i < cap) out[base + i] = b.k[i];
    __syncthreads();
    if (threadIdx.x == 0) b.cnt = 0;
    __syncthreads();
}

__global__ __launch_bounds__(kRBlock, 8) void cc_cross_kernel(const uint32_t* iota,
                                                              const uint32_t* off32,
                                                              const int64_t* off, uint32_t n,
                                                              uint32_t m, const int32_t* nbr,
                                                              const int32_t* cluster,
                                                              uint32_t bits,
                                                              unsigned long long* count,
                                                              unsigned long long* out,
                                                              uint64_t cap) {
    __shared__ KeyBuf buf;
    if (threadIdx.x == 0) buf.cnt = 0;
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) buf.set[i] = kUnclaimed;
    __syncthreads();
    CrossPolicy pol{nbr, cluster, &buf, bits};
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t nchunks = (m + kCrossChunk - 1) / kCrossChunk;
    // workgroup-uniform trip count: one chunk per wavefront per step
    for (uint32_t c0 = blockIdx.x * kRWaves; c0 < nchunks; c0 += gridDim.x * kRWaves) {
        const uint32_t c = c0 + wave;
        if (c < nchunks) {
            const uint32_t eb = c * kCrossChunk;
            expand_range(iota, off32, n, m, off, eb, min(m, eb + kCrossChunk), pol);
        }
        __syncthreads();
        const uint32_t nb = buf.cnt;
        __syncthreads();  // every thread has read nb before anyone can append again
        if (nb > (uint32_t)kKeyCap / 2) keybuf_flush(buf, count, out, cap);
    }
    keybuf_flush(buf, count, out, cap);
}

// The contracted graph keeps only the clusters with an edge to another
// cluster (the others are whole components).  Over the sorted distinct
// keys: flag[i] = 1 where a new source centre starts (flag[mm] = 0).
__global__ __launch_bounds__(kBlock) void cc_first_kernel(const unsigned long long* keys,
                                                          uint32_t mm, uint32_t bits,
                                                          uint32_t* flag) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= mm; i += stride)
        flag[i] = i < mm && (i == 0 || (keys[i] >> bits) != (keys[i - 1] >> bits)) ? 1u : 0u;
}

// At each source's first key: contracted id s = pos[i], rep[s] = the
// centre, map[centre] = s, off2[s] = i; off2[k2] = mm.
__global__ __launch_bounds__(kBlock) void cc_index_kernel(const unsigned long long* keys,
                                                          uint32_t mm, uint32_t bits,
                                                          const uint32_t* flag,
                                                          const uint32_t* pos, uint32_t* rep,
                                                          uint32_t* map, int64_t* off2) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < mm; i += stride) {
        if (flag[i]) {
            const uint32_t s = pos[i];
            const uint32_t c = (uint32_t)(keys[i] >> bits);
            rep[s] = c;
            map[c] = s;
            off2[s] = i;
        }
        if (i == 0) off2[pos[mm]] = mm;
    }
}

// Neighbour ids of the contracted graph.  On a symmetric input every target
// centre is also a source; should the caller's symmetry claim be false, a
// missing target becomes a self-loop (harmless to the rounds) rather than an
// id out of range.
__global__ __launch_bounds__(kBlock) void cc_nbr_kernel(const unsigned long long* keys,
                                                        uint32_t mm, uint32_t bits,
                                                        const uint32_t* flag, const uint32_t* pos,
                                                        const uint32_t* map, int32_t* nbr2) {
    const uint32_t stride = gridDim.x * blockDim.x;
    const unsigned long long lo = (1ull << bits) - 1ull;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < mm; i += stride) {
        const uint32_t t = map[(uint32_t)(keys[i] & lo)];
        nbr2[i] = (int32_t)(t != kNone ? t : pos[i] + flag[i] - 1u);
    }
}

// label[v]: the centre of v's cluster when the cluster is a whole
// component, else the centre standing for the contracted vertex's label.
__global__ __launch_bounds__(kBlock) void cc_compose_kernel(const int32_t* cluster, int64_t n,
                                                            const uint32_t* map,
                                                            const uint32_t* rep,
                                                            const int32_t* sub, int32_t* label) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int32_t c = cluster[v];
        const uint32_t s = map[c];
        label[v] = s == kNone ? c : (int32_t)rep[sub[s]];
    }
}

// Smallest vertex of every label.  Most vertices of a wavefront usually
// share one label (the giant component), so the wavefront's smallest vertex
// stands for them, and the atomic is skipped when the stored value is
// already smaller: a handful of atomics per label instead of one per vertex.
__global__ __launch_bounds__(kBlock) void cc_canon_min_kernel(const int32_t* label, int64_t n,
                                                              uint32_t* minv) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // wave-uniform trip count (the loop bound is rounded to whole wavefronts)
    const int64_t nr = (n + kWave - 1) & ~(int64_t)(kWave - 1);
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nr; v += stride) {
        const bool ok = v < n;
        const int32_t lab = ok ? label[v] : -1;
        // lane 0 holds the wavefront's smallest vertex; it speaks for every
        // lane with the same label
        const int32_t lab0 = __shfl(lab, 0, 64);
        const bool speak = ok && (lab != lab0 || lane_id() == 0);
        if (speak && minv[lab] > (uint32_t)v) atomicMin(&minv[lab], (uint32_t)v);
    }
}

__global__ __launch_bounds__(kBlock) void cc_canon_apply_kernel(int32_t* label, int64_t n,
                                                                const uint32_t* minv) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        label[v] = (int32_t)minv[label[v]];
}

__global__ __launch_bounds__(kBlock) void cc_fill_kernel(uint32_t* x, int64_t n, uint32_t val) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = val;
}

__global__ __launch_bounds__(kBlock) void cc_deg_kernel(const int64_t* off, int64_t n,
                                                        uint32_t* deg) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        deg[v] = (uint32_t)(off[v + 1] - off[v]);
}

// label[v] for the vertices of g: a vertex of v's component, so equal
// exactly when connected.  levels_out accumulates the recursion depth.
// Everything this level takes from the arena is released on return.
static int connect_rec(const GView& g, double beta, uint64_t seed, uint32_t level,
                       int32_t* label, const gbgpu_opts& o, hipStream_t s, Arena& A,
                       int32_t* levels_out) {
    const int64_t n = g.n;
    *levels_out = (int32_t)level + 1;
    // A level leaves the graph as it is only when every edge joins two
    // vertices of equal shift; fresh shifts per level make a long run of
    // such levels vanishingly unlikely, and this bound turns one into an
    // error instead of unbounded recursion.
    if (level >= 256) return set_error(GBGPU_E_HIP, "connectivity did not converge");
    const size_t mark = A.top;
    struct Release {
        Arena& A;
        size_t mark;
        ~Release() { A.top = mark; }
    } release{A, mark};
    int32_t* cluster = nullptr;
    GB_TRY(arena_alloc(A, (size_t)n, &cluster));
    {
        const size_t m2 = A.top;
        LddWs w;
        GB_TRY(new_ldd_ws(A, n, &w));
        GB_TRY(run_ldd(g, beta, seed, level, cluster, o, s, &w, nullptr));
        A.top = m2;  // later kernels on the stream reuse the memory after the LDD's
    }
    auto clusters_are_components = [&]() -> int {
        GB_HIP(hipMemcpyAsync(label, cluster, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
        GB_HIP(hipStreamSynchronize(s));
        return GBGPU_OK;
    };
    if (g.m == 0) return clusters_are_components();
    // the inter-cluster edges as keys, most duplicates already dropped
    uint32_t *iota = nullptr, *off32 = nullptr;
    GB_TRY(arena_alloc(A, (size_t)n, &iota));
    GB_TRY(arena_alloc(A, (size_t)n + 1, &off32));
    hipLaunchKernelGGL(cc_iota_kernel, dim3(gridn(n + 1)), dim3(kBlock), 0, s, n, g.off, iota, off32);
    uint32_t bits = 1;
    while (bits < 32 && (1ll << bits) < n) ++bits;
    unsigned long long* cnt = nullptr;
    GB_TRY(arena_alloc(A, 2, &cnt));
    const uint32_t m32 = (uint32_t)g.m;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(g.m / 4096, o.grid));
    uint64_t cap = (uint64_t)std::min<int64_t>(g.m, std::max<int64_t>(1 << 20, g.m / 64));
    unsigned long long* keys = nullptr;
    uint32_t cross = 0;
    for (;;) {
        const size_t mk = A.top;
        GB_TRY(arena_alloc(A, (size_t)cap, &keys));
        GB_HIP(hipMemsetAsync(cnt, 0, 16, s));
        hipLaunchKernelGGL(cc_cross_kernel, dim3(grid), dim3(kRBlock), 0, s, iota, off32, g.off,
                           (uint32_t)n, m32, g.nbr, cluster, bits, cnt, keys, cap);
        GB_HIP(hipGetLastError());
        unsigned long long hm = 0;
        GB_HIP(hipMemcpyAsync(&hm, cnt, 8, hipMemcpyDeviceToHost, s));
        GB_HIP(hipStreamSynchronize(s));
        if (hm <= cap) {
            cross = (uint32_t)hm;
            break;
        }
        A.top = mk;  // too small: once more with room for every key
        cap = hm;
    }
    if (cross == 0) return clusters_are_components();
    // sort and de-duplicate: the contracted edges
    unsigned long long* keys2 = nullptr;
    GB_TRY(arena_alloc(A, (size_t)cross, &keys2));
    size_t ts = 0, tu = 0, tscan = 0;
    GB_HIP(rocprim::radix_sort_keys(nullptr, ts, keys, keys2, cross, 0u, 2u * bits, s));
    GB_HIP(rocprim::unique(nullptr, tu, keys2, keys, cnt + 1, (size_t)cross,
                           rocprim::equal_to<unsigned long long>(), s));
    uint32_t *flag = nullptr, *pos = nullptr;
    GB_HIP(rocprim::exclusive_scan(nullptr, tscan, flag, pos, 0u, (size_t)cross + 1,
                                   rocprim::plus<uint32_t>(), s));
    const size_t tmax = std::max(std::max(ts, tu), tscan);
    char* tmp = nullptr;
    GB_TRY(arena_alloc(A, tmax, &tmp));
    size_t tsz = tmax;
    GB_HIP(rocprim::radix_sort_keys(tmp, tsz, keys, keys2, cross, 0u, 2u * bits, s));
    tsz = tmax;
    GB_HIP(rocprim::unique(tmp, tsz, keys2, keys, cnt + 1, (size_t)cross,
                           rocprim::equal_to<unsigned long long>(), s));
    unsigned long long hm = 0;
    GB_HIP(hipMemcpyAsync(&hm, cnt + 1, 8, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    const uint32_t mm = (uint32_t)hm;
    // contracted vertices: the centres with an inter-cluster edge, in order
    uint32_t *map = nullptr, *rep = nullptr, *deg2 = nullptr;
    int64_t* off2 = nullptr;
    int32_t *nbr2 = nullptr, *sublabel = nullptr;
    GB_TRY(arena_alloc(A, (size_t)mm + 1, &flag));
    GB_TRY(arena_alloc(A, (size_t)mm + 1, &pos));
    GB_TRY(arena_alloc(A, (size_t)n, &map));
    GB_TRY(arena_alloc(A, (size_t)mm, &rep));
    GB_TRY(arena_alloc(A, (size_t)mm + 1, &off2));
    GB_TRY(arena_alloc(A, (size_t)mm, &nbr2));
    hipLaunchKernelGGL(cc_fill_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, map, n, kNone);
    hipLaunchKernelGGL(cc_first_kernel, dim3(gridn((int64_t)mm + 1)), dim3(kBlock), 0, s, keys, mm,
                       bits, flag);
    tsz = tmax;
    GB_HIP(rocprim::exclusive_scan(tmp, tsz, flag, pos, 0u, (size_t)mm + 1,
                                   rocprim::plus<uint32_t>(), s));
    hipLaunchKernelGGL(cc_index_kernel, dim3(gridn(mm)), dim3(kBlock), 0, s, keys, mm, bits, flag,
                       pos, rep, map, off2);
    hipLaunchKernelGGL(cc_nbr_kernel, dim3(gridn(mm)), dim3(kBlock), 0, s, keys, mm, bits, flag,
                       pos, (const uint32_t*)map, nbr2);
    GB_HIP(hipGetLastError());
    uint32_t k2 = 0;
    GB_HIP(hipMemcpyAsync(&k2, pos + mm, 4, hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    GB_TRY(arena_alloc(A, (size_t)k2, &deg2));
    GB_TRY(arena_alloc(A, (size_t)k2, &sublabel));
    hipLaunchKernelGGL(cc_deg_kernel, dim3(gridn(k2)), dim3(kBlock), 0, s, off2, (int64_t)k2, deg2);
    GB_HIP(hipGetLastError());
    const GView sub{(int64_t)k2, (int64_t)mm, off2, nbr2, deg2};
    GB_TRY(connect_rec(sub, beta, seed, level + 1, sublabel, o, s, A, levels_out));
    hipLaunchKernelGGL(cc_compose_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, cluster, n,
                       (const uint32_t*)map, (const uint32_t*)rep, sublabel, label);
    GB_HIP(hipGetLastError());
    GB_HIP(hipStreamSynchronize(s));
    return GBGPU_OK;
}

}  // namespace gb

using namespace gb;

extern "C" {

int gbgpu_ldd(gbgpu_graph g, double beta, uint64_t seed, int32_t* cluster, const gbgpu_opts* o,
              gbgpu_stats* st, void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!cluster) return set_error(GBGPU_E_INVALID, "output is NULL");
    if (!(beta > 0.0 && beta < 1.0)) return set_error(GBGPU_E_INVALID, "beta must lie in (0, 1)");
    const double t0 = now_ms();
    const gbgpu_opts opt = resolve_opts(o);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g->mu);
    Arena* A = nullptr;
    GB_TRY(arena_begin(g, ldd_ws_bytes(g->n), &A));
    // on every return: the stream drained (an early error may leave kernels
    // queued that use the arena), then the overflow allocations freed
    struct End {
        Arena* A;
        hipStream_t s;
        ~End() {
            (void)hipStreamSynchronize(s);
            arena_end(A);
        }
    } end{A, s};
    LddWs w;
    GB_TRY(new_ldd_ws(*A, g->n, &w));
    const GView v{g->n, g->m, g->off, g->nbr, g->deg};
    int32_t rounds = 0;
    GB_TRY(run_ldd(v, beta, seed, 0, cluster, opt, s, &w, &rounds));
    int64_t k = 0;
    if (st) GB_TRY(count_self(cluster, g->n, w.ctl + 6, s, &k));
    GB_HIP(hipStreamSynchronize(s));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->rounds = rounds;
        st->reached = k;
        st->wall_ms = now_ms() - t0;
    }
    return GBGPU_OK;
}

int gbgpu_connectivity(gbgpu_graph g, double beta, uint64_t seed, int32_t* label,
                       const gbgpu_opts* o, gbgpu_stats* st, void* stream) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!label) return set_error(GBGPU_E_INVALID, "output is NULL");
    if (!(beta > 0.0 && beta < 1.0)) return set_error(GBGPU_E_INVALID, "beta must lie in (0, 1)");
    const double t0 = now_ms();
    const gbgpu_opts opt = resolve_opts(o);
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g->mu);
    const int64_t n = g->n;
    Arena* A = nullptr;
    GB_TRY(arena_begin(g,
                       ldd_ws_bytes(n) + 4 * b256((size_t)n * 4 + 8) +
                           b256(8 * (size_t)std::min<int64_t>(g->m, std::max<int64_t>(1 << 20, g->m / 64))),
                       &A));
    struct End {
        Arena* A;
        hipStream_t s;
        ~End() {
            (void)hipStreamSynchronize(s);
            arena_end(A);
        }
    } end{A, s};
    const GView v{n, g->m, g->off, g->nbr, g->deg};
    int32_t levels = 0;
    GB_TRY(connect_rec(v, beta, seed, 0, label, opt, s, *A, &levels));
    // canonical labels: the smallest vertex id of each component
    uint32_t* minv = nullptr;
    unsigned long long* slot = nullptr;
    GB_TRY(arena_alloc(*A, (size_t)n, &minv));
    GB_TRY(arena_alloc(*A, 1, &slot));
    hipLaunchKernelGGL(cc_fill_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, minv, n, 0xFFFFFFFFu);
    hipLaunchKernelGGL(cc_canon_min_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, label, n, minv);
    hipLaunchKernelGGL(cc_canon_apply_kernel, dim3(gridn(n)), dim3(kBlock), 0, s, label, n, minv);
    GB_HIP(hipGetLastError());
    int64_t comps = 0;
    if (st) GB_TRY(count_self(label, n, slot, s, &comps));
    GB_HIP(hipStreamSynchronize(s));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->rounds = levels;
        st->reached = comps;
        st->wall_ms = now_ms() - t0;
    }
    return GBGPU_OK;
}

}  // extern "C"
