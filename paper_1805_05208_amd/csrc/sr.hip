// General-weight SSSP (Bellman-Ford) and widest path: frontier rounds of
// relaxations over a semiring.
//
// Method (paper: Bellman-Ford algorithm box; "Widest Path (Bottleneck
// Path)" in the Shortest Path Problems section, which runs the same rounds
// over the (max, min) semiring instead of (min, +)):
//   the frontier U_r holds the vertices whose value changed in round r-1
//   (U_0 = {src}).  Round r relaxes every edge (u, v) with u in U_r:
//   c = D[u] (x) w(u,v); when c is better than D[v], D[v] takes it with an
//   atomic minimum (maximum) -- the paper's priority-write -- and the first
//   vertex of the round to improve v puts v on U_{r+1} (test-and-set of its
//   bit in the next-frontier bitmap, the paper's Fl flags).  The rounds end
//   when one changes nothing.  Sparse rounds walk the frontier's edges in
//   edge-balanced blocks; dense rounds let every vertex scan its own list,
//   reduce the candidates of its neighbours in U_r (no early exit: the
//   paper's Cond is constant true) and keep the best.  The fixed point is
//   unique, so the result does not depend on the direction schedule or on
//   the order of updates inside a round.
//
// Semirings:
//   MinPlus  int64 D, unreached INT64_MAX, c = D[u] + w, better = smaller
//   MaxMin   uint32 W, unreached 0, W[src] = 0xFFFFFFFF, c = min(W[u], w),
//            better = larger
//
// Negative weights (Bellman-Ford only): the graph is symmetric, so a
// negative edge reachable from src closes the negative cycle (u, v, u) and
// every vertex of src's component is minus infinity.  A reachability pass
// (the BFS rounds) and one pass over the weights settle that case before any
// relaxation; otherwise the component has no negative weight and the
// rounds terminate.
//
// Workspace: a BfsWs of its own (three frontier bitmaps rotating like the
// BFS ones, two queues with degree prefixes, control block, pinned progress
// words); V holds the reachability bitmap of the negative-weight pass.

#include "common.h"
#include "emit.h"

namespace gb {

size_t bfs_ws_bytes(int64_t n, int64_t nwords);
void bfs_ws_attach(BfsWs* w, void* mem, int64_t n, int64_t nwords);
int bfs_ws_host_init(BfsWs* w);
int run_bfs(gbgpu_graph g, int32_t src, int32_t* dist, int32_t* parent, const gbgpu_opts& o,
            gbgpu_stats* st, hipStream_t stream);

static int ensure_sr_ws(gbgpu_graph g) {
    if (g->sr) return GBGPU_OK;
    BfsWs* w = new BfsWs();
    const size_t total = bfs_ws_bytes(g->n, g->nwords);
    hipError_t e = hipMalloc(&w->block, total);
    if (e != hipSuccess) {
        delete w;
        return set_error(GBGPU_E_NOMEM, "relaxation workspace of %zu bytes: %s", total,
                         hipGetErrorString(e));
    }
    bfs_ws_attach(w, w->block, g->n, g->nwords);
    int s = bfs_ws_host_init(w);
    if (s != GBGPU_OK) {
        free_bfs_ws(w);
        return s;
    }
    g->sr = w;
    return GBGPU_OK;
}

struct MinPlus {
    typedef long long T;
    static constexpr long long kUnset = INT64_MAX;
    __device__ static T extend(T du, int32_t w) { return du + (long long)w; }
    __device__ static bool better(T a, T b) { return a < b; }
    __device__ static T improve(T* p, T x) { return atomicMin(p, x); }
};

struct MaxMin {
    typedef uint32_t T;
    static constexpr uint32_t kUnset = 0u;
    __device__ static T extend(T du, int32_t w) { return min(du, (uint32_t)w); }
    __device__ static bool better(T a, T b) { return a > b; }
    __device__ static T improve(T* p, T x) { return atomicMax(p, x); }
};

__device__ __forceinline__ long long shfl_t(long long x, int s) {
    return (long long)shfl64((uint64_t)x, s);
}
__device__ __forceinline__ uint32_t shfl_t(uint32_t x, int s) { return __shfl(x, s, 64); }
__device__ __forceinline__ long long shfl_down_t(long long x, int d) {
    const uint32_t lo = __shfl_down((uint32_t)x, d, 64);
    const uint32_t hi = __shfl_down((uint32_t)((unsigned long long)x >> 32), d, 64);
    return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t shfl_down_t(uint32_t x, int d) { return __shfl_down(x, d, 64); }
__device__ __forceinline__ long long shfl_xor_t(long long x, int d) {
    const uint32_t lo = __shfl_xor((uint32_t)x, d, 64);
    const uint32_t hi = __shfl_xor((uint32_t)((unsigned long long)x >> 32), d, 64);
    return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ uint32_t shfl_xor_t(uint32_t x, int d) { return __shfl_xor(x, d, 64); }

template <typename T>
struct SrArgs {
    const int64_t* off;
    const int32_t* nbr;
    const int32_t* w;
    const uint32_t* deg;
    T* D;
    uint32_t* F0;
    uint32_t* F1;
    uint32_t* F2;
    uint32_t* Q0;
    uint32_t* Q1;
    uint32_t* P0;
    uint32_t* P1;
    unsigned long long* ctl;  // qcnt at +4, qover at +8, totals at +64
    uint32_t* prog;           // host progress words (device address)
    uint32_t* log;            // host round log (device address)
    const uint4* plan;
    uint32_t nplan;
    uint32_t src;
    int64_t n;
    int64_t nwords;
    uint64_t dense_thresh;    // dense when |U| + sum deg(U) exceeds it
    int32_t force_dir;
    uint32_t chunk_cap;
    T src_val;
};

// D = unreached except D[src]; U_0 = {src} as queue and bitmap.
template <typename S>
__global__ __launch_bounds__(kBlock) void sr_init_kernel(SrArgs<typename S::T> a) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < a.n; v += stride) a.D[v] = v == a.src ? a.src_val : S::kUnset;
    for (int64_t w = tid; w < a.nwords; w += stride) {
        a.F0[w] = (w == (int64_t)(a.src >> 5)) ? (1u << (a.src & 31)) : 0u;
        a.F1[w] = 0u;
        a.F2[w] = 0u;
    }
    if (tid == 0) {
        a.Q0[0] = a.src;
        a.P0[0] = 0;
        unsigned long long* qcnt = a.ctl + 4;
        unsigned long long* qover = a.ctl + 8;
        qcnt[0] = (1ull << 32) | a.deg[a.src];
        for (int i = 1; i < 4; ++i) qcnt[i] = 0;
        for (int i = 0; i < 4; ++i) qover[i] = 0;
    }
    unsigned long long* tot = a.ctl + 64;
    for (int64_t i = tid; i < 4 * kSpread; i += stride)
        tot[i * kSpreadStride] = i == 0 ? ((1ull << 32) | a.deg[a.src]) : 0ull;
}

// Sparse-round edge operation: relax (u, v) and enqueue v if this lane is
// the round's first to improve it.
template <typename S>
struct SrPushPolicy {
    typedef typename S::T T;
    const SrArgs<T>* a;
    uint32_t* Fn;
    WgQueue* q;
    const QueueOut* out;
    static constexpr bool kSkipDead = false;

    __device__ __forceinline__ uint32_t aux(uint32_t) const { return 1u; }

    __device__ __forceinline__ void edge(bool act, uint32_t u, uint32_t, int64_t e, bool) {
        bool take = false;
        uint32_t v = 0, dv = 0;
        if (act) {
            v = (uint32_t)a->nbr[e];
            const T c = S::extend(a->D[u], a->w[e]);
            if (S::better(c, a->D[v])) {
                const T old = S::improve(&a->D[v], c);
                if (S::better(c, old)) {
                    const uint32_t bit = 1u << (v & 31);
                    if (!(atomicOr(&Fn[v >> 5], bit) & bit)) {
                        take = true;
                        dv = a->deg[v];
                    }
                }
            }
        }
        wgq_push(*q, take, v, dv, *out);
    }

    __device__ __forceinline__ void window_done() {}
};

// Dense relaxation of one plan item (wave-uniform).  A run of <= 64
// consecutive vertices has its lists back to back: the wavefront walks them
// 64 edges at a time, each lane testing one edge's source against U_r, and a
// segmented reduction over the lanes of each vertex hands the window's best
// candidate to that vertex's lane.  A run's vertices are written by their
// own lane only.  A piece of one long list is scanned by the whole
// wavefront and its best candidate applied with the atomic (other pieces
// of the same list may run at the same time).
template <typename S>
__device__ __forceinline__ void sr_pull_item(const SrArgs<typename S::T>& a, uint4 it,
                                             const uint32_t* __restrict__ Fc, uint32_t* Fn,
                                             WgQueue& q, const QueueOut& out) {
    typedef typename S::T T;
    const int l = lane_id();
    if (it.z == kPlanHub) {
        const uint32_t vb = it.x, nv = it.y - it.x;
        const bool in = (uint32_t)l < nv;
        const uint32_t v = vb + (uint32_t)l;
        const int64_t base = a.off[vb];
        const uint32_t total = (uint32_t)(a.off[it.y] - base);
        uint32_t s = 0xFFFFFFFFu, d = 0;
        if (in) {
            const int64_t o0 = a.off[v];
            s = (uint32_t)(o0 - base);
            d = (uint32_t)(a.off[v + 1] - o0);
        }
        T acc = S::kUnset;
        for (uint32_t e = 0; e < total; e += 64) {
            const uint32_t t = e + (uint32_t)l;
            // owner lane of edge t: the largest lane whose list starts at or
            // before t (lanes past the run hold s = 0xFFFFFFFF)
            int o = 0;
#pragma unroll
            for (int st = 32; st >= 1; st >>= 1) {
                const uint32_t pv = __shfl(s, o + st, 64);
                if (pv <= t) o += st;
            }
            T c = S::kUnset;
            if (t < total) {
                const uint32_t u = (uint32_t)a.nbr[base + t];
                if (test_bit(Fc, u)) c = S::extend(a.D[u], a.w[base + t]);
            }
            // best over the lanes of each owner, gathered at its first lane
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const T oc = shfl_down_t(c, dd);
                const int oo = __shfl_down(o, dd, 64);
                if (l + dd < 64 && oo == o && S::better(oc, c)) c = oc;
            }
            const uint32_t first = (in && s > e) ? s - e : 0u;
            const T val = shfl_t(c, (int)min(first, 63u));
            if (in && d && s < e + 64u && s + d > e && S::better(val, acc)) acc = val;
        }
        bool take = false;
        if (in && S::better(acc, a.D[v])) {
            a.D[v] = acc;
            atomicOr(&Fn[v >> 5], 1u << (v & 31));
            take = true;
        }
        wgq_push(q, take, v, d, out);
    } else {
        const uint32_t v = it.x;
        T best = S::kUnset;
        for (uint32_t e = it.z; e < it.w; e += 64) {
            const uint32_t t = e + (uint32_t)l;
            if (t < it.w) {
                const uint32_t u = (uint32_t)a.nbr[t];
                if (test_bit(Fc, u)) {
                    const T c = S::extend(a.D[u], a.w[t]);
                    if (S::better(c, best)) best = c;
                }
            }
        }
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) {
            const T oc = shfl_xor_t(best, dd);
            if (S::better(oc, best)) best = oc;
        }
        bool take = false;
        uint32_t dv = 0;
        if (l == 0 && S::better(best, a.D[v])) {
            const T old = S::improve(&a.D[v], best);
            if (S::better(best, old)) {
                const uint32_t bit = 1u << (v & 31);
                take = !(atomicOr(&Fn[v >> 5], bit) & bit);
                if (take) dv = a.deg[v];
            }
        }
        wgq_push(q, take, v, dv, out);
    }
}

// One relaxation round.  Totals of U_r sit in slot r % 4 of the spread
// counters (written by round r-1); the first launch that finds U_r empty
// reports the end to the host, the launches queued behind it return.
template <typename S>
__global__ __launch_bounds__(kRBlock, 8) void sr_round_kernel(SrArgs<typename S::T> a, uint32_t r) {
    __shared__ WgQueue q;
    __shared__ unsigned long long s_tot, s_prev;
    unsigned long long* qcnt = a.ctl + 4;
    unsigned long long* qover = a.ctl + 8;
    unsigned long long* tot = a.ctl + 64;
    const uint32_t rs = r & 3u;
    if (threadIdx.x < kWave) {
        const unsigned long long t = spread_sum(tot + (size_t)rs * kSpread * kSpreadStride);
        if (threadIdx.x == 0) s_tot = t;
    } else if (threadIdx.x < 2 * kWave) {
        const unsigned long long t =
            spread_sum(tot + (size_t)((r + 3) & 3u) * kSpread * kSpreadStride);
        if (threadIdx.x == kWave) s_prev = t;
    }
    wgq_init(q);
    __syncthreads();
    const unsigned long long packed = s_tot;
    const uint32_t r2 = (r + 2) & 3u;
    if (blockIdx.x == 0 && threadIdx.x < kSpread) {
        // slots of round r+2 are unused during round r; cleared
        // unconditionally so launches past the end read an empty frontier
        tot[((size_t)r2 * kSpread + threadIdx.x) * kSpreadStride] = 0ull;
        if (threadIdx.x == 0) {
            qcnt[r2] = 0;
            qover[r2] = 0;
        }
    }
    const uint32_t count = (uint32_t)(packed >> 32);
    const uint32_t edges = (uint32_t)packed;
    if (count == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && (s_prev >> 32) != 0) {
            __threadfence_system();
            host_store(&a.prog[1], r + 1);
        }
        return;
    }
    const bool qvalid = qover[rs] == 0;
    bool push;
    if (a.force_dir == 1) push = true;
    else if (a.force_dir == 2) push = false;
    else push = (uint64_t)count + edges <= a.dense_thresh;
    if (!qvalid) push = false;  // the queue of U_r was abandoned: only the bitmap exists

    uint32_t* Fs[3] = {a.F0, a.F1, a.F2};
    const uint32_t* Fc = Fs[r % 3];
    uint32_t* Fn = Fs[(r + 1) % 3];
    uint32_t* Fclr = Fs[(r + 2) % 3];
    const uint32_t* Qc = (r & 1) ? a.Q1 : a.Q0;
    const uint32_t* Pc = (r & 1) ? a.P1 : a.P0;
    const uint32_t wib = threadIdx.x / kWave;
    const uint32_t gwave = blockIdx.x * kRWaves + wib;
    const uint32_t nwaves = gridDim.x * kRWaves;
    const uint32_t r1 = (r + 1) & 3u;
    QueueOut out;
    out.Q = (r & 1) ? a.Q0 : a.Q1;
    out.P = (r & 1) ? a.P0 : a.P1;
    out.qcnt = &qcnt[r1];
    out.qover = &qover[r1];
    out.qlimit = a.force_dir == 1 ? ~0ull : a.dense_thresh;
    out.tot = tot + (size_t)r1 * kSpread * kSpreadStride;

    if (blockIdx.x == 0 && threadIdx.x == 0) {
        host_store(&a.prog[0], r + 1);
        if (r < (uint32_t)kLogCap) {
            host_store(&a.log[4 * r + 0], push ? 1u : 2u);
            host_store(&a.log[4 * r + 1], count);
            host_store(&a.log[4 * r + 2], edges);
            host_store(&a.log[4 * r + 3], qvalid ? 1u : 0u);
        }
    }
    // clear the bitmap that round r+1 fills
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < a.nwords;
         w += (int64_t)gridDim.x * blockDim.x)
        Fclr[w] = 0u;
    if (push) {
        SrPushPolicy<S> pol{&a, Fn, &q, &out};
        const uint32_t wc = wave_chunk(edges, nwaves, a.chunk_cap);
        const uint32_t nchunks = (edges + wc - 1) / wc;
        for (uint32_t c = gwave; c < nchunks; c += nwaves) {
            const uint32_t eb = c * wc;
            expand_range(Qc, Pc, count, edges, a.off, eb, min(edges, eb + wc), pol);
        }
    } else {
        for (uint32_t i = gwave; i < a.nplan; i += nwaves)
            sr_pull_item<S>(a, a.plan[i], Fc, Fn, q, out);
    }
    wgq_finish(q, out, true);
}

// Negative-weight pass: the reachability bitmap R of src's component from
// the BFS distances, and whether any edge of that component is negative
// (on a symmetric graph an edge is in the component iff its head is).
__global__ __launch_bounds__(kBlock) void sr_reach_kernel(const int32_t* bd, int64_t n,
                                                          int64_t nwords, uint32_t* R,
                                                          unsigned long long* flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0ull;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        uint32_t bits = 0u;
        for (int i = 0; i < 32; ++i) {
            const int64_t v = w * 32 + i;
            if (v < n && bd[v] != INT32_MAX) bits |= 1u << i;
        }
        R[w] = bits;
    }
}

__global__ __launch_bounds__(kBlock) void sr_negative_edge_kernel(const int32_t* nbr,
                                                                  const int32_t* wt, int64_t m,
                                                                  const uint32_t* R,
                                                                  unsigned long long* flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool found = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
        if (wt[e] < 0 && test_bit(R, (uint32_t)nbr[e])) found = true;
    if (ballot(found) && lane_id() == 0) atomicOr(flag, 1ull);
}

__global__ __launch_bounds__(kBlock) void sr_fill_component_kernel(long long* D, int64_t n,
                                                                   const uint32_t* R) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        D[v] = test_bit(R, (uint32_t)v) ? INT64_MIN : INT64_MAX;
}

static int grid_of(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((items + kBlock - 1) / kBlock, 4096));
}

template <typename S>
static int run_sr(gbgpu_graph g, int32_t src, typename S::T* D, typename S::T src_val,
                  const gbgpu_opts& o, gbgpu_stats* st, hipStream_t stream, double t0) {
    typedef typename S::T T;
    BfsWs* w = g->sr;
    SrArgs<T> a;
    a.off = g->off;
    a.nbr = g->nbr;
    a.w = g->w;
    a.deg = g->deg;
    a.D = D;
    a.F0 = w->F[0];
    a.F1 = w->F[1];
    a.F2 = w->F[2];
    a.Q0 = w->Q[0];
    a.Q1 = w->Q[1];
    a.P0 = w->P[0];
    a.P1 = w->P[1];
    a.ctl = w->ctl;
    a.prog = w->hl.d;
    a.log = w->hl.d + kHostLogOff;
    a.plan = g->plan;
    a.nplan = g->nplan;
    a.src = (uint32_t)src;
    a.n = g->n;
    a.nwords = g->nwords;
    a.dense_thresh = (uint64_t)g->m / (uint64_t)o.tau;
    a.force_dir = o.force_direction == 1 || o.force_direction == 2 ? o.force_direction : 0;
    a.chunk_cap = (uint32_t)o.wave_chunk;
    a.src_val = src_val;

    hipLaunchKernelGGL(sr_init_kernel<S>, dim3(grid_of(g->n)), dim3(kBlock), 0, stream, a);
    GB_HIP(hipGetLastError());
    volatile uint32_t* hp = w->hl.h;
    hp[0] = 0;
    hp[1] = 0;
    if (o.profile) GB_HIP(hipEventRecord(w->ev0, stream));
    const int work = (int)std::max<int64_t>(1, std::max<int64_t>(g->nwords / 32, g->m / 4096));
    const int grid = std::min(work, o.grid);
    // without a reachable negative cycle a round changes at least one value,
    // and every value settles within n rounds
    const int64_t max_rounds = std::min<int64_t>(g->n + 2, 0x7FFFFFFF);
    int64_t launches = 0;
    GB_TRY(run_pipeline(
        hp, stream, o.rounds_per_sync, max_rounds,
        [&](int64_t r) {
            hipLaunchKernelGGL(sr_round_kernel<S>, dim3(grid), dim3(kRBlock), 0, stream, a,
                               (uint32_t)r);
        },
        &launches));
    if (o.profile) GB_HIP(hipEventRecord(w->ev1, stream));
    GB_HIP(hipEventRecord(w->done, stream));
    GB_HIP(hipStreamSynchronize(stream));
    const uint32_t rounds = hp[1] - 1;
    w->last_rounds = rounds;
    if (st) {
        memset(st, 0, sizeof(*st));
        if (o.profile) {
            float ms = 0.f;
            GB_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
            st->kernel_ms = ms;
        }
        const uint32_t* lg = w->hl.h + kHostLogOff;
        int64_t ex = 0;
        for (uint32_t i = 0; i < std::min<uint32_t>(rounds, (uint32_t)kLogCap); ++i) {
            if (lg[4 * i] == 2) st->pull_rounds++; else st->push_rounds++;
            ex += lg[4 * i + 2];
        }
        st->rounds = (int32_t)rounds;
        st->edges_examined = ex;
        st->launches = (int32_t)launches;
        st->wall_ms = now_ms() - t0;
    }
    return GBGPU_OK;
}

// Direction threshold: dense when |U| + sum deg(U) > m / tau.  The dense
// pull has no early exit here (every neighbour in U_r is a candidate), so it
// costs a scan of all m edges; the push costs the frontier's edges plus one
// atomic per improvement, and on graphs with hubs those atomics pile up on
// the same few addresses.  Unless the caller sets tau: 20 (as for BFS) when
// the largest degree is at least 64 times the average, else 4 (on the 256^3
// torus all-sparse rounds took half the time of tau = 20).
static gbgpu_opts sr_opts(gbgpu_graph g, const gbgpu_opts* o) {
    gbgpu_opts r = resolve_opts(o);
    if (!o || o->tau <= 0) {
        const double avg = g->n ? (double)g->m / (double)g->n : 0.0;
        r.tau = (double)g->max_degree >= 64.0 * std::max(avg, 1.0) ? 20 : 4;
    }
    return r;
}

static int check_sr_args(gbgpu_graph g, int32_t src, const void* out) {
    if (!g) return set_error(GBGPU_E_INVALID, "graph is NULL");
    if (!g->w) return set_error(GBGPU_E_INVALID, "graph was loaded without weights");
    if (!out) return set_error(GBGPU_E_INVALID, "output is NULL");
    if (src < 0 || src >= g->n)
        return set_error(GBGPU_E_INVALID, "src %d out of range [0, %lld)", src, (long long)g->n);
    return GBGPU_OK;
}

}  // namespace gb

using namespace gb;

extern "C" {

int gbgpu_bellman_ford(gbgpu_graph g, int32_t src, int64_t* dist, const gbgpu_opts* o,
                       gbgpu_stats* st, void* stream) {
    GB_TRY(check_sr_args(g, src, dist));
    const double t0 = now_ms();
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g->mu);
    GB_TRY(ensure_pull_plan(g));
    gbgpu_opts opt = sr_opts(g, o);
    GB_TRY(ensure_sr_ws(g));
    BfsWs* w = g->sr;
    GB_HIP(hipStreamWaitEvent(s, w->done, 0));
    if (g->minw < 0) {
        // reachability of src's component, computed into the output's
        // storage (8n bytes hold the BFS distances and parents), then the
        // negative-edge test
        int32_t* bd = reinterpret_cast<int32_t*>(dist);
        GB_TRY(run_bfs(g, src, bd, bd + g->n, opt, nullptr, s));
        unsigned long long* flag = w->ctl + 20;
        hipLaunchKernelGGL(sr_reach_kernel, dim3(grid_of(g->nwords)), dim3(kBlock), 0, s, bd,
                           g->n, g->nwords, w->V, flag);
        hipLaunchKernelGGL(sr_negative_edge_kernel, dim3(grid_of(g->m)), dim3(kBlock), 0, s,
                           g->nbr, g->w, g->m, w->V, flag);
        GB_HIP(hipGetLastError());
        unsigned long long hflag = 0;
        GB_HIP(hipMemcpyAsync(&hflag, flag, 8, hipMemcpyDeviceToHost, s));
        GB_HIP(hipStreamSynchronize(s));
        if (hflag) {
            hipLaunchKernelGGL(sr_fill_component_kernel, dim3(grid_of(g->n)), dim3(kBlock), 0, s,
                               (long long*)dist, g->n, w->V);
            GB_HIP(hipGetLastError());
            GB_HIP(hipEventRecord(w->done, s));
            GB_HIP(hipStreamSynchronize(s));
            if (st) {
                memset(st, 0, sizeof(*st));
                st->wall_ms = now_ms() - t0;
            }
            return GBGPU_OK;
        }
    }
    return run_sr<MinPlus>(g, src, (long long*)dist, 0ll, opt, st, s, t0);
}

int gbgpu_widest_path(gbgpu_graph g, int32_t src, uint32_t* width, const gbgpu_opts* o,
                      gbgpu_stats* st, void* stream) {
    GB_TRY(check_sr_args(g, src, width));
    if (g->minw < 1) return set_error(GBGPU_E_INVALID, "widest path needs weights >= 1");
    const double t0 = now_ms();
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g->mu);
    GB_TRY(ensure_pull_plan(g));
    gbgpu_opts opt = sr_opts(g, o);
    GB_TRY(ensure_sr_ws(g));
    GB_HIP(hipStreamWaitEvent(s, g->sr->done, 0));
    return run_sr<MaxMin>(g, src, width, 0xFFFFFFFFu, opt, st, s, t0);
}

}  // extern "C"
